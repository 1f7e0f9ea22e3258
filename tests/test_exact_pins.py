"""Pins of the oracle's exact cell-averaged kernel (mesh kernel rule 1, the
m -> infinity limit of the subpoint average of Eq. 10 over a cell).

Each check compares with something other than the function itself: the
circle-in-rectangle angle against a tiling identity and brute angular
sampling; the source's own cell against the independent pyramid-split cube
average; the flux identity (the cell averages of one shell, times l^3,
summed over every cell and image, equal the shell integral of phi, which
holds exactly for cell averages); an uncut cell against a tensor
Gauss-Legendre cubature of the cell; additivity over a split shell; the
convergence of the subpoint rule towards it; and the quadrature order.
"""
import math

import numpy as np
import pytest

import lc_inputs as li
import oracle

KINDS = {
    "flat": li.Atten(kind=0),
    "lw_continuous": li.lw_band(5.0),
    "lw_printed": li.Atten(kind=2, a=1.7, s=5.96, p=0.68, c=0.7, cut=4.98),
}


def test_theta_rect_tiling_and_brute_sampling():
    rng = np.random.default_rng(5)
    # the unit squares of [-6, 6]^2 tile the plane around every circle R < 6
    edges = np.arange(-6.0, 6.0 + 1e-12, 1.0)
    for R in (0.3, 1.0, 2.5, math.sqrt(2.0), 4.7):
        tot = sum(oracle.theta_rect(R, edges[i], edges[i + 1], edges[j], edges[j + 1])
                  for i in range(12) for j in range(12))
        assert abs(tot - 2 * math.pi) < 1e-13
    t = np.linspace(0.0, 2 * math.pi, 2_000_001)[:-1]
    for _ in range(6):
        x0, y0 = rng.uniform(-2, 1.5, 2)
        x1, y1 = x0 + rng.uniform(0.2, 2.0), y0 + rng.uniform(0.2, 2.0)
        R = rng.uniform(0.2, 2.5)
        X, Y = R * np.cos(t), R * np.sin(t)
        frac = np.mean((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1))
        assert abs(oracle.theta_rect(R, x0, x1, y0, y1) - 2 * math.pi * frac) < 2e-5


@pytest.mark.parametrize("name", list(KINDS))
def test_source_cell_equals_pyramid_cube_average(name):
    """Shell [0, r) with r beyond the cell's corners: the whole cube, whose
    average the oracle also forms by the pyramid split (or_self_cell)."""
    at = KINDS[name]
    for l in (1.0, 0.7):
        h = 0.5 * l
        v = oracle.cell_average(at, l, [-h, h, -h, h, -h, h], 0.0, 4.0 * l)
        ref = oracle.self_cell(at, l)
        assert abs(v / ref - 1.0) < 1e-13, (v, ref)


def _gl_cube(at, l, box, n=24):
    x, w = np.polynomial.legendre.leggauss(n)
    pts = [0.5 * (b - a) * x + 0.5 * (a + b) for a, b in zip(box[0::2], box[1::2])]
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    ph = np.vectorize(lambda v: oracle.phi(at, v))(r)
    W = np.einsum("i,j,k->ijk", w, w, w) * np.prod([0.5 * (b - a) for a, b in zip(box[0::2], box[1::2])])
    return at.prefactor * float(np.sum(W * ph / (4 * math.pi * r * r))) / l ** 3


@pytest.mark.parametrize("name", list(KINDS))
def test_uncut_cell_matches_cubature(name):
    at = KINDS[name]
    l = 1.0
    for c in [(2, 1, 0), (3, -1, 2), (0, 0, 3), (-2, 2, -1)]:
        box = [v for d in c for v in (d - 0.5, d + 0.5)]
        v = oracle.cell_average(at, l, box, 0.0, 4.9)   # every corner inside, below every cut
        ref = _gl_cube(at, l, box)
        assert abs(v / ref - 1.0) < 1e-12, (c, v, ref)


@pytest.mark.parametrize("name", list(KINDS))
def test_additivity_over_a_split_shell(name):
    at = KINDS[name]
    rng = np.random.default_rng(11)
    for _ in range(8):
        c = rng.integers(-3, 4, 3)
        box = [v for d in c for v in (d - 0.5, d + 0.5)]
        d = float(np.linalg.norm(c))
        r0, r2 = max(0.0, d - 1.0), d + 1.0
        r1 = rng.uniform(r0, r2)
        whole = oracle.cell_average(at, 1.0, box, r0, r2)
        parts = oracle.cell_average(at, 1.0, box, r0, r1) + oracle.cell_average(at, 1.0, box, r1, r2)
        assert abs(whole - parts) <= 1e-14 * max(1.0, abs(whole))


@pytest.mark.parametrize("name", list(KINDS))
def test_flux_identity_every_cell_and_image(name):
    """Cell averages partition the shell: l^3 sum_c G_k(c) over all cells
    (with their periodic images) equals pref * int_{r_k}^{r_k+1} phi dr,
    with shells cutting through cells and through the source's own cell."""
    at = KINDS[name]
    n, L = 8, 8.0
    radii = np.array([0.0, 0.6, 1.7, 3.2, 4.4])
    G = oracle.build_G_exact(n, L, radii, at)
    l3 = (L / n) ** 3
    for k in range(len(radii) - 1):
        flux = l3 * float(np.sum(G[k]))
        ref = oracle.shell_integral(at, radii[k], radii[k + 1]) * at.prefactor
        assert abs(flux - ref) <= 1e-12 * abs(ref), (k, flux, ref)


def test_subpoint_rule_converges_to_the_exact_average():
    at = KINDS["lw_continuous"]
    n, L = 16, 16.0
    radii = np.array([0.0, 1.0, 2.6, 4.0])
    for disp in [(2, 1, 0), (1, 1, 1), (3, 0, 2)]:
        ex = oracle.G_exact_at(n, L, radii, at, disp)
        errs = [np.abs(oracle.G_at(n, L, radii, m, at, disp) - ex).max() for m in (2, 4, 8)]
        assert errs[2] < errs[0] and errs[2] < 0.05 * np.abs(ex).max()


def test_quadrature_order_converged():
    rng = np.random.default_rng(3)
    for name, at in KINDS.items():
        for _ in range(5):
            c = rng.integers(-2, 3, 3)
            box = [v for d in c for v in (d - 0.5, d + 0.5)]
            r0, r1 = sorted(rng.uniform(0.0, 3.5, 2))
            a = oracle.cell_average(at, 1.0, box, r0, r1, ng=24)
            b = oracle.cell_average(at, 1.0, box, r0, r1, ng=48)
            assert abs(a - b) <= 1e-14 * max(1.0, abs(b)), (name, c, r0, r1, a, b)


@pytest.mark.parametrize("r_lo,r_hi", [(0.5 + 1e-3, 2.76), (0.5 + 1e-6, 2.6), (2.55, 2.5 + 1e-5 + 0.06),
                                       (0.3, 2.5 + 1e-7 + 0.2), (2.6, 3.0)])
def test_near_coincident_breakpoints_vs_mpmath(r_lo, r_hi):
    """Cells on the z axis, [-1/2, 1/2]^2 x [z0, z1] with z0 > 0, phi = 1, and
    shell radii just off the cell's edge distances: the integral in R of
    Theta(R) (2 pi, or 2 pi - 8 acos(1/(2R)) past the edge) times the z
    integral of R / (R^2 + z^2) (atan differences), to 30 digits by mpmath."""
    import mpmath as mp
    mp.mp.dps = 30
    z0, z1 = mp.mpf(2.5), mp.mpf(3.5)
    rl, rh = mp.mpf(r_lo), mp.mpf(r_hi)

    def theta(R):
        return 2 * mp.pi if R <= 0.5 else 2 * mp.pi - 8 * mp.acos(mp.mpf(0.5) / R)

    def V(R):
        lo = max(z0, mp.sqrt(rl ** 2 - R ** 2)) if rl > R else z0
        hi = min(z1, mp.sqrt(rh ** 2 - R ** 2)) if rh > R else mp.mpf(0)
        return mp.atan(hi / R) - mp.atan(lo / R) if hi > lo else mp.mpf(0)

    pts = {mp.mpf(0), mp.mpf(0.5), mp.sqrt(mp.mpf(0.5))}
    for r in (rl, rh):
        for z in (z0, z1):
            if r > z:
                pts.add(mp.sqrt(r * r - z * z))
    pts = sorted(p for p in pts if p <= mp.sqrt(mp.mpf(0.5)))
    ref = mp.quad(lambda R: theta(R) * V(R), pts) / (4 * mp.pi)
    v = oracle.cell_average(li.Atten(kind=0), 1.0, [-0.5, 0.5, -0.5, 0.5, 2.5, 3.5], r_lo, r_hi)
    assert abs(v - float(ref)) <= 1e-13 * max(abs(float(ref)), 1e-3), (v, float(ref))
