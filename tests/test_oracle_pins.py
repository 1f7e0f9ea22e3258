"""Pins of the CPU FP64 oracle against what the paper and mathematics fix.

Every check here compares the oracle with something other than itself:
closed forms (1/(4 pi r^2) shells, flux = shell width, the sine-integral
continuum limit, the cube-average self constant), invariants (cube
symmetries, linearity, translation, Parseval), library routines
(numpy.fft, mpmath quadrature and incomplete gamma) and O(N^6) brute force.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import lc_inputs as li
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")

KAPPA_TEXT = None  # computed below with mpmath


def kappa_mp():
    # J2 = int_0^1 int_0^1 dy dz / (1 + y^2 + z^2); kappa = 12 J2 / (4 pi)
    mp.mp.dps = 30
    J2 = mp.quad(lambda y, z: 1 / (1 + y * y + z * z), [0, 1], [0, 1])
    return float(12 * J2 / (4 * mp.pi))


# --- radial factor, integrals ----------------------------------------------------

def test_paper_fmod_constants_step_at_cut():
    """Eq. 15 as printed: at the cut r = 97.39 alpha the factor is still
    positive (about +6.45e-4), i.e. the printed form has a small step."""
    g = json.load(open(GOLDEN))["fmod"]
    alpha = 1.0
    at = li.Atten(kind=2, a=g["amplitude"], s=g["scale_over_alpha"] * alpha,
                  p=g["exponent"], c=g["offset"], cut=g["cut_over_alpha"] * alpha)
    r = g["cut_over_alpha"] * alpha
    expect = g["amplitude"] * math.exp(-(r / g["scale_over_alpha"]) ** g["exponent"]) - g["offset"]
    assert abs(oracle.phi(at, r) - expect) < 1e-15
    assert 6.4e-4 < expect < 6.5e-4
    assert oracle.phi(at, r * (1 + 1e-9)) == 0.0
    # continuous form has its zero at s * ln(a/c)^(1/p)
    at1 = li.Atten(kind=1, a=1.7, s=116.0, p=0.68, c=0.7)
    x0 = 116.0 * math.log(1.7 / 0.7) ** (1 / 0.68)
    assert abs(x0 - 97.2956) < 1e-3
    assert oracle.phi(at1, x0 * (1 + 1e-9)) == 0.0
    assert oracle.phi(at1, x0 * (1 - 1e-6)) > 0.0


@pytest.mark.parametrize("R", [0.3, 5.0, 50.0, 97.0, 150.0])
def test_Phi_matches_incomplete_gamma(R):
    """int_0^R (a e^{-(r/s)^p} - c) dr = a (s/p) gamma(1/p, (R/s)^p) - c R,
    truncated at the zero of the integrand."""
    a, s, p, c = 1.7, 116.0, 0.68, 0.7
    at = li.Atten(kind=1, a=a, s=s, p=p, c=c)
    mp.mp.dps = 30
    r0 = s * math.log(a / c) ** (1 / p)
    U = min(R, r0)
    ref = a * (s / p) * mp.gammainc(1 / p, 0, (mp.mpf(U) / s) ** p) - c * U
    assert abs(oracle.Phi(at, R) - float(ref)) <= 1e-14 * max(1.0, abs(float(ref)))


def test_self_cell_constant_kappa():
    k = kappa_mp()
    assert abs(k - 0.6106874019515839) < 1e-15
    for l in (1.0, 0.625, 0.78125):
        v = oracle.self_cell(li.Atten(kind=0), l)
        assert abs(v * l * l - k) <= 1e-14 * k


def test_self_cell_with_attenuation_vs_mpmath():
    """Cube average of phi/(4 pi r^2) by the pyramid decomposition with the
    closed-form Phi (incomplete gamma), integrated by mpmath."""
    a, s, p, c = 1.7, 47.6897, 0.68, 0.7
    at = li.Atten(kind=1, a=a, s=s, p=p, c=c)
    l = 0.78125
    mp.mp.dps = 25
    hl = mp.mpf(l) / 2

    def Phi(R):
        return a * (s / p) * mp.gammainc(1 / p, 0, (R / s) ** p) - c * R

    face = mp.quad(lambda y, z: hl * Phi(mp.sqrt(hl ** 2 + y ** 2 + z ** 2)) /
                   (mp.sqrt(hl ** 2 + y ** 2 + z ** 2) ** 3), [0, hl], [0, hl])
    ref = float(6 * 4 * face / (4 * mp.pi) / mp.mpf(l) ** 3)
    assert abs(oracle.self_cell(at, l) - ref) <= 1e-13 * ref


# --- kernel -------------------------------------------------------------------------

def _small_box(n=16, L=10.0, K=3, rmax=None, m=1, kind=0):
    rmax = rmax if rmax is not None else 0.45 * L
    radii = np.array([rmax * k / K for k in range(K + 1)])
    at = li.Atten(kind=kind, a=1.7, s=rmax / li.LW_X0 * 1.3, p=0.68, c=0.7)
    return n, L, radii, m, at


def test_node_rule_single_source_is_delayed_shell():
    """m = 1, shells inside L/2: a unit source in slice k gives
    1/(4 pi r^2) on exactly the nodes with r_k <= r < r_{k+1} (one image)."""
    n, L = 16, 16.0
    radii = np.array([0.0, 2.3, 4.7, 7.1])   # no node distance equals a radius
    at = li.Atten(kind=0)
    G = oracle.build_G(n, L, radii, 1, at)
    l = L / n
    idx = np.arange(n)
    e = np.minimum(idx, n - idx)
    d = np.sqrt(e[:, None, None] ** 2 + e[None, :, None] ** 2 + e[None, None, :] ** 2) * l
    for k in range(1, 3):
        inside = (d >= radii[k]) & (d < radii[k + 1])
        expect = np.where(inside, 1.0 / (4 * np.pi * np.where(d > 0, d, 1) ** 2), 0.0)
        np.testing.assert_allclose(G[k], expect, rtol=1e-15, atol=0)
    # shell 0 holds the self cell (kappa/l^2) plus the nodes in (0, r_1)
    inside0 = (d > 0) & (d < radii[1])
    expect0 = np.where(inside0, 1.0 / (4 * np.pi * np.where(d > 0, d, 1) ** 2), 0.0)
    expect0[0, 0, 0] = 0.6106874019515839 / l ** 2
    np.testing.assert_allclose(G[0], expect0, rtol=1e-14, atol=0)


def test_shell_ties_go_to_the_outer_shell():
    """Reading of the closed window (Sec. 2.1): a node exactly at distance
    r_k belongs to shell k only (half-open [r_k, r_{k+1})), and a node
    exactly at r_K to no shell. With l = 1 and the node rule, node (3, 4, 0)
    is exactly 5 from the source and (0, 0, 7) exactly 7; the expected shell
    of every node comes from exact integer comparisons d^2 vs r_k^2."""
    n, L = 16, 16.0
    radii = np.array([0.0, 2.3, 5.0, 7.0])        # r_2 = 5 and r_3 = 7 are met exactly
    G = oracle.build_G(n, L, radii, 1, li.Atten(kind=0))
    idx = np.arange(n)
    e = np.minimum(idx, n - idx)
    d2 = e[:, None, None] ** 2 + e[None, :, None] ** 2 + e[None, None, :] ** 2   # exact integers
    r2 = [0, None, 25, 49]                        # squares of the exact radii (r_1 = 2.3 is met by no node)
    shell = np.full(d2.shape, -1)
    shell[(d2 > 0) & (d2 * 100 < 529)] = 0        # d < 2.3  <=>  100 d^2 < 529
    shell[(d2 * 100 >= 529) & (d2 < r2[2])] = 1
    shell[(d2 >= r2[2]) & (d2 < r2[3])] = 2
    ties = [(3, 4, 0), (0, 0, 5), (0, 3, 4), (0, 0, 7), (2, 3, 6), (6, 3, 2)]
    assert shell[3, 4, 0] == 2 and shell[0, 0, 5] == 2 and shell[0, 0, 7] == -1 and shell[2, 3, 6] == -1
    for k in (1, 2):
        want = np.where(shell == k, 1.0 / (4 * np.pi * np.where(d2 > 0, d2, 1)), 0.0)
        np.testing.assert_allclose(G[k], want, rtol=1e-15, atol=0)
    for t in ties:
        assert G[1][t] == 0.0                     # never in the inner shell as well
    # the same through route D: a unit source in slice 2 is seen at the tie node
    src = [(np.zeros(0, np.int64), np.zeros(0))] * 3
    src = [src[0], src[1], (np.array([0], np.int64), np.array([1.0]))]
    J = oracle.field_direct(G, src, np.array([(3 * n + 4) * n + 0, (0 * n + 0) * n + 7]))
    assert abs(J[0] - 1.0 / (4 * np.pi * 25.0)) <= 1e-16 and J[1] == 0.0


def test_support_route_equals_dense_route():
    """Route D over the kernel's support (displacements near each shell,
    all bands at once) against route D with the dense kernel, with ties,
    attenuation, the paper's hard cut and an empty slice."""
    n, L = 32, 40.0
    radii = np.array([0.0, 2.5, 5.0, 7.5, 10.0, 12.5, 15.0])   # exact multiples of l = 1.25
    bands = [li.Atten(kind=0), li.lw_band(12.0),
             li.Atten(kind=2, a=1.7, s=116.29 * 0.1, p=0.68, c=0.7, cut=97.39 * 0.1)]
    srcs = [li.random_sources([9, k], n, 40) for k in range(6)]
    srcs[2] = (np.zeros(0, np.int64), np.zeros(0))
    tg = li.sample_cells(5, n, 300)
    JS = oracle.field_direct_support(n, L, radii, 2, bands, srcs, tg)
    for b, at in enumerate(bands):
        JD = oracle.field_direct(oracle.build_G(n, L, radii, 2, at), srcs, tg)
        assert np.max(np.abs(JS[b] - JD)) <= 1e-14 * np.max(np.abs(JD))
    with pytest.raises(ValueError):
        oracle.field_direct_support(n, L, np.array([0.0, 10.0, 19.0]), 2, bands[:1], srcs[:2], tg)


def test_causality_support_exact_zero():
    """A point source in slice k gives exactly 0 at nodes with no image
    distance inside [r_k, r_{k+1}) (route D, node rule)."""
    n, L = 12, 12.0
    radii = np.array([0.0, 1.9, 3.3, 4.9])
    at = li.Atten(kind=0)
    G = oracle.build_G(n, L, radii, 1, at)
    src = [(np.zeros(0, np.int64), np.zeros(0))] * 3
    c0 = (3 * n + 5) * n + 7
    src = [src[0], (np.array([c0]), np.array([2.5])), src[2]]
    targets = np.arange(n ** 3)
    J = oracle.field_direct(G, src, targets)
    i, j, x = np.unravel_index(targets, (n, n, n))
    ci, cj, cx = 3, 5, 7
    dist = []
    for a, b in ((i, ci), (j, cj), (x, cx)):
        dd = np.abs(a - b)
        dist.append(np.minimum(dd, n - dd))
    r = np.sqrt(dist[0] ** 2 + dist[1] ** 2 + dist[2] ** 2) * (L / n)
    outside = (r < radii[1]) | (r >= radii[2])
    assert np.all(J[outside] == 0.0)
    assert np.all(J[~outside] > 0.0)
    np.testing.assert_allclose(J[~outside], 2.5 / (4 * np.pi * r[~outside] ** 2), rtol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 4])
def test_kernel_cube_symmetries_and_real_spectrum(m):
    n, L, radii, _, at = _small_box(n=12, L=9.0, K=3, rmax=11.0, kind=1)
    G = oracle.build_G(n, L, radii, m, at)
    for k in range(G.shape[0]):
        g = G[k]
        # reflections (image sums meet in another order: 1-ulp rounding)
        for ax in range(3):
            np.testing.assert_allclose(g, np.roll(np.flip(g, axis=ax), 1, axis=ax), rtol=1e-14, atol=0)
        # axis permutations
        for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0), (1, 2, 0), (2, 0, 1)]:
            np.testing.assert_allclose(g, np.transpose(g, perm), rtol=1e-14, atol=0)
        Gh = np.fft.fftn(g)
        assert np.max(np.abs(Gh.imag)) <= 1e-14 * np.max(np.abs(Gh.real))


def test_flux_conservation_no_attenuation():
    """l^3 sum_c G_k(c) approximates the shell width r_{k+1} - r_k (the shell
    integral of 1/(4 pi r^2) over its volume)."""
    w = li.points_32c_8s()
    b = w.boxes[0]
    l = b.box / b.n
    G4 = oracle.build_G(b.n, b.box, b.radii, 4, b.bands[0])
    ratio = G4.sum(axis=(1, 2, 3)) * l ** 3 / np.diff(b.radii)
    assert np.max(np.abs(ratio - 1)) <= 5e-3
    G1 = oracle.build_G(b.n, b.box, b.radii, 1, b.bands[0])
    ratio1 = G1.sum(axis=(1, 2, 3)) * l ** 3 / np.diff(b.radii)
    assert np.max(np.abs(ratio1 - 1)) <= 0.05
    Gc = oracle.build_G(b.n, b.box, b.radii, 2, b.bands[0], conserve=1)
    ratio_c = Gc.sum(axis=(1, 2, 3)) * l ** 3 / np.diff(b.radii)
    np.testing.assert_allclose(ratio_c, 1.0, rtol=1e-14)


def test_flux_with_attenuation_vs_closed_form():
    a, s, p, c = 1.7, 20.0 / li.LW_X0, 0.68, 0.7
    at = li.Atten(kind=1, a=a, s=s, p=p, c=c)
    n, L = 32, 32.0                       # 3-cell shells, m = 4
    radii = np.linspace(0.0, 24.0, 9)
    l = L / n
    G = oracle.build_G(n, L, radii, 4, at)
    mp.mp.dps = 20
    r0 = s * math.log(a / c) ** (1 / p)

    def Phi(R):
        U = min(R, r0)
        return float(a * (s / p) * mp.gammainc(1 / p, 0, (mp.mpf(U) / s) ** p) - c * U)

    for k in range(8):
        I = Phi(radii[k + 1]) - Phi(radii[k])
        flux = G[k].sum() * l ** 3
        if I > 0.05 * (radii[k + 1] - radii[k]):
            assert abs(flux / I - 1) <= 5e-3, (k, flux, I)
        else:
            assert abs(flux - I) <= 5e-3 * (radii[k + 1] - radii[k])
        assert abs(oracle.shell_integral(at, radii[k], radii[k + 1]) - I) <= 1e-13 * max(1, abs(I))


def test_continuum_limit_sine_integral():
    """G^_k(p) l^3 -> (Si(kappa r_{k+1}) - Si(kappa r_k))/kappa, kappa = 2 pi |p|/L,
    the Fourier transform of a 1/(4 pi r^2) shell. The discrete kernel differs
    by O((kappa l)^2) (cell window, subpoint rule), so the error must be small
    at |p| = 1 and shrink about 4x when the grid is refined at fixed L."""
    from scipy.special import sici
    L, K = 20.0, 8
    radii = np.linspace(0.0, 20.0, K + 1)
    errs = {}
    for n in (16, 32):
        l = L / n
        G = oracle.build_G(n, L, radii, 4, li.Atten(kind=0))
        worst = 0.0
        for k in range(1, K):
            Gh = oracle.dft3(G[k])
            kap = 2 * np.pi / L
            ref = (sici(kap * radii[k + 1])[0] - sici(kap * radii[k])[0]) / kap
            got = Gh[0, 0, 1].real * l ** 3
            worst = max(worst, abs(got - ref) / (radii[k + 1] - radii[k]))
        errs[n] = worst
    assert errs[32] <= 5e-3
    assert errs[32] <= errs[16] / 2.0


# --- routes, DFT ---------------------------------------------------------------------------

def test_naive_dft_matches_numpy_and_brute_force():
    rng = np.random.default_rng(11)
    for n in (6, 8, 12):
        x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        X = oracle.dft3(x)
        np.testing.assert_allclose(X, np.fft.fftn(x), rtol=0, atol=1e-12 * np.abs(X).max())
        Xb = oracle.dft3_brute(x)
        np.testing.assert_allclose(X, Xb, rtol=0, atol=1e-12 * np.abs(X).max())
        xi = oracle.dft3(X, +1) / n ** 3
        np.testing.assert_allclose(xi, x, rtol=0, atol=1e-13)


def test_dft_identities():
    n = 10
    d = np.zeros((n, n, n)); d[0, 0, 0] = 1.0
    np.testing.assert_allclose(oracle.dft3(d), np.ones((n, n, n)), atol=1e-15)
    one = np.ones((n, n, n))
    D = oracle.dft3(one)
    assert abs(D[0, 0, 0] - n ** 3) < 1e-10
    D[0, 0, 0] = 0
    assert np.max(np.abs(D)) < 1e-11
    rng = np.random.default_rng(3)
    x = rng.standard_normal((n, n, n))
    X = oracle.dft3(x)
    # Parseval
    assert abs(np.sum(x ** 2) - np.sum(np.abs(X) ** 2) / n ** 3) <= 1e-13 * np.sum(x ** 2)
    # shift theorem along each axis
    for ax in range(3):
        Xs = oracle.dft3(np.roll(x, 1, axis=ax))
        ph = np.exp(-2j * np.pi * np.arange(n) / n)
        shape = [1, 1, 1]; shape[ax] = n
        np.testing.assert_allclose(Xs, X * ph.reshape(shape), atol=1e-12 * np.abs(X).max())


def _random_case(n, K, m, kind, seed, L=None):
    L = L or 1.25 * n
    radii = np.linspace(0.0, 0.9 * L, K + 1)
    at = li.Atten(kind=kind, a=1.7, s=0.6 * L / li.LW_X0, p=0.68, c=0.7)
    G = oracle.build_G(n, L, radii, m, at)
    srcs = [li.random_sources([seed, k], n, 17 + 3 * k) for k in range(K)]
    S = np.stack([oracle.deposit(n, c, v) for c, v in srcs])
    return G, S, srcs, radii, at, L


@pytest.mark.parametrize("m,kind", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_brute_force_16(m, kind):
    n, K = 16, 3
    G, S, srcs, *_ = _random_case(n, K, m, kind, seed=100 + m + 10 * kind)
    ref = sum(oracle.conv3_brute(G[k], S[k]) for k in range(K))
    JD = oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape(n, n, n)
    np.testing.assert_allclose(JD, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    JF = oracle.field_dft(G, S)
    np.testing.assert_allclose(JF, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # brute-force DFT of one slice's kernel against the separable one
    np.testing.assert_allclose(oracle.dft3_brute(G[1]), oracle.dft3(G[1]),
                               atol=1e-13 * np.abs(G[1]).sum())


def test_spectral_sum_equals_per_slice_inverse():
    G, S, *_ = _random_case(12, 4, 2, 1, seed=7)
    a = oracle.field_dft(G, S)
    b = oracle.field_per_slice_inverse(G, S)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())


def test_library_fft_route_matches_naive_route():
    G, S, *_ = _random_case(16, 3, 2, 0, seed=8)
    a = oracle.field_dft(G, S)
    b = oracle.field_fft(lambda k: G[k], lambda k: S[k], 3, 16)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


def test_uniform_source_constant_field_and_analytic_mean():
    n, L, K = 16, 20.0, 4
    radii = np.linspace(0.0, 18.0, K + 1)
    s = 0.37
    for conserve in (0, 1):
        G = oracle.build_G(n, L, radii, 2, li.Atten(kind=0), conserve=conserve)
        S = np.full((K, n, n, n), s)
        J = oracle.field_dft(G, S)
        expect = s * G.sum()
        np.testing.assert_allclose(J, expect, rtol=1e-13)
        if conserve:
            l = L / n
            assert abs(expect - (s / l ** 3) * (radii[-1] - radii[0])) <= 1e-13 * expect


def test_mean_of_field_closed_form():
    G, S, srcs, *_ = _random_case(12, 3, 2, 1, seed=9)
    J = oracle.field_dft(G, S)
    assert abs(J.mean() - oracle.mean_field(G, S)) <= 1e-14 * abs(J.mean()) * 10


def test_linearity_translation_nonnegativity():
    n, K = 12, 3
    G, S1, srcs1, *_ = _random_case(n, K, 2, 1, seed=21)
    _, S2, srcs2, *_ = _random_case(n, K, 2, 1, seed=22)
    J1 = oracle.field_dft(G, S1)
    J2 = oracle.field_dft(G, S2)
    J12 = oracle.field_dft(G, 2.0 * S1 - 0.5 * S2)
    np.testing.assert_allclose(J12, 2.0 * J1 - 0.5 * J2, atol=1e-13 * np.abs(J12).max())
    shift = (2, 5, 7)
    Jr = oracle.field_dft(G, np.roll(S1, shift, axis=(1, 2, 3)))
    np.testing.assert_allclose(Jr, np.roll(J1, shift, axis=(0, 1, 2)), atol=1e-13 * np.abs(J1).max())
    JD = oracle.field_direct(G, srcs1, np.arange(n ** 3))
    assert np.all(JD >= 0.0)
    assert J1.min() >= -1e-13 * J1.max()


def test_single_point_source_reproduces_translated_kernel():
    n, K = 12, 3
    G, *_ = _random_case(n, K, 2, 1, seed=1)
    c0 = (4 * n + 1) * n + 9
    for k in range(K):
        srcs = [(np.zeros(0, np.int64), np.zeros(0))] * K
        srcs = list(srcs)
        srcs[k] = (np.array([c0]), np.array([3.0]))
        J = oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape(n, n, n)
        np.testing.assert_array_equal(J, 3.0 * np.roll(G[k], (4, 1, 9), axis=(0, 1, 2)))
        S = np.stack([oracle.deposit(n, c, v) for c, v in srcs])
        JF = oracle.field_dft(G, S)
        np.testing.assert_allclose(JF, J, atol=1e-14 * np.abs(J).max() * 10)


def test_G_at_matches_dense_and_ondemand_route():
    n, L = 16, 24.0
    radii = np.linspace(0.0, 11.0, 5)
    at = li.Atten(kind=1, a=1.7, s=9.0 / li.LW_X0, p=0.68, c=0.7)
    G = oracle.build_G(n, L, radii, 2, at)
    for d in [(0, 0, 0), (1, 2, 3), (15, 0, 8), (5, 11, 2)]:
        np.testing.assert_array_equal(oracle.G_at(n, L, radii, 2, at, d), G[:, d[0], d[1], d[2]])
    srcs = [li.random_sources([5, k], n, 40) for k in range(4)]
    t = li.sample_cells(3, n, 200)
    a = oracle.field_direct(G, srcs, t)
    b = oracle.field_direct_ondemand(n, L, radii, 2, at, srcs, t)
    np.testing.assert_allclose(b, a, rtol=1e-14, atol=1e-16)


def test_image_sum_beyond_half_box():
    """Shells reaching past L/2 collect several periodic images: the node
    rule value equals the explicit sum over images in the shell."""
    n, L = 8, 8.0
    radii = np.array([0.0, 3.0, 9.5])
    G = oracle.build_G(n, L, radii, 1, li.Atten(kind=0))
    for d in [(1, 2, 3), (0, 0, 4), (4, 4, 4)]:
        tot = 0.0
        for u in range(-3, 4):
            for v in range(-3, 4):
                for w in range(-3, 4):
                    r = math.sqrt((d[0] + u * n) ** 2 + (d[1] + v * n) ** 2 + (d[2] + w * n) ** 2)
                    if 3.0 <= r < 9.5:
                        tot += 1 / (4 * math.pi * r * r)
        assert abs(G[1][d] - tot) <= 1e-15 * tot
