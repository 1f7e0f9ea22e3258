"""Pins of the oracle's particle-mesh near-field correction (Sec. 4: direct
summation for nearby sources, the FFT method for the far field), no GPU.

- Node-centred sources with the node rule (m = 1): the exact kernel at a
  node's distance is the mesh kernel's primary image, so the correction
  vanishes exactly.
- One source inside its cell, one periodic image: after the correction the
  field at every node of the near cube but its own is L phi/(4 pi rho^2) at
  the exact distance rho (zero outside the shell), a closed form; nodes
  outside the cube keep the mesh value.
- The correction is linear in the sources and does not depend on where in
  the box a configuration sits (translation by whole cells)."""
import numpy as np

import lc_inputs as li
import oracle


def _mesh(n, L, radii, m, at, positioned):
    G = oracle.build_G(n, L, radii, m, at)
    srcs = [(oracle.ngp_cells(n, L, p), v) for p, v in positioned]
    return oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape((n,) * 3)


def test_node_centred_sources_need_no_correction():
    n, L = 16, 16.0                       # l = 1: node positions are exact
    radii = np.array([0.0, 2.3, 4.6, 6.9])
    at = li.Atten(kind=0)
    rng = np.random.default_rng(3)
    positioned = []
    for k in range(3):
        c = rng.integers(0, n, size=(5, 3)).astype(np.float64)
        positioned.append((c * 1.0, rng.lognormal(size=5)))
    corr = oracle.near_correction(n, L, radii, 1, [at] * 3, positioned, 3)
    assert np.max(np.abs(corr)) == 0.0


def test_single_offnode_source_gets_the_exact_kernel_nearby():
    n, L = 24, 24.0
    radii = np.array([0.0, 1.7, 3.1, 5.0])      # r_K + cube diagonal < L/2: one image
    at = li.lw_band(6.0)
    R = 3
    x_s = np.array([[7.31, 12.68, 3.55]])       # nearest node (7, 13, 4)
    lum = np.array([2.5])
    for k in range(3):
        positioned = [(np.zeros((0, 3)), np.zeros(0))] * 3
        positioned = [positioned[0], positioned[1], positioned[2]]
        positioned[k] = (x_s, lum)
        J = _mesh(n, L, radii, 2, at, positioned) + oracle.near_correction(n, L, radii, 2, [at] * 3, positioned, R)
        Jm = _mesh(n, L, radii, 2, at, positioned)
        c = np.array([7, 13, 4])
        for o in np.ndindex(2 * R + 1, 2 * R + 1, 2 * R + 1):
            o = np.array(o) - R
            x = tuple((c + o) % n)
            if not o.any():
                assert J[x] == Jm[x]            # own node: mesh value kept
                continue
            rho = np.linalg.norm((c + o) * 1.0 - x_s[0])
            want = lum[0] * oracle.phi(at, rho) / (4 * np.pi * rho ** 2) if radii[k] <= rho < radii[k + 1] else 0.0
            assert abs(J[x] - want) <= 1e-14 * max(abs(want), 1e-3), (k, o, J[x], want)
        # outside the cube the field is the mesh field
        mask = np.ones((n,) * 3, bool)
        for o in np.ndindex(2 * R + 1, 2 * R + 1, 2 * R + 1):
            mask[tuple((c + np.array(o) - R) % n)] = False
        assert np.array_equal(J[mask], Jm[mask])


def test_correction_is_linear_and_translation_invariant():
    n, L = 20, 25.0
    radii = np.array([0.0, 2.0, 4.5, 7.0])
    ats = [li.lw_band(8.0), li.Atten(kind=0, prefactor=0.5), li.lw_band(5.0)]
    a = [li.positioned_sources([7, k], L, 6) for k in range(3)]
    b = [li.positioned_sources([8, k], L, 4) for k in range(3)]
    ca = oracle.near_correction(n, L, radii, 2, ats, a, 2)
    cb = oracle.near_correction(n, L, radii, 2, ats, b, 2)
    ab = [(np.concatenate([pa, pb]), np.concatenate([va, 2.0 * vb])) for (pa, va), (pb, vb) in zip(a, b)]
    cab = oracle.near_correction(n, L, radii, 2, ats, ab, 2)
    np.testing.assert_allclose(cab, ca + 2.0 * cb, rtol=1e-12, atol=1e-14 * np.max(np.abs(cab)))
    shift = np.array([3, -2, 5])
    l = L / n
    moved = [(p + shift * l, v) for p, v in a]
    cm = oracle.near_correction(n, L, radii, 2, ats, moved, 2)
    np.testing.assert_allclose(cm, np.roll(ca, tuple(shift), axis=(0, 1, 2)), rtol=1e-12,
                               atol=1e-14 * np.max(np.abs(ca)))
