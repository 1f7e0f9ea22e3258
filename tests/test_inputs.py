"""Seeded input generators: determinism and the counts each recipe fixes."""
import numpy as np

import lc_inputs as li


def test_grid32_deterministic_and_shape():
    a = li.points_32c_8s().boxes[0]
    b = li.points_32c_8s().boxes[0]
    assert a.n == 32 and a.n_slices == 8 and a.supersample == 1
    np.testing.assert_array_equal(a.radii, np.arange(9) * 2.5)
    for (c1, l1), (c2, l2) in zip(a.sources, b.sources):
        np.testing.assert_array_equal(c1, c2)
        np.testing.assert_array_equal(l1, l2)
        assert len(c1) == 200 and c1.min() >= 0 and c1.max() < 32 ** 3
        assert np.all(l1 > 0)


def test_growing_counts():
    cnt = li.growing_counts(40)
    assert cnt[0] == 46585 and cnt[-1] == 200
    assert sum(cnt) == 355816


def test_grf_top_fraction():
    rng = np.random.default_rng([2, 0, 0])
    cells, lum = li.grf_peak_sources(rng, 32)
    assert len(cells) == int(0.01 * 32 ** 3)
    assert len(np.unique(cells)) == len(cells)
    assert np.all(lum > 0)


def test_uneven_mix():
    w = li.uneven_16boxes()
    assert len(w.boxes) == 16
    for b in w.boxes:
        assert b.n in (64, 96, 128, 192, 256)
        assert 8 <= b.n_slices <= 48
        assert abs(b.box / b.n - 0.78125) < 1e-15
    lam = np.mean([len(c) / b.n ** 3 for b in w.boxes[:2] for c, _ in b.sources])
    assert 0.8e-3 < lam < 1.2e-3


def test_lw_band_horizon():
    for h in (100.0, 80.0, 60.0, 40.0):
        at = li.lw_band(h)
        assert abs(at.s * li.LW_X0 - h) < 1e-12 * h
