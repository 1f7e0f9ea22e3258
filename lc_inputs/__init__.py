"""Seeded synthetic inputs for the light-cone field workloads.

This module only draws random inputs: box geometry, slice radii, attenuation
parameters and per-slice point-source lists (flat cell index, luminosity).
It holds none of the method's arithmetic (no shell kernel, no transform, no
slice sum), so both the CPU oracle and the HIP library consume exactly the
same inputs from here and share nothing else.

One input format conversion lives here: `dense_grid` writes a point list as
a per-cell luminosity grid (coincident sources add), the input format of a
simulation that keeps its sources on the mesh. It feeds the library's
dense-grid entry only; the oracle's own grids come from `oracle.deposit`,
and its direct-summation routes take the point lists themselves.

The paper's own source fields (first-star luminosities from a reionization
simulation, Sec. 3) are not available; these recipes stand in for them with
the same shapes: periodic 32^3..512^3 grids, many lookback slices, shells out
to a ~100 Mpc horizon.

Cell convention: flat index (i*N + j)*N + k, with k (x) the contiguous axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# zero of a*exp(-(r/s)^p) - c in units of s, for a=1.7, c=0.7, p=0.68
# (the Lyman-Werner modulation factor, Eq. 15): x0 = ln(17/7)^(1/0.68)
LW_X0 = math.log(1.7 / 0.7) ** (1.0 / 0.68)


@dataclasses.dataclass
class Atten:
    """Radial factor phi(r) multiplying 1/(4 pi r^2) in the shell kernel.

    kind 0: phi = 1
    kind 1: phi = max(0, a*exp(-(r/s)^p) - c)       (continuous form)
    kind 2: phi = a*exp(-(r/s)^p) - c if r <= cut else 0   (Eq. 15 as printed)
    """
    kind: int = 0
    a: float = 1.7
    s: float = 116.0
    p: float = 0.68
    c: float = 0.7
    cut: float = 0.0
    prefactor: float = 1.0


@dataclasses.dataclass
class Box:
    n: int
    box: float
    radii: np.ndarray            # K+1 float64, strictly increasing
    supersample: int
    bands: List[Atten]
    sources: List[Tuple[np.ndarray, np.ndarray]]  # per slice (cells int64, lum float64)
    conserve: int = 0
    rule: int = 0                # mesh kernel: 0 m^3 subpoints, 1 exact cell average

    @property
    def n_slices(self) -> int:
        return len(self.radii) - 1


@dataclasses.dataclass
class Workload:
    name: str
    boxes: List[Box]

    def cell_slices(self) -> int:
        return sum(b.n ** 3 * b.n_slices for b in self.boxes)


def equal_radii(r_max: float, k: int) -> np.ndarray:
    """K equal-width shells spanning [0, r_max]; computed once, passed to both sides."""
    return np.array([r_max * i / k for i in range(k + 1)], dtype=np.float64)


def uniform_sources(rng: np.random.Generator, n_cells: int, count: int):
    cells = rng.integers(0, n_cells, size=count, dtype=np.int64)
    lum = rng.lognormal(mean=0.0, sigma=1.0, size=count)
    return cells, lum.astype(np.float64)


def poisson_sources(rng: np.random.Generator, n: int, density: float):
    """Poisson process of `density` sources per cell: a Poisson total count
    placed at independent uniform cells (equivalent in law to independent
    Poisson(density) counts per cell)."""
    count = rng.poisson(density * n ** 3)
    cells = np.sort(rng.integers(0, n ** 3, size=count, dtype=np.int64))
    lum = rng.lognormal(mean=0.0, sigma=1.0, size=count)
    return cells, lum.astype(np.float64)


def grf_peak_sources(rng: np.random.Generator, n: int, frac: float = 0.01, workers: int = -1):
    """Top `frac` of cells of a Gaussian random field with P(k) ~ k^-2.

    White noise is filtered by |k|^-1 in Fourier space (k=0 mode zeroed).
    Luminosity is the excess of the field over the first rejected value.
    (scipy's transforms give the same bits for any `workers`.)
    """
    import scipy.fft as sfft
    white = rng.standard_normal((n, n, n))
    wk = sfft.rfftn(white, workers=workers)
    del white
    f0 = np.fft.fftfreq(n) * n
    fx = np.fft.rfftfreq(n) * n
    kk = (f0[:, None, None] ** 2 + f0[None, :, None] ** 2 + fx[None, None, :] ** 2)
    kk[0, 0, 0] = 1.0
    wk /= np.sqrt(kk)
    wk[0, 0, 0] = 0.0
    del kk
    delta = sfft.irfftn(wk, s=(n, n, n), workers=workers).ravel()
    del wk
    keep = int(math.floor(frac * n ** 3))
    part = np.argpartition(delta, delta.size - keep - 1)
    top = part[delta.size - keep:]
    thresh = delta[part[delta.size - keep - 1]]
    cells = np.sort(top).astype(np.int64)
    lum = (delta[cells] - thresh).astype(np.float64)
    return cells, lum


def lw_band(horizon: float) -> Atten:
    """Continuous LW modulation with its zero placed at `horizon`."""
    return Atten(kind=1, a=1.7, s=horizon / LW_X0, p=0.68, c=0.7)


# --- the five workloads ------------------------------------------------------

def points_32c_8s(seed_base: int = 1) -> Workload:
    """32^3, 20 Mpc, 8 equal slices over 0-20 Mpc, 200 uniform sources/slice,
    phi = 1, node rule (m = 1)."""
    n, L, K = 32, 20.0, 8
    srcs = []
    for k in range(K):
        rng = np.random.default_rng([seed_base, 0, k])
        srcs.append(uniform_sources(rng, n ** 3, 200))
    b = Box(n=n, box=L, radii=equal_radii(20.0, K), supersample=1,
            bands=[Atten(kind=0)], sources=srcs)
    return Workload("grid32_slices8", [b])


def grf_128c_24s(seed_base: int = 2, n: int = 128) -> Workload:
    """128^3, 100 Mpc, 24 slices over 0-100 Mpc, top-1% GRF peaks, LW-like
    attenuation with s = 116 Mpc, m = 4."""
    L, K = 100.0 * n / 128, 24
    srcs = []
    for k in range(K):
        rng = np.random.default_rng([seed_base, 0, k])
        srcs.append(grf_peak_sources(rng, n))
    b = Box(n=n, box=L, radii=equal_radii(L, K), supersample=4,
            bands=[Atten(kind=1, a=1.7, s=116.0, p=0.68, c=0.7)], sources=srcs)
    return Workload(f"grid{n}_slices24_grf", [b])


def growing_counts(K: int = 40) -> List[int]:
    return [int(round(200 * 1.15 ** (K - 1 - k))) for k in range(K)]


def points_256c_40s(seed_base: int = 3, n: int = 256, K: int = 40) -> Workload:
    """256^3, 200 Mpc, 40 slices of 5 Mpc, uniform lognormal sources whose
    count grows x1.15 per slice toward the present, phi = 1, m = 4."""
    L = 200.0 * n / 256
    srcs = []
    for k, cnt in enumerate(growing_counts(K)):
        rng = np.random.default_rng([seed_base, 0, k])
        srcs.append(uniform_sources(rng, n ** 3, cnt))
    b = Box(n=n, box=L, radii=equal_radii(L, K), supersample=4,
            bands=[Atten(kind=0)], sources=srcs)
    return Workload(f"grid{n}_slices{K}", [b])


def _grf_slice(seed_base: int, k: int, n: int):
    """GRF peak sources of slice k (one process of a pool)."""
    return grf_peak_sources(np.random.default_rng([seed_base, 0, k]), n, workers=1)


def bands_512c_60s(seed_base: int = 4, n: int = 512, K: int = 60,
         horizons=(100.0, 80.0, 60.0, 40.0), recipe: str = "grf", procs: int = 1) -> Workload:
    """512^3, 400 Mpc, 60 slices over 0-100 Mpc, 4 LW-like bands with
    horizons 100/80/60/40 Mpc sharing the sources. With procs > 1 the GRF
    slices are drawn by a pool of that many processes (same values: each
    slice has its own seed)."""
    L = 400.0 * n / 512
    r_max = 100.0 * n / 512
    if recipe == "grf" and procs > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as ex:
            srcs = list(ex.map(_grf_slice, [seed_base] * K, range(K), [n] * K))
    else:
        srcs = []
        for k in range(K):
            rng = np.random.default_rng([seed_base, 0, k])
            if recipe == "grf":
                srcs.append(grf_peak_sources(rng, n))
            else:
                srcs.append(uniform_sources(rng, n ** 3, int(0.01 * n ** 3)))
    bands = [lw_band(h * n / 512) for h in horizons]
    b = Box(n=n, box=L, radii=equal_radii(r_max, K), supersample=4,
            bands=bands, sources=srcs)
    return Workload(f"grid{n}_slices{K}_bands{len(bands)}", [b])


def uneven_16boxes(seed_base: int = 5, sizes=(64, 96, 128, 192, 256), n_boxes: int = 16,
         k_range=(8, 48), density: float = 1e-3) -> Workload:
    """16 independent boxes with N drawn from {64,96,128,192,256}, cell size
    0.78125 Mpc, 8..48 equal slices spanning the box side, Poisson sources."""
    rng0 = np.random.default_rng([seed_base, 0])
    ns = rng0.choice(np.array(sizes), size=n_boxes)
    ks = rng0.integers(k_range[0], k_range[1] + 1, size=n_boxes)
    boxes = []
    for bi in range(n_boxes):
        n, K = int(ns[bi]), int(ks[bi])
        L = 0.78125 * n
        srcs = []
        for k in range(K):
            rng = np.random.default_rng([seed_base, bi + 1, k])
            srcs.append(poisson_sources(rng, n, density))
        boxes.append(Box(n=n, box=L, radii=equal_radii(L, K), supersample=4,
                         bands=[Atten(kind=0)], sources=srcs))
    return Workload(f"uneven{n_boxes}boxes", boxes)


def positioned_sources(seed, L: float, count: int):
    """Sources with continuous positions: uniform in [0, L)^3 (axis order
    i, j, k), lognormal luminosities. Returns (pos (count, 3), lum)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(count, 3))
    lum = rng.lognormal(mean=0.0, sigma=1.0, size=count)
    return pos, lum


def random_sources(seed, n: int, count: int):
    """Small generic case for tests: uniform cells, lognormal luminosity."""
    return uniform_sources(np.random.default_rng(seed), n ** 3, count)


def sample_cells(seed, n: int, count: int) -> np.ndarray:
    """Distinct random target cells for sampled comparisons."""
    rng = np.random.default_rng(seed)
    count = min(count, n ** 3)
    return np.sort(rng.choice(n ** 3, size=count, replace=False)).astype(np.int64)


def sublattice_cells(n: int, stride: int, offset: int = 0) -> np.ndarray:
    idx = np.arange(offset, n, stride, dtype=np.int64)
    i, j, k = np.meshgrid(idx, idx, idx, indexing="ij")
    return ((i * n + j) * n + k).ravel()


def dense_grid(n: int, cells: np.ndarray, lum: np.ndarray, dtype=np.float64) -> np.ndarray:
    """The per-cell luminosity field of a point list (several sources in a
    cell add): the dense source grid of one slice, as the input format of a
    simulation that stores its sources on the mesh."""
    g = np.bincount(np.asarray(cells, np.int64), weights=np.asarray(lum, np.float64),
                    minlength=n ** 3)
    return g.astype(dtype, copy=False)


def sources_digest(box: Box) -> str:
    """SHA-256 of a box's per-slice point lists (cells then luminosities):
    names the exact inputs a stored reference was computed from."""
    import hashlib
    h = hashlib.sha256()
    for c, v in box.sources:
        h.update(np.ascontiguousarray(c, np.int64).tobytes())
        h.update(np.ascontiguousarray(v, np.float64).tobytes())
    return h.hexdigest()
