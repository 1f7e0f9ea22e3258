"""CPU FP64 oracle for the periodic retarded-time (light-cone) field.

TEST INFRASTRUCTURE ONLY. Imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg; never by the product library, which has no CPU
path. It shares no code with the HIP library: only the seeded inputs of
`lc_inputs` are common to both.

Routes (Sec. 2.2, Eqs. 11-13 and algorithm steps 2-6):
  * build_G        - shell kernel G_k by direct summation over images and
                     subpoints (step 2), dense over the grid.
  * field_direct   - route D: the circular convolution sum of Eq. 11 summed
                     over slices (step 6), at any set of target cells.
  * field_dft      - route F: naive separable DFT of Eq. 12, product of
                     Eq. 13 summed over slices, naive inverse, / N^3.
  * field_fft      - route F with a library FFT (scipy.fft, FP64) as the
                     transform step, for grids too large for the naive DFT.
  * field_direct_support - route D summed over the kernel's support (the
                     displacements that can meet each shell), for large grids
                     with an outer radius well inside half the box.
  * field_per_slice_inverse - the paper's literal order (inverse per slice,
                     then sum; steps 5-6), used to check the spectral sum.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Atten(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("a", C.c_double),
                ("s", C.c_double), ("p", C.c_double), ("c", C.c_double),
                ("cut", C.c_double), ("prefactor", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        ap = C.POINTER(_Atten)
        L.or_phi.argtypes = [ap, C.c_double]; L.or_phi.restype = C.c_double
        L.or_Phi.argtypes = [ap, C.c_double]; L.or_Phi.restype = C.c_double
        L.or_shell_integral.argtypes = [ap, C.c_double, C.c_double]
        L.or_shell_integral.restype = C.c_double
        L.or_self_cell.argtypes = [ap, C.c_double]; L.or_self_cell.restype = C.c_double
        L.or_G_at.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int, ap,
                              C.c_int, C.c_int, C.c_int, dp]
        L.or_build_G.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int, ap,
                                 C.c_int, dp]
        L.or_field_direct.argtypes = [C.c_int, C.c_int, dp, ip, ip, dp, C.c_int64, ip, dp]
        L.or_field_direct_ondemand.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int,
                                               ap, ip, ip, dp, C.c_int64, ip, dp]
        L.or_field_direct_support.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int, C.c_int,
                                              ap, ip, ip, dp, C.c_int64, ip, dp]
        L.or_dft3_naive.argtypes = [C.c_int, C.c_int, C.c_void_p]
        L.or_cosmic_time.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_cosmic_time.restype = C.c_double
        L.or_comoving_distance.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_comoving_distance.restype = C.c_double
        L.or_redshift_at_time.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_redshift_at_time.restype = C.c_double
        L.or_build_G_slices.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int, ap, C.c_int, dp]
        L.or_near_correction.argtypes = [C.c_int, C.c_double, C.c_int, dp, C.c_int, ap, ip, dp, dp,
                                         C.c_int, dp, C.c_int, C.c_int]
        L.or_dft3_brute.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        L.or_conv3_brute.argtypes = [C.c_int, dp, dp, dp]
        L.or_num_threads.restype = C.c_int
        L.or_theta_rect.argtypes = [C.c_double] * 5; L.or_theta_rect.restype = C.c_double
        L.or_cell_average.argtypes = [ap, C.c_double, dp, C.c_double, C.c_double, C.c_int]
        L.or_cell_average.restype = C.c_double
        L.or_G_exact_at.argtypes = [C.c_int, C.c_double, C.c_int, dp, ap, C.c_int, C.c_int, C.c_int,
                                    C.c_int, dp]
        L.or_build_G_exact.argtypes = [C.c_int, C.c_double, C.c_int, dp, ap, C.c_int, dp]
        _LIB = L
    return _LIB


def _atten(at) -> _Atten:
    return _Atten(int(at.kind), 0, float(at.a), float(at.s), float(at.p), float(at.c),
                  float(at.cut), float(at.prefactor))


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def num_threads() -> int:
    return int(lib().or_num_threads())


# --- radial factor, integrals, self cell -------------------------------------

def phi(at, r: float) -> float:
    a = _atten(at)
    return lib().or_phi(C.byref(a), float(r))


def Phi(at, R: float) -> float:
    """int_0^R phi(r) dr."""
    a = _atten(at)
    return lib().or_Phi(C.byref(a), float(R))


def shell_integral(at, r0: float, r1: float) -> float:
    a = _atten(at)
    return lib().or_shell_integral(C.byref(a), float(r0), float(r1))


def self_cell(at, l: float) -> float:
    """Cube average of prefactor*phi/(4 pi r^2) over a cell of side l."""
    a = _atten(at)
    return lib().or_self_cell(C.byref(a), float(l))


# --- shell kernel ---------------------------------------------------------------

def G_at(n: int, L: float, radii, m: int, at, disp) -> np.ndarray:
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    out = np.zeros(K)
    a = _atten(at)
    rc = lib().or_G_at(n, L, K, _dptr(radii), m, C.byref(a),
                       int(disp[0]), int(disp[1]), int(disp[2]), _dptr(out))
    assert rc == 0
    return out


def build_G(n: int, L: float, radii, m: int, at, conserve: int = 0) -> np.ndarray:
    """Dense G[k, i, j, x] for all shells, FP64."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    G = np.zeros((K, n, n, n))
    a = _atten(at)
    rc = lib().or_build_G(n, L, K, _dptr(radii), m, C.byref(a), int(conserve), _dptr(G))
    assert rc == 0
    return G


def build_G_slices(n: int, L: float, radii, m: int, attens, conserve: int = 0) -> np.ndarray:
    """Dense G[k] with radial factor attens[k] for slice k (the self cell of
    slice 0 with attens[0])."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    assert len(attens) == K
    G = np.zeros((K, n, n, n))
    arr = (_Atten * K)(*[_atten(a) for a in attens])
    rc = lib().or_build_G_slices(n, L, K, _dptr(radii), m, arr, int(conserve), _dptr(G))
    assert rc == 0
    return G


# --- exact cell-averaged kernel (the m -> infinity limit of the subpoint rule) ----------

EXACT_ORDER = 32   # Gauss-Legendre points per piece of the exact cell average


def theta_rect(R: float, x0: float, x1: float, y0: float, y1: float) -> float:
    """Angle of the circle of radius R (centred at the origin) inside the
    rectangle [x0, x1] x [y0, y1]."""
    return float(lib().or_theta_rect(R, x0, x1, y0, y1))


def cell_average(at, l: float, box, r_lo: float, r_hi: float, ng: int = EXACT_ORDER) -> float:
    """pref / l^3 times the integral over box = (x0, x1, y0, y1, z0, z1) of
    phi(r) / (4 pi r^2) on the shell r_lo <= r < r_hi (source at the origin)."""
    b = np.ascontiguousarray(box, dtype=np.float64)
    a = _atten(at)
    return float(lib().or_cell_average(C.byref(a), float(l), _dptr(b), float(r_lo), float(r_hi), int(ng)))


def G_exact_at(n: int, L: float, radii, at, disp, ng: int = EXACT_ORDER) -> np.ndarray:
    """All K exact cell-averaged shell values at one displacement (every image)."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    out = np.zeros(K)
    a = _atten(at)
    rc = lib().or_G_exact_at(n, L, K, _dptr(radii), C.byref(a), int(disp[0]), int(disp[1]), int(disp[2]),
                             int(ng), _dptr(out))
    assert rc == 0
    return out


def build_G_exact(n: int, L: float, radii, at, ng: int = EXACT_ORDER) -> np.ndarray:
    """Dense exact cell-averaged G[k, i, j, x], FP64."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    G = np.zeros((K, n, n, n))
    a = _atten(at)
    rc = lib().or_build_G_exact(n, L, K, _dptr(radii), C.byref(a), int(ng), _dptr(G))
    assert rc == 0
    return G


# --- cosmology (Sec. 2.1 Eqs. 4-5; Sec. 3 Eqs. 14-17) ---------------------------------

def cosmic_time(h: float, om: float, z: float) -> float:
    """Myr since the big bang at redshift z (flat matter + Lambda)."""
    return float(lib().or_cosmic_time(h, om, z))


def comoving_distance(h: float, om: float, z1: float, z2: float) -> float:
    """Comoving Mpc that light travels between redshifts z2 and z1 (z1 <= z2)."""
    return float(lib().or_comoving_distance(h, om, z1, z2))


def redshift_at_time(h: float, om: float, t: float) -> float:
    return float(lib().or_redshift_at_time(h, om, t))


def cosmo_slices(h: float, om: float, z_obs: float, dt_myr: float, K: int):
    """Slices of equal cosmic time before z_obs: radii r_k = c (tau_obs -
    tau_k) (comoving Mpc, r_0 = 0), edge redshifts z_k at t_obs - k dt and
    source redshifts at the slices' middle times t_obs - (k + 1/2) dt."""
    t0 = cosmic_time(h, om, z_obs)
    z_edge = [z_obs] + [redshift_at_time(h, om, t0 - k * dt_myr) for k in range(1, K + 1)]
    radii = [0.0] + [comoving_distance(h, om, z_obs, z) for z in z_edge[1:]]
    z_src = [redshift_at_time(h, om, t0 - (k + 0.5) * dt_myr) for k in range(K)]
    return np.array(radii), np.array(z_edge), np.array(z_src)


class _LWAtten:
    def __init__(self, kind, s, cut, prefactor):
        self.kind, self.a, self.s, self.p, self.c, self.cut, self.prefactor = kind, 1.7, s, 0.68, 0.7, cut, prefactor


def lw_factors(h: float, om: float, z_obs: float, z_src, kind: int = 2):
    """Per-slice Lyman-Werner factors: Eq. 16's alpha at each slice's source
    redshift, Eq. 15's scale and horizon, and Eq. 14's
    (1+z)^3 / (1+z_s) / (4 pi) (the kernel carries the other 1/(4 pi r^2))."""
    out = []
    for zs in z_src:
        alpha = (h / 0.7) ** -1 * (om / 0.27) ** -0.5 * ((1.0 + zs) / 21.0) ** -0.5
        out.append(_LWAtten(kind, 116.29 * alpha, 97.39 * alpha, (1.0 + z_obs) ** 3 / (1.0 + zs) / (4.0 * math.pi)))
    return out


def ngp_cells(n: int, L: float, pos: np.ndarray) -> np.ndarray:
    """Flat index of each positioned source's nearest node, round(x / l) mod N
    per axis (axis order i, j, k; k contiguous)."""
    l = L / n
    c = np.mod(np.floor(np.asarray(pos, np.float64) / l + 0.5).astype(np.int64), n)
    return (c[:, 0] * n + c[:, 1]) * n + c[:, 2]


def near_correction(n: int, L: float, radii, m: int, attens, positioned, R: int, rule: int = 0) -> np.ndarray:
    """Particle-mesh near-field correction (Sec. 4) of positioned sources:
    positioned[k] = (pos (n_k, 3) in length units, lum (n_k,)); attens[k]
    the radial factor of slice k; rule 1 for a mesh kernel of exact cell
    averages. Returns the N^3 correction grid."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    assert len(attens) == K and len(positioned) == K
    off = np.zeros(K + 1, dtype=np.int64)
    for k, (p, _) in enumerate(positioned):
        off[k + 1] = off[k] + len(p)
    pos = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1, 3) for p, _ in positioned])
                               if off[-1] else np.zeros((0, 3)))
    lum = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64) for _, v in positioned])
                               if off[-1] else np.zeros(0))
    arr = (_Atten * K)(*[_atten(a) for a in attens])
    corr = np.zeros(n ** 3)
    rc = lib().or_near_correction(n, L, K, _dptr(radii), m, arr, _iptr(off), _dptr(pos.ravel()), _dptr(lum),
                                  int(R), _dptr(corr), int(rule), EXACT_ORDER)
    assert rc == 0
    return corr.reshape(n, n, n)


def frozen_sources(sources, slice_: int = 0):
    """The instantaneous field's input (Eq. 18): every slice holds the
    sources of lookback slice `slice_`."""
    return [sources[slice_]] * len(sources)


def fdiff(J, J_inst):
    """(J_inst - J) / J elementwise, 0 where J == 0."""
    J = np.asarray(J, dtype=np.float64)
    Ji = np.asarray(J_inst, dtype=np.float64)
    out = np.zeros_like(J)
    nz = J != 0
    out[nz] = (Ji[nz] - J[nz]) / J[nz]
    return out


# --- sources ----------------------------------------------------------------------

def deposit(n: int, cells: np.ndarray, lum: np.ndarray) -> np.ndarray:
    """Nearest-grid-point deposit (l^3 absorbed, Eq. 11): S(c) = sum of L in c."""
    S = np.zeros(n ** 3)
    np.add.at(S, np.asarray(cells, dtype=np.int64), np.asarray(lum, dtype=np.float64))
    return S.reshape(n, n, n)


def _flatten_sources(sources: Sequence[Tuple[np.ndarray, np.ndarray]]):
    off = np.zeros(len(sources) + 1, dtype=np.int64)
    for k, (c, _) in enumerate(sources):
        off[k + 1] = off[k] + len(c)
    cells = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int64) for c, _ in sources])
                                 if off[-1] else np.zeros(0, np.int64))
    lum = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64) for _, v in sources])
                               if off[-1] else np.zeros(0, np.float64))
    return off, cells, lum


# --- route D ------------------------------------------------------------------------

def field_direct(G: np.ndarray, sources, targets: np.ndarray) -> np.ndarray:
    """J at target cells by direct periodic summation with a dense kernel
    G[k] (one band)."""
    K, n = G.shape[0], G.shape[1]
    assert len(sources) == K
    G = np.ascontiguousarray(G, dtype=np.float64)
    off, cells, lum = _flatten_sources(sources)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    J = np.zeros(len(targets))
    lib().or_field_direct(n, K, _dptr(G), _iptr(off), _iptr(cells), _dptr(lum),
                          len(targets), _iptr(targets), _dptr(J))
    return J


def field_direct_ondemand(n: int, L: float, radii, m: int, at, sources,
                          targets: np.ndarray) -> np.ndarray:
    """Route D evaluating each needed kernel value from its definition
    (no dense kernel in memory); for the largest grids."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    off, cells, lum = _flatten_sources(sources)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    J = np.zeros(len(targets))
    a = _atten(at)
    rc = lib().or_field_direct_ondemand(n, L, K, _dptr(radii), m, C.byref(a), _iptr(off),
                                        _iptr(cells), _dptr(lum), len(targets),
                                        _iptr(targets), _dptr(J))
    assert rc == 0
    return J


def field_direct_support(n: int, L: float, radii, m: int, bands, sources,
                         targets: np.ndarray) -> np.ndarray:
    """Route D written over the kernel's support: for each slice, the kernel
    values at every displacement that can meet the slice's shell (from the
    definition), times the slice's deposited sources. All bands at once;
    returns [band, target]. Needs an outer radius below half the box minus
    two cell diagonals (one periodic image)."""
    radii = np.ascontiguousarray(radii, dtype=np.float64)
    K = len(radii) - 1
    off, cells, lum = _flatten_sources(sources)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    nb = len(bands)
    arr = (_Atten * nb)(*[_atten(b) for b in bands])
    J = np.zeros((nb, len(targets)))
    rc = lib().or_field_direct_support(n, L, K, _dptr(radii), m, nb, arr, _iptr(off), _iptr(cells),
                                       _dptr(lum), len(targets), _iptr(targets), _dptr(J))
    if rc == -2:
        raise ValueError("outer radius too large for the single-image support route")
    assert rc == 0, rc
    return J


# --- DFTs -------------------------------------------------------------------------

def dft3(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Naive separable 3D DFT (unnormalised), sign -1 forward, +1 inverse."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    n = a.shape[0]
    assert a.shape == (n, n, n)
    lib().or_dft3_naive(n, int(sign), a.ctypes.data)
    return a


def dft3_brute(x: np.ndarray, sign: int = -1) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128)
    n = a.shape[0]
    out = np.zeros_like(a)
    lib().or_dft3_brute(n, int(sign), a.ctypes.data, out.ctypes.data)
    return out


def conv3_brute(G: np.ndarray, S: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = G.shape[0]
    out = np.zeros_like(S)
    lib().or_conv3_brute(n, _dptr(G), _dptr(S), _dptr(out))
    return out


# --- route F ------------------------------------------------------------------------

def field_dft(G: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Full field by Eqs. 12-13 with naive DFTs: J = IDFT(sum_k G^_k S^_k)/N^3."""
    K, n = G.shape[0], G.shape[1]
    A = np.zeros((n, n, n), dtype=np.complex128)
    for k in range(K):
        A += dft3(G[k]) * dft3(S[k])
    return (dft3(A, +1) / float(n) ** 3).real


def field_per_slice_inverse(G: np.ndarray, S: np.ndarray) -> np.ndarray:
    """The paper's order of steps 5-6: inverse transform per slice, then sum."""
    K, n = G.shape[0], G.shape[1]
    J = np.zeros((n, n, n))
    for k in range(K):
        J += (dft3(dft3(G[k]) * dft3(S[k]), +1) / float(n) ** 3).real
    return J


def field_fft(G_of_k, S_of_k, K: int, n: int, workers: int = -1) -> np.ndarray:
    """Route F with scipy.fft (FP64 library FFT) as the transform step.
    G_of_k(k) and S_of_k(k) return the dense FP64 grids of slice k."""
    import scipy.fft as sfft
    A = None
    for k in range(K):
        Sk = S_of_k(k)
        if not np.any(Sk):
            continue
        prod = sfft.rfftn(G_of_k(k), workers=workers) * sfft.rfftn(Sk, workers=workers)
        A = prod if A is None else A + prod
    if A is None:
        return np.zeros((n, n, n))
    return sfft.irfftn(A, s=(n, n, n), workers=workers)


# --- closed forms used by the checks ---------------------------------------------------

def mean_field(G: np.ndarray, S: np.ndarray) -> float:
    """mean(J) = sum_k (sum_c G_k)(sum_c S_k) / N^3 (DC bin of Eq. 13)."""
    n = G.shape[1]
    return float(sum(G[k].sum() * S[k].sum() for k in range(G.shape[0]))) / n ** 3


def workload_field_direct(box, targets, band: int = 0, dense_G=None) -> np.ndarray:
    """Route D for an lc_inputs.Box at the given targets."""
    if dense_G is None and box.n <= 128:
        dense_G = build_G(box.n, box.box, box.radii, box.supersample, box.bands[band],
                          box.conserve)
    if dense_G is not None:
        return field_direct(dense_G, box.sources, targets)
    return field_direct_ondemand(box.n, box.box, box.radii, box.supersample,
                                 box.bands[band], box.sources, targets)


def rel_errors(J: np.ndarray, J_ref: np.ndarray):
    """Normwise relative errors: (max|J-J*|/max|J*|, ||J-J*||_2/||J*||_2)."""
    J = np.asarray(J, dtype=np.float64).ravel()
    R = np.asarray(J_ref, dtype=np.float64).ravel()
    d = J - R
    e_max = float(np.max(np.abs(d)) / np.max(np.abs(R)))
    e_rms = float(np.linalg.norm(d) / np.linalg.norm(R))
    return e_max, e_rms
