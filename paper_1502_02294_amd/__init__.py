"""Python binding of the light-cone field library (include/lc.h).

Argument marshalling only: every step of the computation runs in the HIP
library liblc.so (built in-tree for gfx950). PyTorch supplies device
memory (the workspace and the buffers) and the HIP stream. There is no CPU
path: if the library is missing, loading fails with an error.

The C entry points are exposed under their own names (lc_plan,
lc_build_greens, lc_push_sources, lc_advance, lc_field, lc_step,
lc_check_sources, lc_destroy, lc_last_error, lc_workspace_bytes); `Plan`
wraps them for torch tensors and checks every tensor (device, dtype, size,
layout) before its address is handed to the library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblc.so")

LC_OK, LC_EINVAL, LC_ENOMEM, LC_EDEVICE, LC_ESTATE, LC_EUNSUPPORTED, LC_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
LC_PREC_FP64, LC_PREC_FP32_PLAIN, LC_PREC_FP32 = 0, 1, 2
LC_F32, LC_F64 = 0, 1
LC_MEM_HOST, LC_MEM_DEVICE = 0, 1

STATUS_NAMES = {0: "LC_OK", -1: "LC_EINVAL", -2: "LC_ENOMEM", -3: "LC_EDEVICE", -4: "LC_ESTATE",
                -5: "LC_EUNSUPPORTED", -6: "LC_ENONFINITE"}

EXPORTED = ["lc_workspace_bytes", "lc_plan", "lc_build_greens", "lc_push_sources", "lc_advance",
            "lc_field", "lc_step", "lc_check_sources", "lc_destroy", "lc_last_error",
            "lc_greens_imag_ratio", "lc_greens_dc", "lc_time_kernel", "lc_get_schedule",
            "lc_set_schedule", "lc_step_static", "lc_field_frozen", "lc_fdiff", "lc_cosmo_slices",
            "lc_lw_factors", "lc_build_greens_slices", "lc_near_field"]

(LC_KERNEL_X_FWD, LC_KERNEL_COL_Y_FWD, LC_KERNEL_COL_Z_FWD, LC_KERNEL_FUSED_Z, LC_KERNEL_MAC,
 LC_KERNEL_COL_Z_INV, LC_KERNEL_COL_Y_INV, LC_KERNEL_X_INV, LC_KERNEL_XY_FWD, LC_KERNEL_YX_INV) = range(10)


class lc_box_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_slices", C.c_int32), ("n_bands", C.c_int32),
                ("supersample", C.c_int32), ("conserve", C.c_int32), ("rule", C.c_int32),
                ("box", C.c_double), ("radii", C.POINTER(C.c_double))]


class lc_plan_desc(C.Structure):
    _fields_ = [("n_boxes", C.c_int32), ("precision", C.c_int32),
                ("boxes", C.POINTER(lc_box_desc)), ("hip_stream", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("use_graph", C.c_int32), ("autotune", C.c_int32)]


class lc_schedule(C.Structure):
    _fields_ = [("xy_variant", C.c_int32), ("fused_variant", C.c_int32), ("fused_rounds", C.c_int32),
                ("push_group", C.c_int32), ("n_xy", C.c_int32), ("n_fused", C.c_int32),
                ("fused_bands", C.c_int32), ("n_fused_bands", C.c_int32), ("spectra_3d", C.c_int32)]


class lc_atten(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("a", C.c_double),
                ("s", C.c_double), ("p", C.c_double), ("c", C.c_double), ("cut", C.c_double),
                ("prefactor", C.c_double)]


class lc_cosmo(C.Structure):
    _fields_ = [("h", C.c_double), ("omega_m", C.c_double)]


class lc_sources(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("mem", C.c_int32),
                ("reserved", C.c_int32), ("grid", C.c_void_p), ("n", C.c_int64),
                ("cell", C.c_void_p), ("lum", C.c_void_p)]


class Positioned:
    """Sources with positions inside their cells (lc_sources kind 2): pos an
    (n, 3) float64 tensor in length units (axis order i, j, k), lum (n,)
    float32/float64. Deposited to the nearest node; the same list feeds
    Plan.near_field."""

    def __init__(self, pos, lum):
        self.pos, self.lum = pos, lum


class LCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load liblc.so. torch is imported first so that the library binds to
    the same HIP runtime (same soname) as torch's device memory and streams."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime shared with torch)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    L.lc_workspace_bytes.argtypes = [C.POINTER(lc_plan_desc)]
    L.lc_workspace_bytes.restype = C.c_size_t
    L.lc_plan.argtypes = [C.POINTER(lc_plan_desc), C.POINTER(C.c_void_p)]
    L.lc_build_greens.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(lc_atten)]
    L.lc_push_sources.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(lc_sources)]
    L.lc_advance.argtypes = [C.c_void_p, C.c_int32, C.POINTER(lc_sources)]
    L.lc_check_sources.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    L.lc_field.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.c_int32]
    L.lc_step.argtypes = [C.c_void_p, C.POINTER(lc_sources), C.POINTER(C.c_void_p), C.c_int32]
    L.lc_step_static.argtypes = [C.POINTER(lc_plan_desc), C.POINTER(lc_atten), C.POINTER(lc_sources),
                                 C.POINTER(C.c_void_p), C.c_int32]
    L.lc_field_frozen.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p),
                                  C.c_int32, C.c_int32]
    L.lc_fdiff.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    dp = C.POINTER(C.c_double)
    L.lc_cosmo_slices.argtypes = [C.POINTER(lc_cosmo), C.c_double, C.c_double, C.c_int32, dp, dp, dp]
    L.lc_lw_factors.argtypes = [C.POINTER(lc_cosmo), C.c_double, C.c_int32, dp, C.c_int32, C.POINTER(lc_atten)]
    L.lc_build_greens_slices.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(lc_atten)]
    L.lc_near_field.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(lc_sources), C.c_int32, C.c_void_p,
                                C.c_int32]
    L.lc_destroy.argtypes = [C.c_void_p]
    L.lc_destroy.restype = None
    L.lc_last_error.restype = C.c_char_p
    L.lc_greens_imag_ratio.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.lc_greens_dc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.lc_time_kernel.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]
    L.lc_get_schedule.argtypes = [C.c_void_p, C.c_int32, C.POINTER(lc_schedule)]
    L.lc_set_schedule.argtypes = [C.c_void_p, C.c_int32, C.POINTER(lc_schedule)]
    for name in ["lc_plan", "lc_build_greens", "lc_push_sources", "lc_advance", "lc_field", "lc_step",
                 "lc_check_sources", "lc_greens_imag_ratio", "lc_greens_dc", "lc_time_kernel",
                 "lc_get_schedule", "lc_set_schedule", "lc_step_static", "lc_field_frozen", "lc_fdiff",
                 "lc_cosmo_slices", "lc_lw_factors", "lc_build_greens_slices", "lc_near_field"]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def lc_last_error() -> str:
    return load().lc_last_error().decode()


def _check(rc: int):
    if rc != LC_OK:
        raise LCError(rc, lc_last_error())


# ---- descriptor helpers -------------------------------------------------------------

def make_box_desc(n: int, box: float, radii, n_bands: int = 1, supersample: int = 1,
                  conserve: int = 0, rule: int = 0):
    """Returns (desc, keepalive) with radii held in a ctypes double array."""
    r = (C.c_double * len(radii))(*[float(v) for v in radii])
    d = lc_box_desc(int(n), len(radii) - 1, int(n_bands), int(supersample), int(conserve), int(rule),
                    float(box), C.cast(r, C.POINTER(C.c_double)))
    return d, r


def make_plan_desc(boxes: Sequence[lc_box_desc], precision: int, stream: int = 0,
                   workspace: int = 0, workspace_bytes: int = 0, use_graph: int = 0, autotune: int = 0):
    arr = (lc_box_desc * len(boxes))(*boxes)
    d = lc_plan_desc(len(boxes), int(precision), C.cast(arr, C.POINTER(lc_box_desc)),
                     C.c_void_p(stream or None), C.c_void_p(workspace or None), int(workspace_bytes),
                     int(use_graph), int(autotune))
    return d, arr


def make_atten(at) -> lc_atten:
    """From any object with kind, a, s, p, c, cut, prefactor attributes."""
    return lc_atten(int(at.kind), 0, float(at.a), float(at.s), float(at.p), float(at.c),
                    float(getattr(at, "cut", 0.0)), float(getattr(at, "prefactor", 1.0)))


# ---- thin wrappers with the C names ---------------------------------------------------

def lc_workspace_bytes(desc: lc_plan_desc) -> int:
    return int(load().lc_workspace_bytes(C.byref(desc)))


def lc_plan(desc: lc_plan_desc) -> C.c_void_p:
    h = C.c_void_p()
    _check(load().lc_plan(C.byref(desc), C.byref(h)))
    return h


def lc_build_greens(plan, box: int, band: int, atten: lc_atten):
    _check(load().lc_build_greens(plan, box, band, C.byref(atten)))


def lc_push_sources(plan, box: int, slice_: int, src: lc_sources):
    _check(load().lc_push_sources(plan, box, slice_, C.byref(src)))


def lc_advance(plan, box: int, src: lc_sources):
    _check(load().lc_advance(plan, box, C.byref(src)))


def lc_check_sources(plan, box: int = -1) -> int:
    """-1 when no evaluation since the last check saw a non-finite source,
    else raises LCError(LC_ENONFINITE) naming the first flagged lookback slice."""
    v = C.c_int32(-1)
    _check(load().lc_check_sources(plan, box, C.byref(v)))
    return int(v.value)


def lc_field(plan, box: int, band: int, outs: Sequence[int], dtype: int, mem: int):
    arr = (C.c_void_p * len(outs))(*[C.c_void_p(o) for o in outs])
    _check(load().lc_field(plan, box, band, arr, dtype, mem))


def lc_step(plan, srcs: Sequence[lc_sources], outs: Sequence[int], dtype: int):
    sarr = (lc_sources * len(srcs))(*srcs)
    oarr = (C.c_void_p * len(outs))(*[C.c_void_p(o) for o in outs])
    _check(load().lc_step(plan, sarr, oarr, dtype))


def lc_step_static(desc: lc_plan_desc, attens: Sequence[lc_atten], srcs: Sequence[lc_sources],
                   outs: Sequence[int], dtype: int):
    """One whole step of one box with no caller workspace and no allocation
    (static device scratch; synchronises desc.hip_stream)."""
    aarr = (lc_atten * len(attens))(*attens)
    sarr = (lc_sources * len(srcs))(*srcs)
    oarr = (C.c_void_p * len(outs))(*[C.c_void_p(o) for o in outs])
    _check(load().lc_step_static(C.byref(desc), aarr, sarr, oarr, dtype))


LC_STATIC_SCRATCH_BYTES = 128 * 1024 * 1024


def lc_cosmo_slices(h: float, omega_m: float, z_obs: float, dt_myr: float, K: int):
    """Lookback slicing by cosmic time (host only): (radii[K+1] comoving Mpc,
    z_edge[K+1], z_src[K]) as numpy arrays."""
    import numpy as np
    c = lc_cosmo(float(h), float(omega_m))
    r = (C.c_double * (K + 1))()
    ze = (C.c_double * (K + 1))()
    zs = (C.c_double * K)()
    _check(load().lc_cosmo_slices(C.byref(c), float(z_obs), float(dt_myr), int(K), r, ze, zs))
    return np.array(r[:]), np.array(ze[:]), np.array(zs[:])


def lc_lw_factors(h: float, omega_m: float, z_obs: float, z_src, kind: int = 2):
    """Per-slice Lyman-Werner radial factors (host only): list of lc_atten."""
    K = len(z_src)
    c = lc_cosmo(float(h), float(omega_m))
    zs = (C.c_double * K)(*[float(v) for v in z_src])
    out = (lc_atten * K)()
    _check(load().lc_lw_factors(C.byref(c), float(z_obs), K, zs, int(kind), out))
    return [out[k] for k in range(K)]


def fdiff(j, j_inst, out=None):
    """(j_inst - j) / j elementwise on the device (lc_fdiff; 0 where j == 0)."""
    import torch
    if j.shape != j_inst.shape or j.dtype != j_inst.dtype:
        raise ValueError("fdiff: fields of one shape and dtype required")
    a = check_tensor(j, "j", dtypes=(torch.float32, torch.float64), device=j.device)
    b = check_tensor(j_inst, "j_inst", dtypes=(torch.float32, torch.float64), numel=a.numel(), device=a.device)
    if not a.is_cuda:
        raise ValueError("fdiff: device tensors required")
    if out is None:
        out = torch.empty_like(a)
    out = check_tensor(out, "out", dtypes=(a.dtype,), numel=a.numel(), device=a.device, copy_ok=False)
    st = torch.cuda.current_stream(a.device).cuda_stream
    _check(load().lc_fdiff(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr()),
                           a.numel(), LC_F64 if a.dtype == torch.float64 else LC_F32, C.c_void_p(st)))
    return out


def lc_destroy(plan):
    load().lc_destroy(plan)


# ---- tensor checks ----------------------------------------------------------------------

def _same_device(t, device) -> bool:
    if t.device.type != device.type:
        return False
    return device.index is None or t.device.index == device.index


def check_tensor(t, what: str, *, dtypes, numel=None, device=None, allow_host: bool = False,
                 copy_ok: bool = True):
    """Check a tensor before its address goes to the library; returns the
    tensor to pass (a contiguous copy when `copy_ok` and `t` is not
    contiguous; the caller keeps it alive until the stream has used it).

    dtypes: allowed torch dtypes; numel: required element count; device:
    the plan's device (CPU tensors pass only with allow_host). Raises
    TypeError for a wrong type or dtype, ValueError for a wrong size,
    device or layout."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor, not {type(t).__name__}")
    if t.dtype not in dtypes:
        names = ", ".join(str(d).replace("torch.", "") for d in dtypes)
        raise TypeError(f"{what} has dtype {str(t.dtype).replace('torch.', '')}; expected one of {names}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements; expected {numel}")
    if device is not None:
        if t.device.type == "cpu":
            if not allow_host and device.type != "cpu":
                raise ValueError(f"{what} is in host memory; expected a tensor on {device}")
        elif not _same_device(t, device):
            raise ValueError(f"{what} is on {t.device}; expected {device}")
    if not t.is_contiguous():
        if not copy_ok:
            raise ValueError(f"{what} must be contiguous (it is written in place)")
        t = t.contiguous()
    return t


# ---- torch-facing convenience ----------------------------------------------------------

class Plan:
    """A plan over one or more boxes, with its workspace in a torch uint8
    tensor on the current device. The library's work runs on a stream of
    the plan's own (default priority; the legacy default stream cannot be
    captured into a graph); every call first makes that stream wait for the
    caller's current stream and makes the current stream wait for it after.

    boxes: sequence of objects with n, box, radii, bands (list), supersample,
    conserve (e.g. lc_inputs.Box).
    """

    def __init__(self, boxes, precision: int = LC_PREC_FP64, use_graph: bool = False, device=None,
                 autotune: bool = False):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.precision = precision
        self.boxes = list(boxes)
        self._keep = []
        descs = []
        for b in self.boxes:
            d, r = make_box_desc(b.n, b.box, b.radii, len(b.bands), b.supersample,
                                 getattr(b, "conserve", 0), getattr(b, "rule", 0))
            descs.append(d)
            self._keep.append(r)
        probe, arr = make_plan_desc(descs, precision)
        self._keep.append(arr)
        nbytes = lc_workspace_bytes(probe)
        if nbytes == 0:
            raise LCError(LC_EINVAL, lc_last_error())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.Stream(device=self.device)
        self._enter()
        desc, arr2 = make_plan_desc(descs, precision, self.stream.cuda_stream, aligned, nbytes,
                                    1 if use_graph else 0, 1 if autotune else 0)
        self._keep.append(arr2)
        self.handle = lc_plan(desc)
        self._leave()

    # Order the plan's stream after torch's current stream on entry, and the
    # current stream after the plan's work on exit. With the plan's stream
    # current (torch.cuda.stream(plan.stream)) both are skipped, so that
    # consecutive calls start without a cross-stream round trip; the caller
    # then orders the plan's stream against its other streams itself.
    def _enter(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _call(self, fn, *args):
        """One library call ordered against torch's current stream (also when
        the call fails: work it enqueued before failing stays ordered)."""
        self._enter()
        try:
            return fn(*args)
        finally:
            self._leave()

    def build_greens(self, box: int = 0, band: int = 0, atten=None):
        at = atten if atten is not None else self.boxes[box].bands[band]
        self._call(lc_build_greens, self.handle, box, band, make_atten(at))

    def build_greens_slices(self, box: int, band: int, attens):
        """One radial factor per slice (lc_build_greens_slices): attens is a
        sequence of K objects with kind, a, s, p, c, cut, prefactor (or
        lc_atten structs)."""
        K = len(self.boxes[box].radii) - 1
        if len(attens) != K:
            raise ValueError(f"build_greens_slices takes {K} radial factors, got {len(attens)}")
        arr = (lc_atten * K)(*[a if isinstance(a, lc_atten) else make_atten(a) for a in attens])
        self._call(lambda: _check(load().lc_build_greens_slices(self.handle, box, band, arr)))

    def build_all(self):
        for bi, b in enumerate(self.boxes):
            for band in range(len(b.bands)):
                self.build_greens(bi, band)

    def _box_n(self, box: int) -> int:
        if not 0 <= box < len(self.boxes):
            raise ValueError(f"box {box} out of range [0, {len(self.boxes)})")
        return self.boxes[box].n

    def _grid_source(self, box: int, grid, allow_host: bool, what: str):
        """lc_sources of a dense grid (and the tensor to keep alive)."""
        torch = self.torch
        n = self._box_n(box)
        t = check_tensor(grid, what, dtypes=(torch.float32, torch.float64), numel=n ** 3,
                         device=self.device, allow_host=allow_host)
        dt = LC_F64 if t.dtype == torch.float64 else LC_F32
        mem = LC_MEM_DEVICE if t.is_cuda else LC_MEM_HOST
        return lc_sources(0, dt, mem, 0, t.data_ptr(), 0, None, None), t

    def _point_source(self, box: int, cells, lum, allow_host: bool, what: str):
        """lc_sources of a point list (and the tensors to keep alive)."""
        torch = self.torch
        self._box_n(box)
        c = check_tensor(cells, what + " cells", dtypes=(torch.int64,), device=self.device,
                         allow_host=allow_host)
        v = check_tensor(lum, what + " luminosities", dtypes=(torch.float32, torch.float64),
                         numel=c.numel(), device=self.device, allow_host=allow_host)
        if c.device != v.device:
            raise ValueError(f"{what}: cells on {c.device} but luminosities on {v.device}")
        dt = LC_F64 if v.dtype == torch.float64 else LC_F32
        mem = LC_MEM_DEVICE if c.is_cuda else LC_MEM_HOST
        src = lc_sources(1, dt, mem, 0, None, int(c.numel()), c.data_ptr() if c.numel() else None,
                         v.data_ptr() if v.numel() else None)
        return src, (c, v)

    def _positioned_source(self, box: int, s, allow_host: bool, what: str):
        torch = self.torch
        self._box_n(box)
        v = check_tensor(s.lum, what + " luminosities", dtypes=(torch.float32, torch.float64),
                         device=self.device, allow_host=allow_host)
        p = check_tensor(s.pos, what + " positions", dtypes=(torch.float64,), numel=3 * v.numel(),
                         device=self.device, allow_host=allow_host)
        if p.device != v.device:
            raise ValueError(f"{what}: positions on {p.device} but luminosities on {v.device}")
        dt = LC_F64 if v.dtype == torch.float64 else LC_F32
        mem = LC_MEM_DEVICE if p.is_cuda else LC_MEM_HOST
        src = lc_sources(2, dt, mem, 0, p.data_ptr() if v.numel() else None, int(v.numel()), None,
                         v.data_ptr() if v.numel() else None)
        return src, (p, v)

    def _source(self, box: int, s, allow_host: bool, what: str):
        if isinstance(s, Positioned):
            return self._positioned_source(box, s, allow_host, what)
        if isinstance(s, (tuple, list)):
            if len(s) != 2:
                raise ValueError(f"{what}: a point list is a (cells, lum) pair")
            return self._point_source(box, s[0], s[1], allow_host, what)
        return self._grid_source(box, s, allow_host, what)

    def push_grid(self, box: int, slice_: int, grid):
        """Dense source grid: a torch tensor (on the plan's device or on the
        host) of N^3 float32/float64 values."""
        src, t = self._grid_source(box, grid, True, "source grid")
        self._call(lc_push_sources, self.handle, box, slice_, src)
        return t  # caller keeps it alive until the stream reaches the call

    def push_points(self, box: int, slice_: int, cells, lum):
        """Point list: int64 cells and float32/float64 luminosities (torch
        tensors on one device, the plan's or the host)."""
        src, keep = self._point_source(box, cells, lum, True, "point list")
        self._call(lc_push_sources, self.handle, box, slice_, src)
        return keep

    def push_positioned(self, box: int, slice_: int, pos, lum):
        """Positioned sources (lc_sources kind 2): (n, 3) float64 positions in
        length units and their luminosities, on the plan's device or the host."""
        src, keep = self._positioned_source(box, Positioned(pos, lum), True, "positioned sources")
        self._call(lc_push_sources, self.handle, box, slice_, src)
        return keep

    def near_field(self, box: int, band: int, positioned, near_cells: int, out):
        """Add the particle-mesh near-field correction (lc_near_field) of the
        K slices' positioned sources (a list of Positioned, lookback order) to
        the field `out` (device tensor of this box and band)."""
        torch = self.torch
        n = self._box_n(box)
        K = len(self.boxes[box].radii) - 1
        if len(positioned) != K:
            raise ValueError(f"near_field takes {K} positioned source lists, got {len(positioned)}")
        srcs, keep = [], []
        for k, s in enumerate(positioned):
            src, kp = self._positioned_source(box, s, False, f"slice {k} positioned sources")
            srcs.append(src)
            keep.append(kp)
        out = check_tensor(out, "field", dtypes=(torch.float32, torch.float64), numel=n ** 3, device=self.device,
                           copy_ok=False)
        arr = (lc_sources * K)(*srcs)
        dt = LC_F64 if out.dtype == torch.float64 else LC_F32
        self._call(lambda: _check(load().lc_near_field(self.handle, box, band, arr, int(near_cells),
                                                       C.c_void_p(out.data_ptr()), dt)))
        return keep

    def advance(self, box: int, sources):
        """Next observing time (lc_advance): `sources` (a dense grid tensor
        or a (cells, lum) pair, device or host) become lookback slice 0 and
        every other slice moves one slot older. Returns the tensors to keep
        alive until the stream has run the call."""
        src, keep = self._source(box, sources, True, "advance sources")
        self._call(lc_advance, self.handle, box, src)
        return keep

    def check_sources(self, box: int = -1) -> None:
        """Raise LCError(LC_ENONFINITE) if an evaluation since the last check
        met a NaN or infinite source (synchronises the plan's stream)."""
        self._call(lc_check_sources, self.handle, box)

    def field(self, box: int = 0, band: int = 0, dtype=None, out=None):
        torch = self.torch
        n = self._box_n(box)
        dtype = dtype or (torch.float64 if self.precision == LC_PREC_FP64 else torch.float32)
        if out is None:
            out = torch.empty((n, n, n), dtype=dtype, device=self.device)
        out = check_tensor(out, "output field", dtypes=(torch.float32, torch.float64), numel=n ** 3,
                           device=self.device, allow_host=True, copy_ok=False)
        dt = LC_F64 if out.dtype == torch.float64 else LC_F32
        mem = LC_MEM_DEVICE if out.is_cuda else LC_MEM_HOST
        self._call(lc_field, self.handle, box, band, [out.data_ptr()], dt, mem)
        return out

    def field_frozen(self, box: int = 0, band: int = 0, slice_: int = 0, dtype=None, out=None):
        """The instantaneous field (lc_field_frozen): every slice uses the
        sources of lookback slice `slice_`."""
        torch = self.torch
        n = self._box_n(box)
        dtype = dtype or (torch.float64 if self.precision == LC_PREC_FP64 else torch.float32)
        if out is None:
            out = torch.empty((n, n, n), dtype=dtype, device=self.device)
        out = check_tensor(out, "output field", dtypes=(torch.float32, torch.float64), numel=n ** 3,
                           device=self.device, allow_host=True, copy_ok=False)
        dt = LC_F64 if out.dtype == torch.float64 else LC_F32
        mem = LC_MEM_DEVICE if out.is_cuda else LC_MEM_HOST
        arr = (C.c_void_p * 1)(C.c_void_p(out.data_ptr()))
        self._call(lambda: _check(load().lc_field_frozen(self.handle, box, band, slice_, arr, dt, mem)))
        return out

    def greens_dc(self, box: int = 0, band: int = 0):
        K = len(self.boxes[box].radii) - 1
        arr = (C.c_double * K)()
        _check(load().lc_greens_dc(self.handle, box, band, arr))
        return list(arr)

    def greens_imag_ratio(self, box: int = 0, band: int = 0) -> float:
        v = C.c_double()
        _check(load().lc_greens_imag_ratio(self.handle, box, band, C.byref(v)))
        return float(v.value)

    def time_kernel(self, kernel: int, box: int = 0, reps: int = 10) -> float:
        """Mean milliseconds per launch of one kernel of the path (HIP events)."""
        v = C.c_double()
        self._call(lambda: _check(load().lc_time_kernel(self.handle, box, kernel, reps, C.byref(v))))
        return float(v.value)

    def get_schedule(self, box: int = 0) -> dict:
        """Launch shapes of one box's tunable passes (lc_get_schedule)."""
        s = lc_schedule()
        _check(load().lc_get_schedule(self.handle, box, C.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in lc_schedule._fields_}

    def set_schedule(self, box: int = 0, **kw):
        """Change some fields of a box's schedule (lc_set_schedule)."""
        cur = self.get_schedule(box)
        cur.update(kw)
        s = lc_schedule(*[int(cur[f]) for f, _ in lc_schedule._fields_])
        self._call(lambda: _check(load().lc_set_schedule(self.handle, box, C.byref(s))))

    def step(self, grids, outs, dtype=None):
        """One whole step (lc_step): push every slice of every box (box-major
        list of device sources: a dense grid tensor, or a point list given as
        a (cells, lum) pair of tensors) and evaluate every band into outs
        (box-major, band; device tensors of one dtype). Returns, per source,
        the tensor (or (cells, lum) pair) handed to the library, contiguous
        copies where needed; they must stay alive until the stream has run
        the step."""
        torch = self.torch
        nsl = [len(b.radii) - 1 for b in self.boxes]
        nbd = [len(b.bands) for b in self.boxes]
        if len(grids) != sum(nsl):
            raise ValueError(f"step takes {sum(nsl)} sources (all slices of all boxes), got {len(grids)}")
        if len(outs) != sum(nbd):
            raise ValueError(f"step takes {sum(nbd)} outputs (all bands of all boxes), got {len(outs)}")
        srcs, keep = [], []
        i = 0
        for bi, K in enumerate(nsl):
            for k in range(K):
                src, kp = self._source(bi, grids[i], False, f"box {bi} slice {k} sources")
                srcs.append(src)
                keep.append(kp)
                i += 1
        odts = {o.dtype for o in outs}
        if len(odts) != 1:
            raise TypeError("step outputs must share one dtype")
        i = 0
        for bi, B in enumerate(nbd):
            for b in range(B):
                check_tensor(outs[i], f"box {bi} band {b} output", dtypes=(torch.float32, torch.float64),
                             numel=self.boxes[bi].n ** 3, device=self.device, copy_ok=False)
                i += 1
        odt = LC_F64 if outs[0].dtype == torch.float64 else LC_F32
        self._call(lc_step, self.handle, srcs, [o.data_ptr() for o in outs], odt)
        return keep

    def close(self):
        """Destroy the plan and drop its workspace (after the plan's stream
        has finished with it)."""
        if getattr(self, "handle", None):
            self.stream.synchronize()
            lc_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
