"""C-ABI conventions, checked without a GPU: the library loads, exports every
function include/lc.h declares, validates descriptors before any device
call, and reports LC_EDEVICE when no gfx950 device is present."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lc.h")


def _lc():
    import paper_1502_02294_amd as lc
    return lc


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(lc_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lc = _lc()
    lib = lc.load()
    names = header_functions()
    assert "lc_plan" in names and "lc_field" in names and len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in lc.h but not exported"
    assert set(names) == set(lc.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", lc.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lc_\w+)", out))
    assert set(names) <= exported


def _desc(n=32, box=20.0, K=4, m=1, radii=None, prec=0, ws=0, wsb=0, bands=1, **kw):
    lc = _lc()
    r = radii if radii is not None else [box * 0.9 * k / K for k in range(K + 1)]
    d, keep = lc.make_box_desc(n, box, r, bands, m, kw.get("conserve", 0))
    for f in ("rule",):
        if f in kw:
            setattr(d, f, kw[f])
    pd, arr = lc.make_plan_desc([d], prec, 0, ws, wsb, kw.get("use_graph", 0), kw.get("autotune", 0))
    return pd, (keep, arr)


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _plan_status(pd):
    lc = _lc()
    h = C.c_void_p()
    rc = lc.load().lc_plan(C.byref(pd), C.byref(h))
    return rc, lc.lc_last_error()


def test_workspace_bytes_scales_with_problem():
    lc = _lc()
    a, _ = _desc(n=32, K=4)
    b, _ = _desc(n=32, K=8)
    c, _ = _desc(n=64, K=4)
    wa, wb, wc = (lc.lc_workspace_bytes(x) for x in (a, b, c))
    assert 0 < wa < wb and wa < wc
    f32, _ = _desc(n=32, K=4, prec=lc.LC_PREC_FP32)
    assert lc.lc_workspace_bytes(f32) > 0


@pytest.mark.parametrize("case,code", [
    (dict(n=10), "LC_EUNSUPPORTED"),            # not 2^a 3^b
    (dict(n=20), "LC_EUNSUPPORTED"),            # factor 5
    (dict(n=6), "LC_EUNSUPPORTED"),             # below 8
    (dict(n=2048), "LC_EUNSUPPORTED"),          # above 1024
    (dict(n=768), "LC_EUNSUPPORTED"),           # 2^8 3, above the compiled 512
    (dict(m=9), "LC_EUNSUPPORTED"),
    (dict(radii=[0.0, 0.1, 5.0]), "LC_EUNSUPPORTED"),  # self cell straddles slices
    (dict(radii=[0.0, 5.0, 5.0]), "LC_EINVAL"),        # not strictly increasing
    (dict(radii=[-1.0, 5.0, 6.0]), "LC_EINVAL"),       # r_0 < 0
    (dict(radii=[0.0, 5.0, float("nan")]), "LC_EINVAL"),
    (dict(box=-1.0), "LC_EINVAL"),
    (dict(prec=7), "LC_EINVAL"),
    (dict(rule=3), "LC_EINVAL"),
    (dict(autotune=2), "LC_EINVAL"),
])
def test_invalid_descriptors_rejected_before_device(case, code):
    lc = _lc()
    pd, keep = _desc(**case)
    assert lc.lc_workspace_bytes(pd) == 0
    pd2, keep2 = _desc(ws=256 * 4096, wsb=1 << 40, **case)
    rc, msg = _plan_status(pd2)
    assert lc.STATUS_NAMES[rc] == code, msg
    assert msg and msg != "no error"


def test_exact_rule_accepts_a_source_cell_split_between_shells():
    """r_1 < (sqrt 3 / 2) l splits the source's own cell between slices 0
    and 1: rejected for the subpoint rule, accepted for the exact cell
    average (rule 1), which integrates each shell's part of the cell."""
    lc = _lc()
    radii = [0.0, 0.1, 5.0]
    pd0, k0 = _desc(radii=radii)
    assert lc.lc_workspace_bytes(pd0) == 0
    pd1, k1 = _desc(radii=radii, rule=1)
    need = lc.lc_workspace_bytes(pd1)
    assert need > 0
    if _has_gpu():
        pytest.skip("the descriptor's workspace address is a placeholder, not device memory")
    pd2, k2 = _desc(radii=radii, rule=1, ws=256 * 4096, wsb=need)
    rc, msg = _plan_status(pd2)
    assert rc == lc.LC_EDEVICE, msg


def test_workspace_checks_then_device():
    lc = _lc()
    pd, keep = _desc()
    need = lc.lc_workspace_bytes(pd)
    small, k2 = _desc(ws=256 * 4096, wsb=need - 1)
    rc, msg = _plan_status(small)
    assert rc == lc.LC_ENOMEM, msg
    misaligned, k3 = _desc(ws=256 * 4096 + 8, wsb=need)
    rc, msg = _plan_status(misaligned)
    assert rc == lc.LC_ENOMEM, msg
    null_ws, k4 = _desc(ws=0, wsb=need)
    rc, msg = _plan_status(null_ws)
    assert rc == lc.LC_EINVAL, msg
    if not _has_gpu():
        # (only without a device: the workspace address is a placeholder)
        ok, k5 = _desc(ws=256 * 4096, wsb=need)
        rc, msg = _plan_status(ok)
        assert rc == lc.LC_EDEVICE, msg


def test_null_handles_and_last_error():
    lc = _lc()
    L = lc.load()
    assert L.lc_build_greens(None, 0, 0, None) == lc.LC_EINVAL
    assert "NULL" in lc.lc_last_error()
    assert L.lc_push_sources(None, 0, 0, None) == lc.LC_EINVAL
    assert L.lc_field(None, 0, 0, None, 0, 0) == lc.LC_EINVAL
    assert L.lc_step(None, None, None, 0) == lc.LC_EINVAL
    assert L.lc_time_kernel(None, 0, 0, 1, None) == lc.LC_EINVAL
    assert L.lc_get_schedule(None, 0, None) == lc.LC_EINVAL
    assert L.lc_advance(None, 0, None) == lc.LC_EINVAL
    assert L.lc_check_sources(None, 0, None) == lc.LC_EINVAL
    assert L.lc_set_schedule(None, 0, None) == lc.LC_EINVAL
    L.lc_destroy(None)          # no-op


def test_struct_layouts_match_header():
    """Field offsets of the Python mirrors equal a C compilation of lc.h."""
    lc = _lc()
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "lc.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(lc_box_desc), offsetof(lc_box_desc, box), offsetof(lc_box_desc, radii), offsetof(lc_box_desc, rule));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(lc_plan_desc), offsetof(lc_plan_desc, hip_stream), offsetof(lc_plan_desc, workspace_bytes), offsetof(lc_plan_desc, use_graph), offsetof(lc_plan_desc, boxes), offsetof(lc_plan_desc, autotune));
  printf("%zu %zu %zu %zu %zu\n", sizeof(lc_schedule), offsetof(lc_schedule, push_group), offsetof(lc_schedule, n_fused), offsetof(lc_schedule, n_fused_bands), offsetof(lc_schedule, spectra_3d));
  printf("%zu %zu %zu\n", sizeof(lc_atten), offsetof(lc_atten, a), offsetof(lc_atten, prefactor));
  printf("%zu %zu %zu %zu\n", sizeof(lc_sources), offsetof(lc_sources, grid), offsetof(lc_sources, n), offsetof(lc_sources, lum));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        cfile = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(cfile, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), cfile, "-o", exe])
        out = subprocess.check_output([exe], text=True).split("\n")
    b = list(map(int, out[0].split()))
    assert b == [C.sizeof(lc.lc_box_desc), lc.lc_box_desc.box.offset, lc.lc_box_desc.radii.offset,
                 lc.lc_box_desc.rule.offset]
    p = list(map(int, out[1].split()))
    assert p == [C.sizeof(lc.lc_plan_desc), lc.lc_plan_desc.hip_stream.offset,
                 lc.lc_plan_desc.workspace_bytes.offset, lc.lc_plan_desc.use_graph.offset,
                 lc.lc_plan_desc.boxes.offset, lc.lc_plan_desc.autotune.offset]
    sc = list(map(int, out[2].split()))
    assert sc == [C.sizeof(lc.lc_schedule), lc.lc_schedule.push_group.offset, lc.lc_schedule.n_fused.offset,
                  lc.lc_schedule.n_fused_bands.offset, lc.lc_schedule.spectra_3d.offset]
    a = list(map(int, out[3].split()))
    assert a == [C.sizeof(lc.lc_atten), lc.lc_atten.a.offset, lc.lc_atten.prefactor.offset]
    s = list(map(int, out[4].split()))
    assert s == [C.sizeof(lc.lc_sources), lc.lc_sources.grid.offset, lc.lc_sources.n.offset,
                 lc.lc_sources.lum.offset]


def test_plain_c_caller_builds_against_the_header(tmp_path):
    """tests/c_abi_example.c (the GPU test's C caller) compiles as C11 with
    gcc against include/lc.h and links against the built liblc.so."""
    from test_gpu_c_abi import build_example
    exe = build_example(str(tmp_path))
    assert os.path.exists(exe)
