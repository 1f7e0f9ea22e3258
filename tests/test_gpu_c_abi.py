"""The C ABI from a plain C program (tests/c_abi_example.c), with no Python
in the process that calls the library: lc_workspace_bytes, lc_plan,
lc_build_greens, lc_push_sources (host point lists) and lc_field (host
output); then lc_step over dense device grids into device memory, captured
in a HIP graph and replayed. Both fields against the CPU FP64 oracle
(route D, full grid): FP64 form e_max <= 1e-12, FP32 form e_rms <= 1e-5 and
e_max <= 1e-4.
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import lc_inputs as li
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build_example(dst_dir):
    """Compile the C caller with gcc against include/lc.h and the built
    liblc.so (the library itself is not rebuilt here)."""
    exe = os.path.join(dst_dir, "c_abi_example")
    lib = os.path.join(ROOT, "paper_1502_02294_amd", "liblc.so")
    cmd = ["gcc", "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c_abi_example.c"), "-o", exe, lib,
           "-Wl,-rpath," + os.path.dirname(lib), "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def write_input(path, box):
    with open(path, "wb") as f:
        f.write(struct.pack("<iiid", box.n, box.n_slices, box.supersample, box.box))
        f.write(np.asarray(box.radii, dtype="<f8").tobytes())
        for cells, lum in box.sources:
            f.write(struct.pack("<q", len(cells)))
            f.write(np.asarray(cells, dtype="<i8").tobytes())
            f.write(np.asarray(lum, dtype="<f8").tobytes())


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_plain_c_caller_matches_oracle(tmp_path, form):
    import paper_1502_02294_amd as lc
    b0 = li.points_32c_8s().boxes[0]
    box = li.Box(n=b0.n, box=b0.box, radii=b0.radii, supersample=2, bands=b0.bands, sources=b0.sources)
    exe = build_example(str(tmp_path))
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_input(inp, box)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    print(f"case c_abi_example {form} n={box.n} K={box.n_slices} m=2", flush=True)
    r = subprocess.run([exe, inp, out, str(prec)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    n3 = box.n ** 3
    J = np.fromfile(out, dtype="<f8")
    assert J.size == 2 * n3
    G = oracle.build_G(box.n, box.box, box.radii, box.supersample, box.bands[0])
    Jr = oracle.field_direct(G, box.sources, np.arange(n3))
    for what, Jx in (("point lists + lc_field", J[:n3]), ("dense grids + lc_step replay", J[n3:])):
        e_max, e_rms = oracle.rel_errors(Jx, Jr)
        print(f"  {what}: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        if form == "fp64":
            assert e_max <= 1e-12
        else:
            assert e_rms <= 1e-5 and e_max <= 1e-4
