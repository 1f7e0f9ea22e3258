"""The paper's order against the path's order of the slice sum.

Algorithm steps 5-6 of Sec. 2.2 invert each slice's product and then sum
the slices; the path sums the products in spectral space and inverts once
per band (Eq. 13 is linear in the slices). Here the field of all K slices
is compared with the sum, in FP64, of the K fields that each hold one slice
alone (the other slices zero): equal up to rounding. FP64 form e_max <=
1e-13; FP32 forms e_rms <= 1e-6 (one field against K fields of FP32
rounding each). Cases: 48^3 x 6 slices x 2 bands in all three forms, and
the benchmark's 256^3 x 40 plan (autotuned, graph-replayed lc_step).
"""
import numpy as np
import pytest

import lc_inputs as li
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lc():
    import paper_1502_02294_amd as lc
    return lc


def _fields_by_slice(lc, box, precision, grids, autotune, use_graph):
    """The full field and the per-slice fields (one slice pushed, the others
    zero), every band, through lc_step; FP64 outputs on the device."""
    plan = lc.Plan([box], precision=precision, use_graph=use_graph, autotune=autotune)
    plan.build_all()
    B = len(box.bands)
    n = box.n
    outs = [torch.empty((n,) * 3, dtype=torch.float64, device="cuda") for _ in range(B)]
    zero = torch.zeros_like(grids[0])
    keep = plan.step(grids, outs)
    torch.cuda.synchronize()
    full = [o.clone() for o in outs]
    acc = [torch.zeros_like(o) for o in outs]
    for k in range(len(grids)):
        only = [grids[j] if j == k else zero for j in range(len(grids))]
        keep = plan.step(only, outs)
        torch.cuda.synchronize()
        for b in range(B):
            acc[b] += outs[b]
    del keep
    plan.close()
    return full, acc


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp32_plain"])
def test_sum_then_invert_equals_invert_then_sum_48(form):
    lc = _lc()
    n, K = 48, 6
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.45 * L, K + 1)
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.Atten(kind=0), li.lw_band(0.3 * L)],
                 sources=[li.random_sources([61, k], n, 300) for k in range(K)])
    prec = {"fp64": lc.LC_PREC_FP64, "fp32": lc.LC_PREC_FP32, "fp32_plain": lc.LC_PREC_FP32_PLAIN}[form]
    dt = np.float64 if form == "fp64" else np.float32
    grids = [torch.from_numpy(li.dense_grid(n, c, v, dt)).cuda() for c, v in box.sources]
    print(f"case slice order n={n} K={K} bands=2 {form}", flush=True)
    full, acc = _fields_by_slice(lc, box, prec, grids, autotune=False, use_graph=False)
    for b in range(2):
        e_max, e_rms = oracle.rel_errors(acc[b].cpu().numpy(), full[b].cpu().numpy())
        print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        if form == "fp64":
            assert e_max <= 1e-13
        else:
            assert e_rms <= 1e-6


def test_sum_then_invert_equals_invert_then_sum_benchmark_plan():
    lc = _lc()
    box = li.points_256c_40s().boxes[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(256)
    # zero-mean grids, so that the FP32 part of the field (not the FP64 mean) is compared
    grids = [torch.randn(box.n ** 3, device="cuda", generator=gen) for _ in range(box.n_slices)]
    print("case slice order 256^3 x 40, the benchmark's plan", flush=True)
    full, acc = _fields_by_slice(lc, box, lc.LC_PREC_FP32, grids, autotune=True, use_graph=True)
    e_max, e_rms = oracle.rel_errors(acc[0].cpu().numpy(), full[0].cpu().numpy())
    print(f"  e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
    assert e_rms <= 1e-6
