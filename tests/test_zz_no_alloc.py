"""lc_step_static (the entry point for callers that cannot allocate) against
lc_plan + lc_build_greens + lc_step on the same inputs, through the C ABI:
two calls in a row, the second with a smaller box, then an FP64 call; the
results must be bitwise equal (same kernels and launch shapes, both eager).
Also its size and argument checks."""
import ctypes as C

import numpy as np
import pytest

import lc_inputs as li
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lc():
    import paper_1502_02294_amd as lc
    return lc


def _case(n, L, K, m, bands, seed):
    radii = np.linspace(0.0, 0.8 * L, K + 1)
    srcs = [li.random_sources([seed, k], n, 40 + 5 * k) for k in range(K)]
    return li.Box(n=n, box=L, radii=radii, supersample=m, bands=bands, sources=srcs)


def _static(box, prec, dt):
    """One lc_step_static call through the C ABI; returns the band fields."""
    lc = _lc()
    d, keep_r = lc.make_box_desc(box.n, box.box, box.radii, len(box.bands), box.supersample)
    stream = torch.cuda.current_stream()
    pd, keep_a = lc.make_plan_desc([d], prec, stream.cuda_stream)
    grids = [torch.from_numpy(li.dense_grid(box.n, c, v)).to(dt).cuda() for c, v in box.sources]
    srcs = [lc.lc_sources(0, lc.LC_F64 if dt == torch.float64 else lc.LC_F32, lc.LC_MEM_DEVICE, 0,
                          g.data_ptr(), 0, None, None) for g in grids]
    outs = [torch.full((box.n,) * 3, float("nan"), dtype=dt, device="cuda") for _ in box.bands]
    attens = [lc.make_atten(b) for b in box.bands]
    lc.lc_step_static(pd, attens, srcs, [o.data_ptr() for o in outs],
                      lc.LC_F64 if dt == torch.float64 else lc.LC_F32)
    torch.cuda.synchronize()
    return [o.clone() for o in outs]


def _planned(box, prec, dt):
    """The same step through lc_plan (caller workspace), lc_build_greens and lc_step."""
    lc = _lc()
    plan = lc.Plan([box], precision=prec)
    plan.build_all()
    grids = [torch.from_numpy(li.dense_grid(box.n, c, v)).to(dt).cuda() for c, v in box.sources]
    outs = [torch.empty((box.n,) * 3, dtype=dt, device="cuda") for _ in box.bands]
    plan.step(grids, outs)
    torch.cuda.synchronize()
    plan.close()
    return outs


def test_static_step_equals_planned_step_twice_then_smaller():
    lc = _lc()
    big = _case(64, 50.0, 12, 2, [li.Atten(kind=0), li.lw_band(30.0)], 31)
    small = _case(32, 30.0, 5, 2, [li.lw_band(20.0)], 32)
    for label, box, prec, dt in (("64^3 x 12, 2 bands, FP32", big, lc.LC_PREC_FP32, torch.float32),
                                 ("32^3 x 5, 1 band, FP32", small, lc.LC_PREC_FP32, torch.float32),
                                 ("32^3 x 5, 1 band, FP64", small, lc.LC_PREC_FP64, torch.float64)):
        print(f"case static step {label}", flush=True)
        got = _static(box, prec, dt)
        ref = _planned(box, prec, dt)
        for b, (g, r) in enumerate(zip(got, ref)):
            assert torch.equal(g, r), f"{label} band {b}: max diff {float((g - r).abs().max())}"
    # and the small box against the oracle
    G = oracle.build_G(small.n, small.box, small.radii, small.supersample, small.bands[0])
    Jr = oracle.field_direct(G, small.sources, np.arange(small.n ** 3))
    e_max, _ = oracle.rel_errors(got[0].double().cpu().numpy().ravel(), Jr)
    assert e_max <= 1e-12


def test_static_step_rejections():
    lc = _lc()
    L = lc.load()
    big = li.points_256c_40s().boxes[0]
    d, kr = lc.make_box_desc(big.n, big.box, big.radii, 1, big.supersample)
    pd, ka = lc.make_plan_desc([d], lc.LC_PREC_FP32, 0)
    at = (lc.lc_atten * 1)(lc.make_atten(big.bands[0]))
    src = (lc.lc_sources * big.n_slices)()
    out = (C.c_void_p * 1)(C.c_void_p(16))
    rc = L.lc_step_static(C.byref(pd), at, src, out, lc.LC_F32)
    assert rc == lc.LC_ENOMEM and "static maximum" in lc.lc_last_error()
    assert lc.lc_workspace_bytes(pd) > lc.LC_STATIC_SCRATCH_BYTES
    small = _case(32, 30.0, 5, 2, [li.Atten(kind=0)], 33)
    d, kr = lc.make_box_desc(small.n, small.box, small.radii, 1, 2)
    pd, ka = lc.make_plan_desc([d], lc.LC_PREC_FP32, 0, workspace=4096, workspace_bytes=4096)
    rc = L.lc_step_static(C.byref(pd), at, src, out, lc.LC_F32)
    assert rc == lc.LC_EINVAL and "workspace" in lc.lc_last_error()
    pd, ka = lc.make_plan_desc([d, d], lc.LC_PREC_FP32, 0)
    rc = L.lc_step_static(C.byref(pd), at, src, out, lc.LC_F32)
    assert rc == lc.LC_EINVAL and "one box" in lc.lc_last_error()
