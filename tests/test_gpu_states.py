"""The call order and the error codes of the C ABI on a device.

lc_plan fixes the boxes (algorithm step 1); every (box, band) kernel must
be built (steps 2-3) before a field (steps 5-6) or a step is asked for:
LC_ESTATE otherwise. Indices out of range give LC_EINVAL before any device
work. A failed call leaves the plan as it was: after the errors, building
the kernels and pushing the sources gives the same field, bit for bit, as a
plan that never saw an error, and that field matches the oracle (route D,
full grid).
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


def _code(fn):
    lc = _lc()
    with pytest.raises(lc.LCError) as ei:
        fn()
    assert str(ei.value)          # the library's message is carried along
    return ei.value.code


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_state_errors_leave_the_plan_usable(form):
    lc = _lc()
    w = li.points_32c_8s()
    b0 = w.boxes[0]
    box = li.Box(n=b0.n, box=b0.box, radii=b0.radii, supersample=1, bands=[li.Atten(kind=0), li.lw_band(12.0)],
                 sources=b0.sources)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    dt = np.float64 if form == "fp64" else np.float32
    n, K = box.n, box.n_slices
    grids = [torch.from_numpy(li.dense_grid(n, c, v, dt)).cuda() for c, v in box.sources]
    outs = [torch.empty((n,) * 3, dtype=torch.float64, device="cuda") for _ in box.bands]
    print(f"case call order and error codes {form}", flush=True)

    p = lc.Plan([box], precision=prec)
    # nothing built: fields and steps are out of order
    assert _code(lambda: p.field(0, 0)) == lc.LC_ESTATE
    assert _code(lambda: p.step(grids, outs)) == lc.LC_ESTATE
    p.build_greens(0, 0)
    # band 1 still missing
    assert _code(lambda: p.field(0, 1)) == lc.LC_ESTATE
    assert _code(lambda: p.step(grids, outs)) == lc.LC_ESTATE
    # indices out of range
    assert _code(lambda: p.build_greens(0, 2, li.Atten(kind=0))) == lc.LC_EINVAL
    assert _code(lambda: p.build_greens(1, 0, li.Atten(kind=0))) == lc.LC_EINVAL
    assert _code(lambda: p.push_grid(0, K, grids[0])) == lc.LC_EINVAL
    assert _code(lambda: p.push_grid(0, -1, grids[0])) == lc.LC_EINVAL
    bad_at = li.Atten(kind=1, a=1.7, s=-1.0, p=0.68, c=0.7)
    assert _code(lambda: p.build_greens(0, 1, bad_at)) == lc.LC_EINVAL
    # now in order
    p.build_greens(0, 1)
    keep = [p.push_grid(0, k, g) for k, g in enumerate(grids)]
    J = [p.field(0, b, dtype=torch.float64).cpu().numpy() for b in range(2)]

    clean = lc.Plan([box], precision=prec)
    clean.build_all()
    keep += [clean.push_grid(0, k, g) for k, g in enumerate(grids)]
    Jc = [clean.field(0, b, dtype=torch.float64).cpu().numpy() for b in range(2)]
    for b in range(2):
        assert np.array_equal(J[b], Jc[b])
        G = oracle.build_G(n, box.box, box.radii, box.supersample, box.bands[b])
        Jr = oracle.field_direct(G, box.sources, np.arange(n ** 3)).reshape(J[b].shape)
        e_max, e_rms = oracle.rel_errors(J[b], Jr)
        print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        assert (e_max <= 1e-12) if form == "fp64" else (e_rms <= 1e-5 and e_max <= 1e-4)
    p.close()
    clean.close()
    del keep
