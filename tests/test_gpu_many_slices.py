"""Many lookback slices: more than one forward launch's worth, up to the
largest K a box accepts (1024).

The slice count of algorithm step 1 is not tied to the grid. Forward passes
take at most 64 slices per launch, so K = 150 runs three launches per step
and K = 1024 sixteen; the slice sum runs over all K in one fused pass. Thin
shells (r_0 > 0, so no shell holds the source's own cell) leave many slices
with an all-zero kernel, which the sum must skip exactly. Both forms, whole
steps (lc_step, graph-replayed) and per-slice pushes, against route D on
the full grid: FP64 e_max <= 1e-12, FP32 e_rms <= 1e-5 and e_max <= 1e-4.
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


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("n,K,m", [(24, 150, 2), (8, 1024, 4)])
def test_many_slices_match_oracle(n, K, m, form):
    lc = _lc()
    L = 0.78125 * n
    radii = np.linspace(0.5, 0.45 * L, K + 1)
    srcs = [li.random_sources([71, n, k], n, 3) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=m, bands=[li.lw_band(0.3 * L)], sources=srcs)
    G = oracle.build_G(n, L, radii, m, box.bands[0])
    empty = int(np.sum(~np.any(G.reshape(K, -1), axis=1)))
    print(f"case many slices n={n} K={K} m={m} {form}: {empty} slices with an all-zero kernel", flush=True)
    Jr = oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape((n,) * 3)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    dt = np.float64 if form == "fp64" else np.float32
    grids = [torch.from_numpy(li.dense_grid(n, c, v, dt)).cuda() for c, v in srcs]

    def check(J, what):
        e_max, e_rms = oracle.rel_errors(J, Jr)
        print(f"  {what}: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        if form == "fp64":
            assert e_max <= 1e-12
        else:
            assert e_rms <= 1e-5 and e_max <= 1e-4

    plan = lc.Plan([box], precision=prec, use_graph=True)
    plan.build_all()
    out = [torch.empty((n,) * 3, dtype=torch.float64, device="cuda")]
    for rep in range(2):          # capture, then replay
        keep = plan.step(grids, out)
        torch.cuda.synchronize()
        check(out[0].cpu().numpy(), f"lc_step {'capture' if rep == 0 else 'replay'}")
    keep = [plan.push_grid(0, k, g) for k, g in enumerate(grids)]
    check(plan.field(0, 0, dtype=torch.float64).cpu().numpy(), "per-slice pushes + lc_field")
    plan.close()
    del keep
