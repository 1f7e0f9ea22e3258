"""A single unit source: the field is the kernel itself.

With one unit source at cell c0 in lookback slice k and no other sources,
Eq. 11 gives J(x) = G_k(x - c0): the delayed, periodically summed shell of
slice k with its 1/(4 pi r^2) falloff and radial factor (Sec. 2.2, algorithm
step 2). Every slice is checked in turn against the oracle's dense kernel
shifted to c0, at every cell, so the builder (steps 2-3), the transforms and
the slice sum are all pinned to the kernel's definition. Cases: the m^3
subpoint average with two bands (phi = 1 and a Lyman-Werner factor), and
the exact cell average (rule 1). Tolerances: FP64 e_max <= 1e-12, FP32
e_rms <= 1e-5 and e_max <= 1e-4 (normwise).
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


CASES = {
    "subpoints_32": dict(n=32, K=6, m=2, rule=0, bands=("flat", "lw")),
    "subpoints_48": dict(n=48, K=4, m=3, rule=0, bands=("flat",)),
    "exact_16": dict(n=16, K=3, m=1, rule=1, bands=("flat", "lw")),
}


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_unit_source_gives_the_kernel(case, form):
    lc = _lc()
    cfg = CASES[case]
    n, K = cfg["n"], cfg["K"]
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.45 * L, K + 1)
    ats = [li.Atten(kind=0) if b == "flat" else li.lw_band(0.35 * L) for b in cfg["bands"]]
    box = li.Box(n=n, box=L, radii=radii, supersample=cfg["m"], bands=ats, sources=[], rule=cfg["rule"])
    if cfg["rule"] == 1:
        Gs = [oracle.build_G_exact(n, L, radii, at) for at in ats]
    else:
        Gs = [oracle.build_G(n, L, radii, cfg["m"], at) for at in ats]
    c0 = (3, n - 5, 7)
    cell = np.array([(c0[0] * n + c0[1]) * n + c0[2]], dtype=np.int64)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    plan = lc.Plan([box], precision=prec)
    plan.build_all()
    none_c = torch.zeros(0, dtype=torch.int64, device="cuda")
    none_v = torch.zeros(0, dtype=torch.float64, device="cuda")
    one_c = torch.from_numpy(cell).cuda()
    one_v = torch.ones(1, dtype=torch.float64, device="cuda")
    for k in range(K):
        print(f"case unit source {case} {form} slice={k}", flush=True)
        keep = [plan.push_points(0, j, one_c if j == k else none_c, one_v if j == k else none_v) for j in range(K)]
        for b, G in enumerate(Gs):
            J = plan.field(0, b, dtype=torch.float64).cpu().numpy()
            ref = np.roll(G[k], shift=c0, axis=(0, 1, 2))
            if not np.any(ref):
                assert not np.any(J)
                continue
            e_max, e_rms = oracle.rel_errors(J, ref)
            print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
            if form == "fp64":
                assert e_max <= 1e-12
            else:
                assert e_rms <= 1e-5 and e_max <= 1e-4
        del keep
    plan.close()
