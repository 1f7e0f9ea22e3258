"""The transform passes at every compiled grid size, through the whole path.

With one slice whose shell [0, 0.9 l) holds only the source's own cell (the
node rule, m = 1: the next nodes are a full cell away, the periodic images
N cells away), the kernel is c times a unit impulse, c = G_0(0) the exact
cube average of 1/(4 pi r^2) over the own cell (Sec. 2.2, the shell of
algorithm step 2). Its spectrum is the constant c, so the field of Eq. 13 is
J = IDFT(c DFT(S)) / N^3 = c S: every forward and inverse pass of the path
(x, y, z, the fused passes, the DC mode) must give back the source grid.
The reference c S needs no transform; c comes from the oracle's kernel at
the own cell, and the oracle's kernel at the nearest displacements is
checked to be zero.

Tolerances: FP64 e_max <= 1e-12 (normwise); FP32 forms e_rms <= 1e-6 and
e_max <= 1e-5 (a transform pair in FP32 on random normal data, no slice
sum).
"""
import numpy as np
import pytest

import lc_inputs as li
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512]


def _lc():
    import paper_1502_02294_amd as lc
    return lc


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp32_plain"])
@pytest.mark.parametrize("n", SIZES)
def test_impulse_kernel_returns_the_sources(n, form):
    lc = _lc()
    L = float(n)                       # cell size l = 1
    radii = np.array([0.0, 0.9])
    at = li.Atten(kind=0)
    c = oracle.G_at(n, L, radii, 1, at, (0, 0, 0))[0]
    for d in ((1, 0, 0), (0, 1, 1), (1, 1, 1), (n - 1, 0, 0)):
        assert oracle.G_at(n, L, radii, 1, at, d)[0] == 0.0
    assert c > 0.0
    prec = {"fp64": lc.LC_PREC_FP64, "fp32": lc.LC_PREC_FP32, "fp32_plain": lc.LC_PREC_FP32_PLAIN}[form]
    box = li.Box(n=n, box=L, radii=radii, supersample=1, bands=[at], sources=[])
    print(f"case impulse kernel n={n} {form}", flush=True)
    plan = lc.Plan([box], precision=prec, autotune=(form == "fp32"))
    plan.build_all()
    rng = np.random.default_rng([31, n])
    S = rng.standard_normal(n ** 3)
    if form != "fp64":
        S = S.astype(np.float32)
    g = torch.from_numpy(S).cuda()
    plan.push_grid(0, 0, g)
    J = plan.field(0, 0, dtype=torch.float64).cpu().numpy().ravel()
    plan.close()
    ref = c * S.astype(np.float64)
    e_max, e_rms = oracle.rel_errors(J, ref)
    print(f"  schedule-independent reference c*S: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
    if form == "fp64":
        assert e_max <= 1e-12
    else:
        assert e_rms <= 1e-6 and e_max <= 1e-5
