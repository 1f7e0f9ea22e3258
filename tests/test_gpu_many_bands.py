"""More bands than one fused launch takes.

A box may carry any number B of radial factors (Sec. 3: Lyman-Werner
factors per frequency band share the sources). The fused pass takes at most
two bands per launch at N <= 256 and four at N = 384, 512, so B = 5 at 48^3
runs launches of 2 + 2 + 1 bands (compensated sums) and B = 6 at 384^3
launches of 4 + 2 (plain sums, then compensated). Every band against the
oracle (route D): the full grid at 48^3, 1500 sampled cells at 384^3. Both
forms at 48^3; the FP32 form at 384^3. FP64 e_max <= 1e-12, FP32 e_rms <=
1e-5 and e_max <= 1e-4.
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


def _run(box, prec, dt, targets, refs, form):
    lc = _lc()
    n = box.n
    plan = lc.Plan([box], precision=prec)
    plan.build_all()
    keep = [plan.push_grid(0, k, torch.from_numpy(li.dense_grid(n, c, v, dt)).cuda())
            for k, (c, v) in enumerate(box.sources)]
    for b in range(len(box.bands)):
        J = plan.field(0, b, dtype=torch.float64).cpu().numpy().ravel()[targets]
        e_max, e_rms = oracle.rel_errors(J, refs[b])
        print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        if form == "fp64":
            assert e_max <= 1e-12
        else:
            assert e_rms <= 1e-5 and e_max <= 1e-4
    plan.close()
    del keep


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_five_bands_48(form):
    lc = _lc()
    n, K = 48, 5
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.45 * L, K + 1)
    hz = [0.45, 0.38, 0.3, 0.22, 0.15]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.lw_band(h * L) for h in hz],
                 sources=[li.random_sources([81, k], n, 200) for k in range(K)])
    tg = np.arange(n ** 3)
    refs = [oracle.field_direct(oracle.build_G(n, L, radii, 2, at), box.sources, tg) for at in box.bands]
    print(f"case five bands n={n} {form}", flush=True)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    _run(box, prec, np.float64 if form == "fp64" else np.float32, tg, refs, form)


def test_six_bands_384():
    lc = _lc()
    n, K = 384, 4
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.45 * L, K + 1)
    hz = [0.44, 0.36, 0.28, 0.2, 0.14, 0.1]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.lw_band(h * L) for h in hz],
                 sources=[li.random_sources([83, k], n, 120) for k in range(K)])
    tg = li.sample_cells([85, n], n, 1500)
    refs = [oracle.field_direct_ondemand(n, L, radii, 2, at, box.sources, tg) for at in box.bands]
    print(f"case six bands n={n} fp32", flush=True)
    _run(box, lc.LC_PREC_FP32, np.float32, tg, refs, "fp32")
