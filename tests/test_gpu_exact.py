"""GPU parity of the exact cell-averaged mesh kernel (lc_box_desc.rule = 1,
the m -> infinity limit of the subpoint average of Eq. 10 over a cell),
through the C ABI, against the CPU FP64 oracle's own exact cell average
(route D with the dense exact kernel): the FP64 form to e_max <= 1e-12, the
FP32 form to e_rms <= 1e-5; shells that cut through the source's own cell
(allowed with the exact rule only); the particle-mesh correction on top of
the exact mesh kernel."""
import numpy as np
import pytest

import lc_inputs as li
import oracle
from parity_log import record

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lc():
    import paper_1502_02294_amd as lc
    return lc


def _run(box, prec, dtype):
    lc = _lc()
    plan = lc.Plan([box], precision=prec)
    plan.build_all()
    keep = [plan.push_points(0, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
            for k, (c, v) in enumerate(box.sources)]
    Js = [plan.field(0, b, dtype=dtype).double().cpu().numpy() for b in range(len(box.bands))]
    dcs = [plan.greens_dc(0, b) for b in range(len(box.bands))]
    torch.cuda.synchronize()
    del keep
    plan.close()
    return Js, dcs


@pytest.mark.parametrize("n,radii", [
    (16, [0.0, 0.6, 2.1, 4.5, 7.9]),      # r_1 < (sqrt 3 / 2) l: the source cell spans two shells
    (24, [0.5, 3.0, 6.5, 11.0]),           # r_0 > 0 inside the source cell
])
def test_exact_rule_fp64_and_fp32_full_grid(n, radii):
    lc = _lc()
    L = float(n)
    radii = np.asarray(radii)
    K = len(radii) - 1
    bands = [li.Atten(kind=0), li.lw_band(0.8 * radii[-1]),
             li.Atten(kind=2, a=1.7, s=0.55 * radii[-1], p=0.68, c=0.7, cut=0.7 * radii[-1])]
    srcs = [li.random_sources([51, n, k], n, 12 + 5 * k) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=1, bands=bands, sources=srcs, rule=1)
    Gs = [oracle.build_G_exact(n, L, radii, at) for at in bands]
    Jr = [oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape((n,) * 3) for G in Gs]
    for prec, dt, name in ((lc.LC_PREC_FP64, torch.float64, "fp64"), (lc.LC_PREC_FP32, torch.float32, "fp32")):
        print(f"case exact rule n={n} {name}", flush=True)
        Js, dcs = _run(box, prec, dt)
        for b in range(len(bands)):
            e_max, e_rms = oracle.rel_errors(Js[b], Jr[b])
            print(f"  band {b}: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
            record(f"exact cell average {n}^3 band {b}", name, e_max, e_rms, Js[b].size)
            if name == "fp64":
                assert e_max <= 1e-12
                # G^_k(0) = sum_c G_k(c): with exact cell averages, l^3 times
                # it is the shell integral of phi (l = 1 here)
                np.testing.assert_allclose(dcs[b], Gs[b].sum(axis=(1, 2, 3)), rtol=1e-12)
                flux = [oracle.shell_integral(bands[b], radii[k], radii[k + 1]) for k in range(K)]
                np.testing.assert_allclose(dcs[b], flux, rtol=1e-12)
            else:
                assert e_rms <= 1e-5 and e_max <= 1e-4


def test_exact_rule_near_field_correction():
    lc = _lc()
    print("case exact rule near field 32^3", flush=True)
    n, L, K, R = 32, 40.0, 3, 3
    radii = np.array([0.0, 1.0, 6.0, 12.0])
    at = li.lw_band(11.0)
    positioned = [li.positioned_sources([93, k], L, 20 + 10 * k) for k in range(K)]
    cells = [(oracle.ngp_cells(n, L, p), v) for p, v in positioned]
    box = li.Box(n=n, box=L, radii=radii, supersample=1, bands=[at], sources=cells, rule=1)
    plan = lc.Plan([box], precision=lc.LC_PREC_FP64)
    plan.build_all()
    dev = [lc.Positioned(torch.from_numpy(np.ascontiguousarray(p)).cuda(), torch.from_numpy(v).cuda())
           for p, v in positioned]
    keep = [plan.push_positioned(0, k, s.pos, s.lum) for k, s in enumerate(dev)]
    J = plan.field(0, 0, dtype=torch.float64)
    plan.near_field(0, 0, dev, R, J)
    Jc = J.cpu().numpy()
    G = oracle.build_G_exact(n, L, radii, at)
    Jr = (oracle.field_direct(G, cells, np.arange(n ** 3)).reshape((n,) * 3)
          + oracle.near_correction(n, L, radii, 1, [at] * K, positioned, R, rule=1))
    e_max, e_rms = oracle.rel_errors(Jc, Jr)
    print(f"exact rule near field: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
    record("exact cell average + near field 32^3", "fp64", e_max, e_rms, Jc.size)
    assert e_max <= 1e-12
    del keep
    plan.close()
