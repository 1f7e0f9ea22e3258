"""GPU test of positioned sources (nearest-node deposit, lc_sources kind 2)
and the particle-mesh near-field correction (lc_near_field, Sec. 4),
through the C ABI, against the CPU FP64 oracle: the mesh field of the
deposited sources (route D) plus the oracle's correction, both forms, two
bands with different factors, per-slice factors."""
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


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_near_field_correction_against_oracle(form):
    lc = _lc()
    n, L, K, m, R = 32, 40.0, 4, 2, 3
    radii = np.array([0.0, 3.0, 7.0, 12.0, 18.0])
    bands = [li.lw_band(16.0), li.Atten(kind=0, prefactor=1.0 / (4 * np.pi))]
    positioned = [li.positioned_sources([90, k], L, 25 + 10 * k) for k in range(K)]
    cells = [(oracle.ngp_cells(n, L, p), v) for p, v in positioned]
    box = li.Box(n=n, box=L, radii=radii, supersample=m, bands=bands, sources=cells)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    dt = torch.float64 if form == "fp64" else torch.float32
    plan = lc.Plan([box], precision=prec)
    plan.build_all()
    dev = [lc.Positioned(torch.from_numpy(np.ascontiguousarray(p)).cuda(), torch.from_numpy(v).cuda())
           for p, v in positioned]
    keep = [plan.push_positioned(0, k, s.pos, s.lum) for k, s in enumerate(dev)]
    for b, at in enumerate(bands):
        J = plan.field(0, b, dtype=dt)
        Jmesh = J.double().cpu().numpy()
        plan.near_field(0, b, dev, R, J)
        Jc = J.double().cpu().numpy()
        G = oracle.build_G(n, L, radii, m, at)
        Jr_mesh = oracle.field_direct(G, cells, np.arange(n ** 3)).reshape((n,) * 3)
        corr = oracle.near_correction(n, L, radii, m, [at] * K, positioned, R)
        Jr = Jr_mesh + corr
        for label, a, r in (("mesh", Jmesh, Jr_mesh), ("corrected", Jc, Jr)):
            e_max, e_rms = oracle.rel_errors(a, r)
            print(f"near {form} band {b} {label}: e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
            record(f"near field band {b} {label} 32^3", form, e_max, e_rms, a.size)
            if form == "fp64":
                assert e_max <= 1e-12
            else:
                assert e_rms <= 1e-5 and e_max <= 1e-4
        # the correction itself, where it is large enough to measure
        dc = Jc - Jmesh
        big = np.abs(corr) > 1e-3 * np.abs(corr).max()
        rel = np.max(np.abs(dc[big] - corr[big])) / np.abs(corr).max()
        print(f"near {form} band {b}: correction rel err {rel:.3e} on {big.sum()} cells", flush=True)
        assert rel <= (1e-12 if form == "fp64" else 1e-5)
    plan.close()


def test_near_field_argument_checks():
    lc = _lc()
    n, L, K = 16, 16.0, 2
    radii = np.array([0.0, 2.0, 4.0])
    box = li.Box(n=n, box=L, radii=radii, supersample=1, bands=[li.Atten(kind=0)],
                 sources=[li.random_sources([1, k], n, 3) for k in range(K)])
    plan = lc.Plan([box], precision=lc.LC_PREC_FP64)
    plan.build_all()
    pos, lum = li.positioned_sources([2, 0], L, 5)
    dev = [lc.Positioned(torch.from_numpy(pos).cuda(), torch.from_numpy(lum).cuda())] * K
    out = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(lc.LCError):
        plan.near_field(0, 0, dev, 9, out)        # beyond the supported radius
    with pytest.raises(lc.LCError):
        plan.near_field(0, 0, dev, 4, out)        # (R+1) sqrt 3 l >= L / 2
    plan.near_field(0, 0, dev, 2, out)
    plan.close()
