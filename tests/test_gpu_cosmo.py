"""GPU tests of the cosmological radial factors and the light-cone vs
instantaneous comparison (Sec. 3, Eqs. 14-18), through the C ABI, against
the CPU FP64 oracle.

Lyman-Werner field: slices of 2 Myr of cosmic time before z = 27.9 in a
periodic box of side 114/h Mpc scaled to the grid (the paper's set-up at a
coarser cell), per-slice factors (1+z)^3/(1+z_s) and alpha(z_s); radii and
factors are the oracle's, fed to both sides. Instantaneous field: every
slice's sources frozen at the observing time (lc_field_frozen), and the
fractional difference map (lc_fdiff)."""
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


def say(msg):
    print(msg, flush=True)


def _lw_box(n, K, kind, seed):
    h, om, z_obs, dt = 0.7, 0.27, 27.9, 2.0
    radii, _, z_src = oracle.cosmo_slices(h, om, z_obs, dt, K)
    L = 114.0 / h * n / 256 * 4          # 0.636 Mpc cells x 4 (coarser than the paper's 256^3)
    attens = oracle.lw_factors(h, om, z_obs, z_src, kind)
    # sources grow toward the present (first stars switching on)
    srcs = [li.random_sources([seed, k], n, 60 - 8 * k) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.Atten(kind=0)], sources=srcs)
    return box, attens


def _gpu(box, attens, prec, frozen=False, as_points=True):
    lc = _lc()
    plan = lc.Plan([box], precision=prec)
    plan.build_greens_slices(0, 0, attens)
    keep = []
    for k, (c, v) in enumerate(box.sources):
        if as_points:
            keep.append(plan.push_points(0, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda()))
        else:
            g = torch.from_numpy(li.dense_grid(box.n, c, v)).cuda()
            keep.append(plan.push_grid(0, k, g if prec == lc.LC_PREC_FP64 else g.float()))
    odt = torch.float64 if prec == lc.LC_PREC_FP64 else torch.float32
    J = plan.field(0, 0, dtype=odt)
    Ji = plan.field_frozen(0, 0, 0, dtype=odt)
    F = lc.fdiff(J, Ji)
    torch.cuda.synchronize()
    res = [t.double().cpu().numpy() for t in (J, Ji, F)]
    plan.close()
    return res


@pytest.mark.parametrize("kind", [2, 1])
def test_lw_lightcone_and_instantaneous_fields(kind):
    lc = _lc()
    box, attens = _lw_box(32, 5, kind, 400 + kind)
    say(f"case LW cosmology kind={kind}: radii {np.round(box.radii, 2)} L={box.box:.2f}")
    G = oracle.build_G_slices(box.n, box.box, box.radii, box.supersample, attens)
    tg = np.arange(box.n ** 3)
    Jr = oracle.field_direct(G, box.sources, tg).reshape((box.n,) * 3)
    Jir = oracle.field_direct(G, oracle.frozen_sources(box.sources), tg).reshape((box.n,) * 3)
    Fr = oracle.fdiff(Jr, Jir)
    big = Jr > 1e-2 * Jr.max()
    for form, prec in (("fp64", lc.LC_PREC_FP64), ("fp32", lc.LC_PREC_FP32)):
        J, Ji, F = _gpu(box, attens, prec, as_points=(form == "fp64"))
        for name, a, b in (("light-cone", J, Jr), ("instantaneous", Ji, Jir)):
            e_max, e_rms = oracle.rel_errors(a, b)
            say(f"LW kind={kind} {form} {name}: e_max={e_max:.3e} e_rms={e_rms:.3e}")
            record(f"LW cosmology kind {kind} {name} 32^3 full grid", form, e_max, e_rms, a.size)
            if form == "fp64":
                assert e_max <= 1e-12
            else:
                assert e_rms <= 1e-5 and e_max <= 1e-4
        dF = np.max(np.abs(F[big] - Fr[big]))
        say(f"LW kind={kind} {form} f_diff on cells with J > 1% max: max abs diff {dF:.3e}, "
            f"mean f_diff {Fr[big].mean():+.4f}")
        assert dF <= (1e-11 if form == "fp64" else 1e-4)


def test_frozen_field_after_advance_and_two_bands():
    """The frozen slice follows the ring (lookback 0 after lc_advance), in
    the fused FP32 form with two bands in one launch, and in the FP64 form."""
    lc = _lc()
    n, L, K = 32, 30.0, 4
    radii = np.linspace(0.0, 24.0, K + 1)
    bins = [li.random_sources([55, j], n, 40) for j in range(K + 1)]
    bands = [li.lw_band(22.0), li.lw_band(12.0)]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=bands, sources=[bins[K - 1 - k] for k in range(K)])
    for prec, tol in ((lc.LC_PREC_FP64, 1e-12), (lc.LC_PREC_FP32, 1e-5)):
        plan = lc.Plan([box], precision=prec)
        plan.build_all()
        keep = [plan.push_points(0, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
                for k, (c, v) in enumerate(box.sources)]
        keep.append(plan.advance(0, (torch.from_numpy(bins[K][0]).cuda(), torch.from_numpy(bins[K][1]).cuda())))
        now = [bins[K - k] for k in range(K)]          # lookback order after the advance
        for band, at in enumerate(bands):
            G = oracle.build_G(n, L, radii, 2, at)
            Jir = oracle.field_direct(G, oracle.frozen_sources(now), np.arange(n ** 3))
            Ji = plan.field_frozen(0, band, 0).double().cpu().numpy().ravel()
            e_max, e_rms = oracle.rel_errors(Ji, Jir)
            say(f"frozen after advance prec={prec} band={band}: e_max={e_max:.3e} e_rms={e_rms:.3e}")
            assert (e_max if prec == lc.LC_PREC_FP64 else e_rms) <= tol
            # frozen at another lookback slice
            Jir2 = oracle.field_direct(G, oracle.frozen_sources(now, 2), np.arange(n ** 3))
            Ji2 = plan.field_frozen(0, band, 2).double().cpu().numpy().ravel()
            e_max, e_rms = oracle.rel_errors(Ji2, Jir2)
            assert (e_max if prec == lc.LC_PREC_FP64 else e_rms) <= tol
        with pytest.raises(lc.LCError):
            plan.field_frozen(0, 0, K)
        plan.close()
