"""GPU parity of fused z launches that take three or four bands at once.

At N = 384 and 512 one fused z launch can take up to four bands (radial
factors of Sec. 3 sharing the sources), reading each slice spectrum once for
all of them; those launches keep plain FP32 sums over the slices, the launches
of one or two bands compensated ones. Every bands-per-launch setting, with both
scheduling modes of the fused pass, is compared with the CPU FP64 oracle
(route D, the kernel evaluated from its definition at sampled cells) and with
the two-band launches. Tolerance: the FP32 form's e_rms <= 1e-5 (normwise) with
e_max <= 1e-4; plain and compensated sums agree to 1e-5 rms.
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


def _box(n, K, bands, seed):
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.45 * L, K + 1)
    srcs = [li.random_sources([seed, n, k], n, 150) for k in range(K)]
    return li.Box(n=n, box=L, radii=radii, supersample=2, bands=bands, sources=srcs)


@pytest.mark.parametrize("nbands,order", [(4, "falling"), (3, "falling"), (4, "rising")])
def test_bands_per_fused_launch_384(nbands, order):
    lc = _lc()
    n, K = 384, 4
    L = 0.78125 * n
    # horizons inside the lookback range: the later bands carry fewer slices
    # ("rising": the last band of a launch reaches the most slices, so the
    # launch's slice count must come from every band, not the first two)
    horizons = [0.44 * L, 0.3 * L, 0.2 * L, 0.12 * L][:nbands]
    if order == "rising":
        horizons = horizons[::-1]
    box = _box(n, K, [li.lw_band(h) for h in horizons], seed=41 + nbands + (order == "rising"))
    tg = li.sample_cells([9, n], n, 2000)
    Jr = [oracle.field_direct_ondemand(n, L, box.radii, box.supersample, at, box.sources, tg)
          for at in box.bands]
    plan = lc.Plan([box], precision=lc.LC_PREC_FP32)
    plan.build_all()
    s = plan.get_schedule(0)
    assert s["n_fused_bands"] == nbands and s["fused_bands"] == nbands
    keep = [plan.push_grid(0, k, torch.from_numpy(li.dense_grid(n, cells, lum, np.float32)).cuda())
            for k, (cells, lum) in enumerate(box.sources)]
    torch.cuda.synchronize()
    ref2 = None
    for fb in (2, nbands, 1):
        for r in (1, 0):
            print(f"case n={n} nbands={nbands} {order} fused_bands={fb} rounds={r}", flush=True)
            plan.set_schedule(0, fused_bands=fb, fused_rounds=r)
            Js = [plan.field(0, b).double().cpu().numpy().ravel() for b in range(nbands)]
            for b in range(nbands):
                e_max, e_rms = oracle.rel_errors(Js[b][tg], Jr[b])
                print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
                assert e_rms <= 1e-5 and e_max <= 1e-4
            if ref2 is None:
                ref2 = Js
            else:
                for b in range(nbands):
                    d = np.sqrt(np.mean((Js[b] - ref2[b]) ** 2) / np.mean(ref2[b] ** 2))
                    print(f"  band={b} vs two-band launches: rel rms {d:.3e}", flush=True)
                    assert d <= 1e-5
    # 3D spectra in the slice-sum pass's tile order (8-column tiles at 384):
    # pushed again, then the product and sum alone, every bands-per-launch
    # setting
    plan.set_schedule(0, spectra_3d=1, fused_rounds=1)
    keep += [plan.push_grid(0, k, torch.from_numpy(li.dense_grid(n, cells, lum, np.float32)).cuda())
             for k, (cells, lum) in enumerate(box.sources)]
    for fb in (nbands, 2):
        print(f"case n={n} nbands={nbands} {order} spectra_3d fused_bands={fb}", flush=True)
        plan.set_schedule(0, fused_bands=fb)
        for b in range(nbands):
            J = plan.field(0, b).double().cpu().numpy().ravel()
            e_max, e_rms = oracle.rel_errors(J[tg], Jr[b])
            d = np.sqrt(np.mean((J - ref2[b]) ** 2) / np.mean(ref2[b] ** 2))
            print(f"  band={b} e_max={e_max:.3e} e_rms={e_rms:.3e} vs default {d:.3e}", flush=True)
            assert e_rms <= 1e-5 and e_max <= 1e-4 and d <= 1e-5
    del keep
    plan.close()
