"""GPU tests of the rolling light-cone (lc_advance), the non-finite source
check (LC_ENONFINITE) and graph recapture after a kernel rebuild.

Rolling light-cone (the paragraph after the algorithm of Sec. 2.2): sources
are drawn per absolute time bin; at observing step t the slice of lookback
k holds bin t + K - 1 - k. After each lc_advance the field must equal the
oracle's field for the lookback-ordered sources, and be bitwise equal to a
fresh plan into which the same sources were pushed in lookback order (the
slice sum runs over lookback slices in the same order either way).
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


def say(msg):
    print(msg, flush=True)


def _bins(n, count, seed):
    return [li.random_sources([seed, j], n, 30 + 7 * j) for j in range(count)]


def _lookback(bins, K, t):
    return [bins[t + K - 1 - k] for k in range(K)]


def _push(plan, box, k, src, as_points, f64):
    c, v = src
    if as_points:
        return plan.push_points(box, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
    g = torch.from_numpy(li.dense_grid(plan.boxes[box].n, c, v)).cuda()
    return plan.push_grid(box, k, g if f64 else g.float())


def _advance(plan, box, src, as_points, f64):
    c, v = src
    if as_points:
        return plan.advance(box, (torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda()))
    g = torch.from_numpy(li.dense_grid(plan.boxes[box].n, c, v)).cuda()
    return plan.advance(box, g if f64 else g.float())


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("as_points", [True, False])
def test_rolling_matches_oracle_and_fresh_plan(form, as_points):
    lc = _lc()
    n, L, K, steps = 32, 30.0, 5, 4
    radii = np.linspace(0.0, 26.0, K + 1)
    bins = _bins(n, K + steps, 77)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    f64 = form == "fp64"
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.lw_band(22.0)], sources=_lookback(bins, K, 0))
    G = oracle.build_G(n, L, radii, 2, box.bands[0])
    roll = lc.Plan([box], precision=prec)
    roll.build_all()
    keep = [_push(roll, 0, k, s, as_points, f64) for k, s in enumerate(box.sources)]
    for t in range(steps):
        if t > 0:
            keep.append(_advance(roll, 0, bins[t + K - 1], as_points, f64))
        J = roll.field(0, 0).double().cpu().numpy()
        srcs = _lookback(bins, K, t)
        Jr = oracle.field_direct(G, srcs, np.arange(n ** 3)).reshape((n,) * 3)
        e_max, e_rms = oracle.rel_errors(J, Jr)
        say(f"rolling {form} points={as_points} t={t}: e_max={e_max:.3e} e_rms={e_rms:.3e}")
        assert (e_max <= 1e-12) if f64 else (e_rms <= 1e-5 and e_max <= 1e-4)
        fresh = lc.Plan([box], precision=prec)
        fresh.build_all()
        kf = [_push(fresh, 0, k, s, as_points, f64) for k, s in enumerate(srcs)]
        Jf = fresh.field(0, 0).double().cpu().numpy()
        fresh.close()
        if as_points and not f64:
            # coincident points are deposited with FP64 atomics in any order
            assert np.max(np.abs(J - Jf)) <= 1e-6 * np.max(np.abs(Jf))
        else:
            assert np.array_equal(J, Jf)
        del kf
    roll.close()


# (24: a fused tile of 64 columns, wider than the Nyquist set and than the
# main set's last tile, so the tile order's narrower last tiles are used;
# 256 and 512: the eight-element schedule with one slice prefetched)
@pytest.mark.parametrize("n,bands", [(24, 1), (32, 1), (48, 2), (128, 1), (256, 1), (512, 1)])
def test_rolling_with_3d_spectra(n, bands):
    """spectra_3d = 1: every push (lc_push_sources, lc_advance, lc_step)
    also transforms the slice along z, and a field is the product with G^
    and the sum over slices alone. Four observing times against the oracle
    and against the default schedule (which transforms along z in the
    fused pass: equal up to FP32 rounding), and lc_step at the last ring
    position against lc_field."""
    lc = _lc()
    K, steps = 5, 4
    L = 0.9 * n
    radii = np.linspace(0.0, 0.85 * L, K + 1)
    bins = _bins(n, K + steps, 55 + n)
    ats = [li.lw_band(0.8 * L), li.Atten(kind=0)][:bands]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=ats, sources=_lookback(bins, K, 0))
    tg = np.arange(n ** 3) if n <= 48 else li.sample_cells([3, n], n, 2000)
    Gs = [oracle.build_G(n, L, radii, 2, at) for at in ats] if n <= 48 else None
    plans = {}
    for s3 in (0, 1):
        p = lc.Plan([box], precision=lc.LC_PREC_FP32)
        p.build_all()
        if s3:
            sch = p.get_schedule(0)
            xv = sch["xy_variant"]
            if xv >= 0 and xv >= {192: 2, 256: 4}.get(n, 99):
                xv = 0
            p.set_schedule(0, spectra_3d=1, xy_variant=xv)
            assert p.get_schedule(0)["spectra_3d"] == 1
            if n in (256, 512):
                # eight elements per thread, prefetch depth 1
                p.set_schedule(0, fused_variant={256: 3, 512: 1}[n])
        plans[s3] = p
    grids = [torch.from_numpy(li.dense_grid(n, c, v)).float().cuda() for c, v in bins]
    keep = []
    for s3, p in plans.items():
        for k in range(K):
            keep.append(p.push_grid(0, k, grids[K - 1 - k]))
    for t in range(steps):
        srcs = _lookback(bins, K, t)
        for s3, p in plans.items():
            if t > 0:
                p.advance(0, grids[t + K - 1])
        for b, at in enumerate(ats):
            J3 = plans[1].field(0, b).double().cpu().numpy().ravel()
            J0 = plans[0].field(0, b).double().cpu().numpy().ravel()
            if Gs is not None:
                Jr = oracle.field_direct(Gs[b], srcs, tg)
            else:
                Jr = oracle.field_direct_ondemand(n, L, radii, 2, at, srcs, tg)
            e_max, e_rms = oracle.rel_errors(J3[tg], Jr)
            d = np.sqrt(np.mean((J3 - J0) ** 2) / np.mean(J0 ** 2))
            say(f"rolling 3d n={n} t={t} band={b}: e_max={e_max:.3e} e_rms={e_rms:.3e} vs default {d:.3e}")
            assert e_rms <= 1e-5 and e_max <= 1e-4
            assert d <= 1e-6
    # a whole step at the last ring position equals the eager field
    out = [torch.empty((n,) * 3, dtype=torch.float32, device="cuda") for _ in ats]
    t = steps - 1
    plans[1].step([grids[t + K - 1 - k] for k in range(K)], out)
    for b in range(bands):
        Jf = plans[1].field(0, b)
        torch.cuda.synchronize()
        assert torch.equal(out[b], Jf)
    for p in plans.values():
        p.close()


def test_spectra_3d_schedule_checks():
    lc = _lc()
    n, K = 256, 2
    box = li.Box(n=n, box=200.0, radii=np.linspace(0.0, 20.0, K + 1), supersample=1, bands=[li.Atten()],
                 sources=_bins(n, K, 5))
    p = lc.Plan([box], precision=lc.LC_PREC_FP32)
    for bad in (dict(spectra_3d=2), dict(spectra_3d=1, xy_variant=4), dict(spectra_3d=-1)):
        with pytest.raises(lc.LCError) as ei:
            p.set_schedule(0, **bad)
        assert ei.value.code == lc.LC_EINVAL
    p.set_schedule(0, spectra_3d=1, xy_variant=1)
    assert p.get_schedule(0)["spectra_3d"] == 1
    p.close()
    p64 = lc.Plan([box], precision=lc.LC_PREC_FP64)
    assert p64.get_schedule(0)["spectra_3d"] == -1
    with pytest.raises(lc.LCError):
        p64.set_schedule(0, spectra_3d=1)
    p64.close()


def test_rolling_step_after_advance_parity_layout():
    """256^3 with the autotuned (parity layout) shapes: lc_step captures a
    graph for the current ring position; after lc_advance the next lc_step
    captures again and both equal fresh plans bitwise."""
    lc = _lc()
    n, L, K = 256, 200.0, 4
    radii = np.linspace(0.0, 24.0, K + 1)
    bins = _bins(n, K + 2, 91)
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.Atten(kind=0)], sources=_lookback(bins, K, 0))
    grids = [torch.from_numpy(li.dense_grid(n, c, v)).float().cuda() for c, v in bins]
    roll = lc.Plan([box], precision=lc.LC_PREC_FP32, use_graph=True, autotune=True)
    roll.build_all()
    say(f"rolling 256 schedule {roll.get_schedule(0)}")
    out = [torch.empty((n,) * 3, dtype=torch.float32, device="cuda")]
    results = []
    for t in range(3):
        if t == 0:
            roll.step([grids[K - 1 - k] for k in range(K)], out)
            J = out[0].clone()
        else:
            roll.advance(0, grids[t + K - 1])
            J = roll.field(0, 0)
            # a whole step at this ring position (graph captured again)
            roll.step([grids[t + K - 1 - k] for k in range(K)], out)
            torch.cuda.synchronize()
            assert torch.equal(out[0], J)
        fresh = lc.Plan([box], precision=lc.LC_PREC_FP32, autotune=False)
        fresh.set_schedule(0, **{k: v for k, v in roll.get_schedule(0).items() if k not in ("n_xy", "n_fused", "n_fused_bands")})
        fresh.build_all()
        for k in range(K):
            fresh.push_grid(0, k, grids[t + K - 1 - k])
        Jf = fresh.field(0, 0)
        torch.cuda.synchronize()
        fresh.close()
        say(f"rolling 256 t={t}: max diff vs fresh {float((J - Jf).abs().max()):.3e}")
        assert torch.equal(J, Jf)
        results.append(J)
    roll.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_nonfinite_sources_are_reported(form):
    lc = _lc()
    n, L, K = 32, 30.0, 4
    radii = np.linspace(0.0, 20.0, K + 1)
    srcs = [li.random_sources([5, k], n, 30) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=1, bands=[li.Atten(kind=0)], sources=srcs)
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    dt = torch.float64 if form == "fp64" else torch.float32
    plan = lc.Plan([box], precision=prec, use_graph=True)
    plan.build_all()
    grids = [torch.from_numpy(li.dense_grid(n, c, v)).to(dt).cuda() for c, v in srcs]
    for k in range(K):
        plan.push_grid(0, k, grids[k])
    plan.field(0, 0)
    plan.check_sources()                      # all finite: no error
    bad = grids[2].clone()
    bad[123] = float("nan")
    plan.push_grid(0, 2, bad)
    with pytest.raises(lc.LCError) as ei:     # host output: reported by lc_field itself
        plan.field(0, 0, out=torch.empty((n,) * 3, dtype=dt))
    assert ei.value.code == lc.LC_ENONFINITE and "lookback slice 2" in str(ei.value)
    plan.check_sources()                      # the flag was cleared by that report
    inf = grids[1].clone()
    inf[7] = float("inf")
    out = [torch.empty((n,) * 3, dtype=dt, device="cuda")]
    plan.step([grids[0], inf, grids[2], grids[3]], out)   # device outputs: no sync, no error
    with pytest.raises(lc.LCError) as ei:
        plan.check_sources(0)
    assert ei.value.code == lc.LC_ENONFINITE and "lookback slice 1" in str(ei.value)
    plan.step(grids, out)
    plan.check_sources(0)
    plan.close()


def test_rebuilt_kernel_recaptures_the_step():
    """A captured step holds each band's slice count; rebuilding a band so
    that its kernel reaches more slices must not replay the old graph."""
    lc = _lc()
    n, L, K = 32, 30.0, 6
    radii = np.linspace(0.0, 24.0, K + 1)
    srcs = [li.random_sources([8, k], n, 25) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=2,
                 bands=[li.Atten(kind=2, a=1.7, s=116.29 * 0.1, p=0.68, c=0.7, cut=9.0)], sources=srcs)
    for prec in (lc.LC_PREC_FP32, lc.LC_PREC_FP64):
        dt = torch.float64 if prec == lc.LC_PREC_FP64 else torch.float32
        plan = lc.Plan([box], precision=prec, use_graph=True)
        plan.build_all()                      # hard cut at 9: slices beyond it carry no kernel
        grids = [torch.from_numpy(li.dense_grid(n, c, v)).to(dt).cuda() for c, v in srcs]
        out = [torch.empty((n,) * 3, dtype=dt, device="cuda")]
        plan.step(grids, out)
        plan.build_greens(0, 0, li.Atten(kind=0))   # now every slice has a kernel
        plan.step(grids, out)
        for k in range(K):
            plan.push_grid(0, k, grids[k])
        eager = plan.field(0, 0)
        torch.cuda.synchronize()
        assert torch.equal(out[0], eager)
        G = oracle.build_G(n, L, radii, 2, li.Atten(kind=0))
        Jr = oracle.field_direct(G, srcs, np.arange(n ** 3))
        e_max, e_rms = oracle.rel_errors(out[0].double().cpu().numpy().ravel(), Jr)
        say(f"recapture prec={prec}: e_max={e_max:.3e} e_rms={e_rms:.3e}")
        assert (e_max <= 1e-12) if prec == lc.LC_PREC_FP64 else (e_rms <= 1e-5)
        plan.close()


@pytest.mark.parametrize("form,s3", [("fp64", 0), ("fp32", 0), ("fp32", 1)])
def test_rolling_through_several_ring_wraps(form, s3):
    """23 observing times with K = 5 slices: the ring's head wraps four
    times. Every fourth field (and the last) against the oracle's field for
    the lookback-ordered sources, route D on the full grid; new slices
    alternate between point lists and dense grids; FP32 forms with and
    without 3D spectra."""
    lc = _lc()
    n, L, K, steps = 24, 18.0, 5, 23
    radii = np.linspace(0.0, 16.0, K + 1)
    bins = _bins(n, K + steps, 91)
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.lw_band(14.0)], sources=_lookback(bins, K, 0))
    G = oracle.build_G(n, L, radii, 2, box.bands[0])
    f64 = form == "fp64"
    p = lc.Plan([box], precision=lc.LC_PREC_FP64 if f64 else lc.LC_PREC_FP32)
    p.build_all()
    if s3:
        p.set_schedule(0, spectra_3d=1, xy_variant=p.get_schedule(0)["xy_variant"])
    keep = [_push(p, 0, k, s, False, f64) for k, s in enumerate(box.sources)]
    for t in range(steps):
        if t > 0:
            keep.append(_advance(p, 0, bins[t + K - 1], t % 2 == 0, f64))
        if t % 4 and t != steps - 1:
            continue
        J = p.field(0, 0).double().cpu().numpy().ravel()
        Jr = oracle.field_direct(G, _lookback(bins, K, t), np.arange(n ** 3))
        e_max, e_rms = oracle.rel_errors(J, Jr)
        say(f"rolling wraps {form} spectra_3d={s3} t={t}: e_max={e_max:.3e} e_rms={e_rms:.3e}")
        assert (e_max <= 1e-12) if f64 else (e_rms <= 1e-5 and e_max <= 1e-4)
    p.close()
    del keep
