"""GPU parity at the workload sizes, through the C ABI, against the CPU FP64
oracle (full field where the oracle finishes in seconds, sampled cells
otherwise), plus graph replay, repeatability and edge cases.

Tolerances: FP64 form e_max <= 1e-12; FP32 forms e_rms <= 1e-5 (normwise,
over the full field or the sample); e_max of the FP32 forms <= 1e-4.
"""
import math

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


def _box(n, L, radii, m, bands, sources, conserve=0):
    return li.Box(n=n, box=L, radii=np.asarray(radii, dtype=np.float64), supersample=m,
                  bands=bands, sources=sources, conserve=conserve)


def gpu_fields(boxes, precision, as_points=True, use_graph=False, step=False, out_dtype=None):
    """All bands of all boxes from one plan. Returns [box][band] float64 arrays."""
    lc = _lc()
    plan = lc.Plan(boxes, precision=precision, use_graph=use_graph)
    plan.build_all()
    keep = []
    odt = out_dtype or (torch.float64 if precision == lc.LC_PREC_FP64 else torch.float32)
    if step:
        grids = []
        for b in boxes:
            for c, v in b.sources:
                g = torch.from_numpy(li.dense_grid(b.n, c, v)).cuda()
                grids.append(g if precision == lc.LC_PREC_FP64 else g.float())
        outs = [torch.empty((b.n,) * 3, dtype=odt, device="cuda") for b in boxes for _ in b.bands]
        plan.step(grids, outs)
        keep.append(grids)
    else:
        for bi, b in enumerate(boxes):
            for k, (c, v) in enumerate(b.sources):
                if as_points:
                    keep.append(plan.push_points(bi, k, torch.from_numpy(np.ascontiguousarray(c)).cuda(),
                                                 torch.from_numpy(np.ascontiguousarray(v)).cuda()))
                else:
                    g = torch.from_numpy(li.dense_grid(b.n, c, v)).cuda()
                    keep.append(plan.push_grid(bi, k, g if precision == lc.LC_PREC_FP64 else g.float()))
        outs = [plan.field(bi, band, dtype=odt) for bi, b in enumerate(boxes) for band in range(len(b.bands))]
    torch.cuda.synchronize()
    res, i = [], 0
    for b in boxes:
        res.append([outs[i + j].double().cpu().numpy() for j in range(len(b.bands))])
        i += len(b.bands)
    plan.close()
    return res


def check(J, Jr, form, label):
    e_max, e_rms = oracle.rel_errors(J, Jr)
    say(f"{label}: {form} e_max={e_max:.3e} e_rms={e_rms:.3e}")
    record(label, form, e_max, e_rms, np.size(Jr))
    if form == "fp64":
        assert e_max <= 1e-12, (label, e_max)
    else:
        assert e_rms <= 1e-5, (label, e_rms)
        assert e_max <= 1e-4, (label, e_max)
    return e_max, e_rms


# --- full-grid parity: 128^3 x 24 slices, GRF peaks, LW-like attenuation ---------------

@pytest.fixture(scope="module")
def grid128_ref():
    b = li.grf_128c_24s().boxes[0]
    say("grid128: oracle kernel and spectral route with naive DFTs (Eqs. 12-13)")
    G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
    S = np.stack([oracle.deposit(b.n, c, v) for c, v in b.sources])
    J = oracle.field_dft(G, S)
    say("grid128: library-FFT route and route D at sampled cells (cross-checks)")
    JF = oracle.field_fft(lambda k: G[k], lambda k: S[k], b.n_slices, b.n)
    targets = li.sample_cells(2024, b.n, 256)
    JD = oracle.field_direct(G, b.sources, targets)
    return b, J, targets, JD, JF


def test_grid128_routes_agree(grid128_ref):
    """The three oracle routes agree: naive DFTs (the reference the GPU is held
    to), the library FFT, and the circular convolution sum of Eq. 11 at
    sampled cells."""
    b, J, targets, JD, JF = grid128_ref
    e_max, _ = oracle.rel_errors(J.ravel()[targets], JD)
    assert e_max <= 1e-12
    e_max, _ = oracle.rel_errors(J.ravel(), JF.ravel())
    assert e_max <= 1e-12


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp32_plain"])
def test_grid128_full_grid(grid128_ref, form):
    lc = _lc()
    b, J, targets, JD, _ = grid128_ref
    prec = {"fp64": lc.LC_PREC_FP64, "fp32": lc.LC_PREC_FP32, "fp32_plain": lc.LC_PREC_FP32_PLAIN}[form]
    say(f"case grid128 {form}")
    Jg = gpu_fields([b], prec, as_points=True)[0][0]
    check(Jg, J, form, "grid128 full grid")
    check(Jg.ravel()[targets], JD, form, "grid128 sampled route D")


# --- mean of the field: the FP64 DC mode -------------------------------------------------

@pytest.mark.parametrize("form", ["fp64", "fp32", "fp32_plain"])
def test_grid128_mean_is_fp64_dc(grid128_ref, form):
    """mean(J) = sum_k G^_k(0) S^_k(0) / N^3 (the DC bin of Eq. 13), with
    G^_k(0) = sum_c G_k(c) and S^_k(0) = sum_c S_k(c) from the oracle. The
    FP32 form keeps this bin in FP64, so its mean (FP64 output) is right to
    far below FP32 rounding; the plain FP32 form is held to FP32 rounding."""
    lc = _lc()
    b, J, targets, JD, _ = grid128_ref
    G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
    S = [oracle.deposit(b.n, c, v) for c, v in b.sources]
    mu = oracle.mean_field(G, np.stack(S))
    prec = {"fp64": lc.LC_PREC_FP64, "fp32": lc.LC_PREC_FP32, "fp32_plain": lc.LC_PREC_FP32_PLAIN}[form]
    Jg = gpu_fields([b], prec, as_points=True, out_dtype=torch.float64)[0][0]
    rel = abs(Jg.mean() - mu) / mu
    say(f"grid128 {form} mean rel error {rel:.3e}")
    assert rel <= {"fp64": 1e-13, "fp32": 1e-9, "fp32_plain": 1e-5}[form]


# --- 256^3 x 40 slices (the benchmark workload), on the benchmark's plan --------------------
# Stored reference: route D with the dense kernel on the 64^3 stride-4
# sub-lattice (tests/golden/make_golden.py), with the kernel sums G^_k(0).

def _golden(name):
    import json
    import os
    base = os.path.join(os.path.dirname(__file__), "golden", name)
    meta = json.load(open(base + ".json"))
    with np.load(base + ".npz", allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    return arrays, meta


@pytest.fixture(scope="module")
def grid256_golden():
    b = li.points_256c_40s().boxes[0]
    arrays, meta = _golden("grid256_slices40_sublattice4")
    assert meta["inputs_sha256"] == li.sources_digest(b), "stored reference was computed from other inputs"
    tg = li.sublattice_cells(b.n, 4)
    ssum = np.array([math.fsum(v) for _, v in b.sources])
    mu = float(np.dot(arrays["gsum"], ssum)) / b.n ** 3
    return b, tg, arrays["J"], mu


def _bench_plan_fields(b, precision, out_dtype):
    """The benchmark's configuration: dense grids resident on the device,
    autotuned launch shapes (FP32 form), one graph-captured lc_step."""
    lc = _lc()
    fused = precision == lc.LC_PREC_FP32
    plan = lc.Plan([b], precision=precision, use_graph=True, autotune=fused)
    plan.build_all()
    gdt = torch.float64 if precision == lc.LC_PREC_FP64 else torch.float32
    grids = [torch.from_numpy(li.dense_grid(b.n, c, v)).to(gdt).cuda() for c, v in b.sources]
    outs = [torch.empty((b.n,) * 3, dtype=out_dtype, device="cuda") for _ in b.bands]
    plan.step(grids, outs)
    plan.step(grids, outs)     # a replay of the captured graph
    torch.cuda.synchronize()
    sched = plan.get_schedule(0)
    plan.close()
    return [o.double().cpu().numpy() for o in outs], sched


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_grid256_bench_plan_sublattice(grid256_golden, form):
    """Element by element on the 64^3 stride-4 sub-lattice, with the plan the
    benchmark times (autotuned shapes, all 40 slices per forward launch,
    graph replay); FP64 output of the FP32 form also checks the FP64 mean."""
    lc = _lc()
    b, tg, JD, mu = grid256_golden
    prec = lc.LC_PREC_FP64 if form == "fp64" else lc.LC_PREC_FP32
    say(f"case grid256 {form} benchmark plan")
    outs, sched = _bench_plan_fields(b, prec, torch.float32 if form == "fp32" else torch.float64)
    say(f"grid256 {form} schedule {sched}")
    if form == "fp32":
        assert sched["push_group"] == b.n_slices
    check(outs[0].ravel()[tg], JD, form, "grid256 sub-lattice 64^3")
    if form == "fp64":
        rel = abs(outs[0].mean() - mu) / mu
        say(f"grid256 fp64 mean rel error {rel:.3e}")
        assert rel <= 1e-13


def test_grid256_fp32_mean_fp64_output(grid256_golden):
    lc = _lc()
    b, tg, JD, mu = grid256_golden
    outs, _ = _bench_plan_fields(b, lc.LC_PREC_FP32, torch.float64)
    rel = abs(outs[0].mean() - mu) / mu
    say(f"grid256 fp32 mean rel error {rel:.3e}")
    assert rel <= 1e-9
    check(outs[0].ravel()[tg], JD, "fp32", "grid256 sub-lattice 64^3, FP64 output")


def test_grid256_fp32_vs_fp64_full_grid(grid256_golden):
    lc = _lc()
    b = grid256_golden[0]
    say("case grid256 fp32 vs fp64 full grid")
    J64 = gpu_fields([b], lc.LC_PREC_FP64, step=True)[0][0]
    J32 = gpu_fields([b], lc.LC_PREC_FP32, step=True)[0][0]
    e_max, e_rms = oracle.rel_errors(J32, J64)
    say(f"grid256 fp32 vs gpu fp64: e_max={e_max:.3e} e_rms={e_rms:.3e}")
    assert e_rms <= 1e-5 and e_max <= 1e-4


# --- batched bands: 512^3 x 60 slices x 4 bands, Gaussian-field peak sources ----------------
# Stored reference: route D over the kernel's support, 16^3 stride-32
# sub-lattice per band.

def test_grid512_bands_sublattice():
    lc = _lc()
    say("grid512: drawing the Gaussian-field peak sources (16 processes)")
    b = li.bands_512c_60s(procs=16).boxes[0]
    arrays, meta = _golden("grid512_slices60_bands4_sublattice32")
    assert meta["inputs_sha256"] == li.sources_digest(b), "stored reference was computed from other inputs"
    tg = li.sublattice_cells(b.n, 32)
    say("case grid512 fp32 4 bands, benchmark plan (dense FP32 grids, graph)")
    plan = lc.Plan([b], precision=lc.LC_PREC_FP32, use_graph=True, autotune=True)
    plan.build_all()
    grids = []
    for c, v in b.sources:
        # top-1% cells of a field are distinct: the grid is a plain scatter
        g = torch.zeros(b.n ** 3, dtype=torch.float32, device="cuda")
        g[torch.from_numpy(c).cuda()] = torch.from_numpy(v).cuda().float()
        grids.append(g)
    outs = [torch.empty((b.n,) * 3, dtype=torch.float32, device="cuda") for _ in b.bands]
    plan.step(grids, outs)
    torch.cuda.synchronize()
    plan.close()
    del grids
    for band in range(4):
        Jg = outs[band].reshape(-1)[torch.from_numpy(tg).cuda()].double().cpu().numpy()
        check(Jg, arrays["J"][band], "fp32", f"grid512 band {band} sub-lattice 16^3")


# --- batched uneven boxes in one captured step ---------------------------------------------
# Boxes with N <= 128: the whole field against route F (naive DFT).
# Boxes with N > 128: the 16^3 sub-lattice against the stored route D.

@pytest.fixture(scope="module")
def uneven_step():
    lc = _lc()
    w = li.uneven_16boxes()
    say("case uneven fp32 16 boxes, one graph-captured step (autotuned)")
    plan = lc.Plan(w.boxes, precision=lc.LC_PREC_FP32, use_graph=True, autotune=True)
    plan.build_all()
    grids = [torch.from_numpy(li.dense_grid(b.n, c, v)).float().cuda() for b in w.boxes for c, v in b.sources]
    outs = [torch.empty((b.n,) * 3, dtype=torch.float32, device="cuda") for b in w.boxes]
    plan.step(grids, outs)
    torch.cuda.synchronize()
    plan.close()
    return w, [o.double().cpu().numpy() for o in outs]


@pytest.mark.parametrize("bi", range(16))
def test_uneven_box(uneven_step, bi):
    w, Js = uneven_step
    b = w.boxes[bi]
    if b.n <= 128:
        G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
        S = np.stack([oracle.deposit(b.n, c, v) for c, v in b.sources])
        Jr = oracle.field_dft(G, S)
        check(Js[bi], Jr, "fp32", f"uneven box {bi} N={b.n} K={b.n_slices} full grid vs naive DFT")
    else:
        arrays, meta = _golden("uneven16boxes_sublattice16")
        assert meta["boxes"][str(bi)]["inputs_sha256"] == li.sources_digest(b)
        tg = li.sublattice_cells(b.n, b.n // 16)
        check(Js[bi].ravel()[tg], arrays[f"J{bi}"], "fp32",
              f"uneven box {bi} N={b.n} K={b.n_slices} sub-lattice 16^3")


# --- graph replay, repeatability, input forms ---------------------------------------------

def test_graph_replay_equals_eager_and_is_repeatable():
    lc = _lc()
    n, L, K = 64, 50.0, 12
    radii = np.linspace(0.0, 50.0, K + 1)
    srcs = [li.random_sources([61, k], n, 300) for k in range(K)]
    b = _box(n, L, radii, 4, [li.Atten(kind=0)], srcs)
    say("case graph replay fp32")
    plan = lc.Plan([b], precision=lc.LC_PREC_FP32, use_graph=True)
    plan.build_all()
    grids = [torch.from_numpy(li.dense_grid(n, c, v)).float().cuda() for c, v in srcs]
    outs = [torch.empty((n,) * 3, dtype=torch.float32, device="cuda")]
    res = []
    for rep in range(3):
        plan.step(grids, outs)          # first call captures, later calls replay
        torch.cuda.synchronize()
        res.append(outs[0].clone())
        if rep == 1:
            torch.cuda.synchronize()
            grids[0].mul_(1.0)          # unrelated eager work between replays
    for k in range(K):
        plan.push_grid(0, k, grids[k])
    eager = plan.field(0, 0)
    torch.cuda.synchronize()
    plan.close()
    for r in res:
        assert torch.equal(r, res[0])   # bitwise repeatable
    assert torch.equal(eager, res[0])


def test_point_list_equals_dense_grid_fp64():
    lc = _lc()
    n, L, K = 32, 30.0, 5
    radii = np.linspace(0.0, 29.0, K + 1)
    srcs = [li.random_sources([71, k], n, 80) for k in range(K)]
    b = _box(n, L, radii, 2, [li.lw_band(20.0)], srcs)
    say("case points vs dense fp64")
    a = gpu_fields([b], lc.LC_PREC_FP64, as_points=True)[0][0]
    d = gpu_fields([b], lc.LC_PREC_FP64, as_points=False)[0][0]
    assert np.max(np.abs(a - d)) <= 1e-14 * np.max(np.abs(d))


# --- edge cases against the oracle ------------------------------------------------------------

def _small_case(n=24, L=30.0, radii=None, m=2, at=None, conserve=0, seed=0, counts=None):
    radii = np.linspace(0.0, 27.0, 5) if radii is None else np.asarray(radii)
    K = len(radii) - 1
    counts = counts or [20] * K
    srcs = [li.random_sources([seed, k], n, counts[k]) for k in range(K)]
    return _box(n, L, radii, m, [at or li.Atten(kind=0)], srcs, conserve)


def _oracle_full(b, band=0):
    G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[band], b.conserve)
    return oracle.field_direct(G, b.sources, np.arange(b.n ** 3)).reshape((b.n,) * 3), G


@pytest.mark.parametrize("label,kw", [
    ("conserve", dict(conserve=1)),
    ("paper_hard_cut", dict(at=li.Atten(kind=2, a=1.7, s=116.29 * 0.15, p=0.68, c=0.7, cut=97.39 * 0.15))),
    ("r0_positive", dict(radii=[3.0, 8.0, 13.0, 40.0])),
    ("prefactor", dict(at=li.Atten(kind=0, prefactor=1.0 / (4 * np.pi)))),
    ("m3_odd_subpoints", dict(m=3)),
    ("empty_slices", dict(counts=[0, 15, 0, 9])),
    ("images_beyond_box", dict(radii=[0.0, 10.0, 35.0, 70.0])),
])
def test_edge_cases_fp64_and_fp32(label, kw):
    lc = _lc()
    b = _small_case(**kw)
    Jr, G = _oracle_full(b)
    for form, prec in (("fp64", lc.LC_PREC_FP64), ("fp32", lc.LC_PREC_FP32)):
        say(f"case edge {label} {form}")
        J = gpu_fields([b], prec)[0][0]
        if not np.any(Jr):
            assert np.max(np.abs(J)) == 0.0
            continue
        check(J, Jr, form, f"edge {label}")


def test_all_sources_empty_gives_zero_field():
    lc = _lc()
    b = _small_case(counts=[0, 0, 0, 0])
    for prec in (lc.LC_PREC_FP64, lc.LC_PREC_FP32, lc.LC_PREC_FP32_PLAIN):
        J = gpu_fields([b], prec)[0][0]
        assert np.max(np.abs(J)) == 0.0


def test_builder_dc_and_real_spectrum_grid128():
    lc = _lc()
    b = li.grf_128c_24s(n=64).boxes[0]
    plan = lc.Plan([b], precision=lc.LC_PREC_FP32)
    plan.build_all()
    dc = np.array(plan.greens_dc(0, 0))
    im = plan.greens_imag_ratio(0, 0)
    plan.close()
    G = oracle.build_G(b.n, b.box, b.radii, b.supersample, b.bands[0])
    np.testing.assert_allclose(dc, G.sum(axis=(1, 2, 3)), rtol=1e-13)
    assert im <= 1e-14


def test_time_kernel_reports_positive_durations():
    lc = _lc()
    b = _small_case(n=64, L=60.0, radii=np.linspace(0.0, 55.0, 7))
    plan = lc.Plan([b], precision=lc.LC_PREC_FP32)
    plan.build_all()
    for kid in (lc.LC_KERNEL_X_FWD, lc.LC_KERNEL_COL_Y_FWD, lc.LC_KERNEL_FUSED_Z, lc.LC_KERNEL_COL_Y_INV,
                lc.LC_KERNEL_X_INV):
        assert plan.time_kernel(kid, 0, 2) > 0.0
    with pytest.raises(lc.LCError):
        plan.time_kernel(lc.LC_KERNEL_MAC, 0, 2)     # not part of the fused form
    with pytest.raises(lc.LCError):
        plan.time_kernel(lc.LC_KERNEL_YX_INV, 0, 2)  # parity-layout schedules only
    plan.close()


def test_grid512_forward_x_pass_forms():
    """N = 512 (the x pass alone, rows in batches with the untangle by lane
    moves): FP32 and plain-FP32 forms, dense FP32 grids and FP64 point lists,
    two slices, sampled cells against route D."""
    lc = _lc()
    n, K = 512, 2
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.06 * L, K + 1)
    srcs = [li.random_sources([512, k], n, 300) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.Atten(kind=0)], sources=srcs)
    tg = li.sample_cells([512, 1], n, 1500)
    Jr = oracle.field_direct_ondemand(n, L, radii, 2, box.bands[0], srcs, tg)
    for prec in (lc.LC_PREC_FP32, lc.LC_PREC_FP32_PLAIN):
        plan = lc.Plan([box], precision=prec)
        plan.build_all()
        for dense in (True, False):
            print(f"case n=512 prec={prec} dense={dense}", flush=True)
            if dense:
                keep = [plan.push_grid(0, k, torch.from_numpy(li.dense_grid(n, c, v, np.float32)).cuda())
                        for k, (c, v) in enumerate(srcs)]
            else:
                keep = [plan.push_points(0, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
                        for k, (c, v) in enumerate(srcs)]
            J = plan.field(0, 0).double().cpu().numpy().ravel()
            torch.cuda.synchronize()
            del keep
            e_max, e_rms = oracle.rel_errors(J[tg], Jr)
            print(f"n=512 prec={prec} dense={dense} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
            assert e_rms <= 1e-5 and e_max <= 1e-4
        plan.close()


def test_grid384_sampled_fp64_and_fp32():
    """N = 384 (radix 3 in every pass; eight-element fused schedule with
    8-column tiles): two slices, sampled cells against route D."""
    lc = _lc()
    n, K = 384, 2
    L = 0.78125 * n
    radii = np.linspace(0.0, 0.12 * L, K + 1)
    srcs = [li.random_sources([384, k], n, 300) for k in range(K)]
    box = li.Box(n=n, box=L, radii=radii, supersample=2, bands=[li.Atten(kind=0)], sources=srcs)
    tg = li.sample_cells([384, 1], n, 1500)
    Jr = oracle.field_direct_ondemand(n, L, radii, 2, box.bands[0], srcs, tg)
    for prec, tol in ((lc.LC_PREC_FP64, 1e-12), (lc.LC_PREC_FP32, 1e-5)):
        print(f"case n=384 prec={prec}", flush=True)
        plan = lc.Plan([box], precision=prec)
        plan.build_all()
        keep = [plan.push_points(0, k, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
                for k, (c, v) in enumerate(srcs)]
        J = plan.field(0, 0).double().cpu().numpy().ravel()
        plan.close()
        e_max, e_rms = oracle.rel_errors(J[tg], Jr)
        print(f"n=384 prec={prec} e_max={e_max:.3e} e_rms={e_rms:.3e}", flush=True)
        assert (e_max if prec == lc.LC_PREC_FP64 else e_rms) <= tol
