#!/usr/bin/env python3
"""Benchmark of the light-cone field on one MI355X.

One step = the whole path over one batch of synthetic input: every slice's
source grid (already resident in HBM) is staged and transformed, and the
field of every band is evaluated (lc_step, replayed from a captured HIP
graph). Kernel construction is precomputation and is timed separately.

Prints ONE JSON line. Headline workload: 256^3 grid, 200 Mpc box, 40 slices
of 5 Mpc, FP32 form (Kahan slice sum, FP64 mean and kernels); the plain FP64
method is timed at the same shape for comparison. Beside the headline the
line carries the 512^3 x 60 x 4-band step, the 16 uneven boxes in one step,
and the rolling light-cone (one new slice per observing time).

roofline: the whole step against HBM bandwidth on the method's compulsory
bytes per step (read every source grid and every kernel octant once, write
every band's field once), with the bytes the implemented passes move and the
measured traffic beside it; the dominant kernel's own figures are in
roofline.dominant.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "retarded-field cell-updates/s (cells×slices/s) + HBM GB/s vs peak; FP32 vs FP64"
SRC_FILES = ["lc_fft_device.h", "lc_fft.hip", "lc_xy.hip", "lc_field.hip", "lc_greens.hip", "lc_host.cpp",
             "lc_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash() -> str:
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, "paper_1502_02294_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name):
    import lc_inputs as li
    if name == "grid256":
        w = li.points_256c_40s()
        desc = ("256^3 periodic grid, 200 Mpc box, 40 slices of 5 Mpc (0-200 Mpc), "
                "uniform lognormal sources x1.15 per slice (355816 total), phi=1, m=4")
    elif name == "grid32":
        w = li.points_32c_8s()
        desc = "32^3 grid, 20 Mpc box, 8 slices over 0-20 Mpc, 200 sources/slice, phi=1, m=1"
    elif name == "grid128":
        w = li.grf_128c_24s()
        desc = ("128^3 grid, 100 Mpc box, 24 slices over 0-100 Mpc, top-1% GRF peaks, "
                "LW-like attenuation s=116 Mpc, m=4")
    else:
        raise SystemExit(f"unknown workload {name}")
    return w, desc


def oct_bytes(n, rsz):
    return (n // 2 + 1) ** 3 * rsz


def compulsory_bytes(n, K, B, rsz=4):
    """The method's compulsory HBM bytes per field evaluation: every slice's
    source grid read once, every (slice, band) kernel octant read once, every
    band's field written once (FP32: 4 + 0.5 B bytes per cell-slice plus the
    fields)."""
    return n ** 3 * K * rsz + oct_bytes(n, rsz) * K * B + n ** 3 * rsz * B


def bytes_model(n, K, B, fused, csz, rsz):
    """Bytes each kernel launch moves in the implemented passes (FP32:
    csz=8, rsz=4); B = bands handled per launch."""
    n3 = n ** 3
    spec = n * n * (n // 2 + 1) * csz
    octb = oct_bytes(n, rsz)
    m = {
        "xy_fwd": n3 * rsz + spec,            # fused x + y: read the grid, write the y-transformed spectrum
        "x_fwd": n3 * rsz + spec,             # read the source grid, write the half spectrum
        "col_y_fwd": 2 * spec,                # read + write one spectrum
        "col_y_inv": 2 * spec,
        "x_inv": spec + n3 * rsz,             # read spectrum, write the field
        "yx_inv": spec + n3 * rsz,            # fused inverse y + x (parity layout): read A, write the field
    }
    if fused:
        m["fused_z"] = K * (spec + octb * B) + B * spec   # every slice + its kernel octants, write A once
    else:
        m["col_z_fwd"] = 2 * spec
        m["mac"] = spec + octb + 2 * spec               # read S^, G^, read-modify-write A
        m["col_z_inv"] = 2 * spec
    return m


def compulsory_share(name, n, K, B, group, rsz=4):
    """Compulsory bytes attributed to one launch of a kernel: the forward
    pass reads the source grids, the slice sum reads the kernel octants, the
    last inverse pass writes the field."""
    n3 = n ** 3
    if name in ("xy_fwd", "x_fwd"):
        return n3 * rsz * group
    if name == "fused_z":
        return oct_bytes(n, rsz) * K * B
    if name in ("yx_inv", "x_inv"):
        return n3 * rsz
    return 0


def timed_steps(torch, plan, grids, outs, steps, warmup):
    st = plan.stream          # the stream the kernels run on
    # steps are issued with the plan's stream current, as a loop of steps
    # would run in production: no cross-stream ordering between steps
    with torch.cuda.stream(st):
        for _ in range(max(1, warmup)):
            plan.step(grids, outs)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            plan.step(grids, outs)
        e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return e0.elapsed_time(e1) / steps, 1e3 * wall / steps


def copy_probe_gbps(torch, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of nbytes (the runtime's copy kernel),
    bytes read plus bytes written per second: what a copy-like pass reaches
    on this device."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, c
    torch.cuda.empty_cache()
    return gbps


def per_step_times(torch, plan, grids, outs, steps):
    """Median and minimum of single steps, each bracketed by its own pair of
    events on the plan's stream (after the timed region; not `value`)."""
    st = plan.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    with torch.cuda.stream(st):
        for a, b in ev:
            a.record(st)
            plan.step(grids, outs)
            b.record(st)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return {"median": t[len(t) // 2], "min": t[0], "count": steps}


def run_form(lc, torch, boxes, grids, precision, steps, warmup, time_kernels=True):
    """Build, then time `steps` graph-replayed lc_step calls over all boxes."""
    fused = precision == lc.LC_PREC_FP32
    plan = lc.Plan(boxes, precision=precision, use_graph=True, autotune=fused)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.build_all()
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    odt = torch.float64 if precision == lc.LC_PREC_FP64 else torch.float32
    outs = [torch.empty((b.n,) * 3, dtype=odt, device="cuda") for b in boxes for _ in b.bands]
    ms, wall_ms = timed_steps(torch, plan, grids, outs, steps, warmup)
    cells = sum(b.n ** 3 * b.n_slices for b in boxes)
    res = {"ms_per_step": ms, "wall_ms_per_step": wall_ms, "build_s": t_build,
           "step_ms": per_step_times(torch, plan, grids, outs, steps),
           "value": cells / (ms * 1e-3), "schedule": plan.get_schedule(0)}
    if time_kernels:
        res["kernels"] = kernel_times(lc, plan, boxes[0], precision, ms)
    return res, outs, plan


def kernel_times(lc, plan, box, precision, ms):
    K, B, n = box.n_slices, len(box.bands), box.n
    fused = precision == lc.LC_PREC_FP32
    sched = plan.get_schedule(0)
    group = 1
    if sched["xy_variant"] >= 0:
        # timed in the step's launch configuration: `group` slices per launch
        group = min(sched["push_group"], K)
        ids = {"xy_fwd": lc.LC_KERNEL_XY_FWD}
        per_step = {"xy_fwd": K / group}
    else:
        ids = {"x_fwd": lc.LC_KERNEL_X_FWD, "col_y_fwd": lc.LC_KERNEL_COL_Y_FWD}
        per_step = {"x_fwd": K, "col_y_fwd": K}
    # the parity-layout schedule fuses the inverse y and x passes
    try:
        plan.time_kernel(lc.LC_KERNEL_YX_INV, 0, 1)
        ids["yx_inv"] = lc.LC_KERNEL_YX_INV
        per_step["yx_inv"] = B
    except lc.LCError:
        ids.update({"col_y_inv": lc.LC_KERNEL_COL_Y_INV, "x_inv": lc.LC_KERNEL_X_INV})
        per_step.update({"col_y_inv": B, "x_inv": B})
    if fused:
        ids["fused_z"] = lc.LC_KERNEL_FUSED_Z
        per_step["fused_z"] = (B + 1) // 2
    else:
        ids.update({"col_z_fwd": lc.LC_KERNEL_COL_Z_FWD, "mac": lc.LC_KERNEL_MAC,
                    "col_z_inv": lc.LC_KERNEL_COL_Z_INV})
        per_step.update({"col_z_fwd": K, "mac": K * B, "col_z_inv": B})
    csz, rsz = (16, 8) if precision == lc.LC_PREC_FP64 else (8, 4)
    bl = min(B, 2) if fused else 1
    model = bytes_model(n, K, bl, fused, csz, rsz)
    model["xy_fwd"] *= group
    kern = {}
    for name, kid in ids.items():
        reps = 3 if name == "fused_z" else (2 * K if name != "xy_fwd" else max(3, 2 * K // group))
        t = plan.time_kernel(kid, 0, reps)
        comp = compulsory_share(name, n, K, bl, group, rsz)
        kern[name] = {"avg_ms": t, "launches_per_step": per_step[name],
                      "slices_per_launch": group if name == "xy_fwd" else 1,
                      "pass_bytes": model[name], "pass_GBps": model[name] / (t * 1e-3) / 1e9,
                      "compulsory_bytes": comp, "compulsory_GBps": comp / (t * 1e-3) / 1e9,
                      "step_share": t * per_step[name] / ms}
    return kern


def load_traffic(wname, kern):
    """Per-launch HBM traffic of each kernel from the committed profiler
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), while the kernel sources
    still hash to the profiled ones; else None."""
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tpath):
        return {}
    try:
        tj = json.load(open(tpath))
    except Exception:
        return {}
    out = {}
    h = src_hash()
    ent = tj.get(f"{wname}:step")
    if ent and ent.get("src_hash") == h:
        out["step"] = ent["bytes_per_step"]
    for name, kd in kern.items():
        ent = tj.get(f"{wname}:{name}")
        if not ent or ent.get("src_hash") != h:
            continue
        if "bytes_per_slice" in ent:   # kernels launched over several slices
            out[name] = ent["bytes_per_slice"] * kd["slices_per_launch"]
        else:
            out[name] = ent["bytes_per_launch"]
    return out


def vs_oracle(box, J32, J64):
    """Errors against the stored FP64 oracle reference on the 64^3 stride-4
    sub-lattice (route D, written by tests/golden/make_golden.py), when it
    belongs to exactly these inputs."""
    import lc_inputs as li
    base = os.path.join(ROOT, "tests", "golden", "grid256_slices40_sublattice4")
    if not (os.path.exists(base + ".npz") and os.path.exists(base + ".json")):
        return None
    meta = json.load(open(base + ".json"))
    if meta.get("inputs_sha256") != li.sources_digest(box):
        return None
    with np.load(base + ".npz", allow_pickle=False) as z:
        ref = z["J"]
    tg = li.sublattice_cells(box.n, 4)
    res = {"cells": int(len(tg)), "reference": "route D, 64^3 stride-4 sub-lattice (stored)"}
    for name, J in (("fp32", J32), ("fp64_plain", J64)):
        if J is None:
            continue
        v = J.reshape(-1)[__import__("torch").from_numpy(tg).to(J.device)].double().cpu().numpy()
        d = v - ref
        res[name] = {"e_max": float(np.max(np.abs(d)) / np.max(np.abs(ref))),
                     "e_rms": float(np.linalg.norm(d) / np.linalg.norm(ref))}
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(box, seconds):
    """The CPU FP64 oracle on the host's cores: route D (direct periodic
    summation, kernel from its definition) on a seeded sample of target
    cells, all slices, scaled to cell-slices/s; the builder and route F
    (naive DFT) timed on samples and extrapolated to one field."""
    import lc_inputs as li
    import oracle
    K = box.n_slices
    band = box.bands[0]
    cores = oracle.num_threads()
    pilot = li.sample_cells(901, box.n, cores)
    t0 = time.perf_counter()
    oracle.field_direct_ondemand(box.n, box.box, box.radii, box.supersample, band, box.sources, pilot)
    tp = max(time.perf_counter() - t0, 1e-3)
    T = int(max(cores, min(16384, cores * seconds / tp)))
    targets = li.sample_cells(902, box.n, T)
    t0 = time.perf_counter()
    oracle.field_direct_ondemand(box.n, box.box, box.radii, box.supersample, band, box.sources, targets)
    t = time.perf_counter() - t0
    # builder: all K kernel values at a sample of displacements (the oracle
    # evaluates every cell of the grid), extrapolated to N^3 cells
    disp = li.sample_cells(903, box.n, 256)
    t0 = time.perf_counter()
    for c in disp:
        i, j, x = np.unravel_index(int(c), (box.n,) * 3)
        oracle.G_at(box.n, box.box, box.radii, box.supersample, band, (int(i), int(j), int(x)))
    tb = (time.perf_counter() - t0) / len(disp) * box.n ** 3 / cores
    # route F: one naive separable 3D DFT of N^3 (2K + 1 of them per field)
    x = np.random.default_rng(904).standard_normal((box.n,) * 3)
    t0 = time.perf_counter()
    oracle.dft3(x)
    tf = time.perf_counter() - t0
    # context (not the oracle and not a target): the same spectral method on
    # the CPU with a library FFT (scipy.fft, FP64, all cores), kernel spectra
    # precomputed as on the GPU; one forward transform, product and sum per
    # slice, one inverse per field, timed on one slice and scaled to K
    import scipy.fft as sfft
    n = box.n
    Gh = np.random.default_rng(905).standard_normal((n, n, n // 2 + 1))
    A = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    tfw, tmac, tinv = [], [], []
    for _ in range(3):
        t0 = time.perf_counter()
        Sh = sfft.rfftn(x, workers=cores)
        tfw.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        Sh *= Gh
        A += Sh
        tmac.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        sfft.irfftn(A, s=(n, n, n), workers=cores)
        tinv.append(time.perf_counter() - t0)
    t_step = K * (min(tfw) + min(tmac)) + min(tinv)
    context = {"value": n ** 3 * K / t_step, "unit": "cell-slices/s", "cores": cores,
               "kind": "context: the spectral method with scipy.fft FP64 (not the oracle)",
               "sample": f"one {n}^3 forward transform, product-sum and inverse (best of 3), "
                         f"scaled to {K} slices per field",
               "s_per_field": t_step}
    return {"value": T * K / t, "unit": "cell-slices/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{T} seeded target cells x all {K} slices, route D (direct periodic summation, "
                      f"kernel from its definition), {t:.1f} s",
            "route_D_full_grid_s_extrapolated": t / T * box.n ** 3,
            "builder_s_extrapolated": tb,
            "builder_sample": f"256 displacements x {K} slices, serial, scaled to N^3 cells over {cores} threads",
            "route_F_dft3_s": tf,
            "route_F_field_s_extrapolated": tf * (2 * K + 1),
            "spectral_library_fft": context}


def bands_leg(lc, torch, steps, fp64_steps):
    """512^3 x 60 slices x 4 bands (horizons 100/80/60/40 Mpc), FP32 form in
    batched launches; the plain FP64 method beside it. Timing inputs: dense
    uniform random grids drawn on the device (run time does not depend on
    the values; the Gaussian-field recipe is checked for parity in the tests)."""
    import lc_inputs as li
    n, K = 512, 60
    L = 400.0
    radii = li.equal_radii(100.0, K)
    box = li.Box(n=n, box=L, radii=radii, supersample=4, bands=[li.lw_band(h) for h in (100.0, 80.0, 60.0, 40.0)],
                 sources=[])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4512)
    res = {"workload": "grid512_slices60_bands4: 512^3 grid, 400 Mpc box, 60 slices over 0-100 Mpc, "
                       "4 bands (LW-like horizons 100/80/60/40 Mpc), m=4",
           "input": "dense uniform random FP32 grids drawn on the device (timing only)"}
    grids = [torch.rand(n ** 3, device="cuda", generator=gen) for _ in range(K)]
    log("grid512 bands: fp32 form build + timed steps")
    r32, outs, plan = run_form(lc, torch, [box], grids, lc.LC_PREC_FP32, steps, 1, time_kernels=False)
    plan.close()
    del outs
    res["fp32"] = {"ms_per_step": r32["ms_per_step"], "cell_slices_per_s": r32["value"],
                   "cell_slice_bands_per_s": r32["value"] * 4, "build_s": r32["build_s"],
                   "schedule": r32["schedule"],
                   "compulsory_GBps": compulsory_bytes(n, K, 4) / (r32["ms_per_step"] * 1e-3) / 1e9}
    res["fp32"]["compulsory_frac"] = res["fp32"]["compulsory_GBps"] / HBM_PEAK_GBPS
    log(f"grid512 fp32 {r32['ms_per_step']:.2f} ms/step")
    if fp64_steps > 0:
        g64 = []
        for g in grids:
            g64.append(g.double())
        del grids
        torch.cuda.empty_cache()
        log("grid512 bands: fp64 plain build + timed steps")
        r64, outs, plan = run_form(lc, torch, [box], g64, lc.LC_PREC_FP64, fp64_steps, 1, time_kernels=False)
        plan.close()
        del outs, g64
        res["fp64_plain"] = {"ms_per_step": r64["ms_per_step"], "cell_slices_per_s": r64["value"]}
        res["speedup_vs_fp64_plain"] = r64["ms_per_step"] / r32["ms_per_step"]
        log(f"grid512 fp64 {r64['ms_per_step']:.2f} ms/step")
    else:
        del grids
    torch.cuda.empty_cache()
    return res


def uneven_leg(lc, torch, steps, fp64_steps):
    """16 periodic boxes of 64^3..256^3 with 8..48 slices in one
    graph-captured step (boxes on four concurrent lanes), FP32 form with
    per-size autotuned shapes; the plain FP64 method beside it. Inputs: the
    seeded Poisson point lists deposited to dense grids on the device."""
    import lc_inputs as li
    w = li.uneven_16boxes()
    res = {"workload": "uneven16boxes: 16 boxes N in {64,96,128,192,256} (seeded mix), 8-48 slices each, "
                       "Poisson sources 1e-3/cell, lognormal L, phi=1, m=4",
           "cell_slices": w.cell_slices()}

    def grids_of(dt):
        out = []
        for b in w.boxes:
            for c, v in b.sources:
                g = torch.zeros(b.n ** 3, dtype=dt, device="cuda")
                g.index_add_(0, torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda().to(dt))
                out.append(g)
        return out

    for name, prec, dt, nsteps in (("fp32", lc.LC_PREC_FP32, torch.float32, steps),
                                   ("fp64_plain", lc.LC_PREC_FP64, torch.float64, fp64_steps)):
        if nsteps <= 0:
            continue
        log(f"uneven boxes: {name} build + timed steps")
        grids = grids_of(dt)
        r, outs, plan = run_form(lc, torch, w.boxes, grids, prec, nsteps, 1, time_kernels=False)
        plan.close()
        del outs, grids
        res[name] = {"ms_per_step": r["ms_per_step"], "cell_slices_per_s": r["value"]}
        log(f"uneven {name} {r['ms_per_step']:.2f} ms/step")
    if "fp64_plain" in res:
        res["speedup_vs_fp64_plain"] = res["fp64_plain"]["ms_per_step"] / res["fp32"]["ms_per_step"]
    torch.cuda.empty_cache()
    return res


def rolling_leg(lc, torch, box, grids, steps):
    """The rolling light-cone at the headline shape: per observing time one
    new slice (lc_advance: one forward transform) and the field over all K
    lookback slices (lc_field: slice sum + one inverse), FP32 form. Two
    schedules: the default one, whose fused pass transforms every slice along
    z at each field, and spectra_3d, which transforms each slice along z once
    when it is pushed, so that the field is the product and sum alone."""
    n, K = box.n, box.n_slices
    res = {}
    for mode in ("fused_z", "spectra_3d"):
        plan = lc.Plan([box], precision=lc.LC_PREC_FP32, autotune=True)
        plan.build_all()
        if mode == "spectra_3d":
            sch = plan.get_schedule(0)
            # the fastest whole-plane xy shape (3D spectra need one)
            best = None
            for v in range(sch["n_xy"]):
                try:
                    plan.set_schedule(0, xy_variant=v, spectra_3d=1)
                except lc.LCError:
                    continue
                t = plan.time_kernel(lc.LC_KERNEL_XY_FWD, 0, 3)
                if best is None or t < best[0]:
                    best = (t, v)
            plan.set_schedule(0, xy_variant=best[1], spectra_3d=1)
        out = torch.empty((n,) * 3, dtype=torch.float32, device="cuda")
        if mode == "spectra_3d":
            # the fastest slice-sum schedule on 3D spectra (the plan-time
            # autotuner tuned it on the default layout)
            with torch.cuda.stream(plan.stream):
                for k in range(K):
                    plan.push_grid(0, k, grids[k])
            torch.cuda.synchronize()
            best = None
            for v in range(plan.get_schedule(0)["n_fused"]):
                for r in (1, 0):
                    plan.set_schedule(0, fused_variant=v, fused_rounds=r)
                    t = plan.time_kernel(lc.LC_KERNEL_FUSED_Z, 0, 3)
                    if best is None or t < best[0]:
                        best = (t, v, r)
            plan.set_schedule(0, fused_variant=best[1], fused_rounds=best[2])
        st = plan.stream
        with torch.cuda.stream(st):
            for k in range(K):
                plan.push_grid(0, k, grids[k])
            for j in range(3):
                plan.advance(0, grids[j % K])
                plan.field(0, 0, out=out)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            e0.record(st)
            for j in range(steps):
                plan.advance(0, grids[j % K])
                plan.field(0, 0, out=out)
            e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        t_fz = plan.time_kernel(lc.LC_KERNEL_FUSED_Z, 0, 3)
        res[mode] = {"ms_per_observing_step": ms, "cell_slices_per_s": n ** 3 * K / (ms * 1e-3),
                     "fused_z_ms": t_fz, "schedule": plan.get_schedule(0)}
        plan.close()
    res["note"] = ("one lc_advance (1 forward transform) + one lc_field (slice sum over all 40 slices, "
                   "1 inverse) per observing time, issued eagerly on the plan's stream")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid256", choices=["grid32", "grid128", "grid256"])
    ap.add_argument("--extras", default="grid512_bands4,uneven16,rolling",
                    help="comma list of legs reported beside the headline (grid512_bands4, uneven16, "
                         "rolling); empty for none")
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the legs named by --extras (for profiler runs of one leg) and print them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-kernel-times", action="store_true",
                    help="skip the per-kernel timing (for profiler runs of the step alone)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times "
                         "(reference for the profiler's byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the path runs on a "
              f"single MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import lc_inputs as li
    import paper_1502_02294_amd as lc
    lc.load()
    extras = [e for e in args.extras.split(",") if e]
    if args.skip_headline:
        line = {}
        if "grid512_bands4" in extras:
            line["grid512_bands4"] = bands_leg(lc, torch, max(3, args.steps // 4), 0 if args.no_fp64 else 2)
        if "uneven16" in extras:
            line["uneven16"] = uneven_leg(lc, torch, max(5, args.steps // 2), 0 if args.no_fp64 else 3)
        if "rolling" in extras:
            w, _ = workload(args.workload)
            box = w.boxes[0]
            g32 = [torch.from_numpy(li.dense_grid(box.n, c, v).astype(np.float32)).cuda() for c, v in box.sources]
            line["rolling"] = rolling_leg(lc, torch, box, g32, max(10, args.steps))
        print(json.dumps(line), flush=True)
        return
    w, desc = workload(args.workload)
    box = w.boxes[0]
    n, K, B = box.n, box.n_slices, len(box.bands)
    log(f"workload {w.name}: generating dense source grids")
    host = [li.dense_grid(n, c, v) for c, v in box.sources]
    g32 = [torch.from_numpy(h.astype(np.float32)).cuda() for h in host]
    log("fp32 form: build + timed steps")
    r32, out32, plan32 = run_form(lc, torch, [box], g32, lc.LC_PREC_FP32, args.steps, args.warmup,
                                  time_kernels=not args.no_kernel_times)
    plan32.close()
    del plan32
    log(f"fp32 {r32['ms_per_step']:.3f} ms/step")
    line = {
        "metric": METRIC, "value": r32["value"], "unit": "cell-slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
        "step_ms": r32["step_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {desc}", "grid": n, "slices": K, "bands": B,
                   "form": "FP32 butterflies, Kahan slice sum, FP64 twiddles/kernels/mean",
                   "input": "dense FP32 source grids resident in HBM", "graph": True,
                   "schedule": r32["schedule"]},
    }
    if args.no_kernel_times:
        print(json.dumps(line), flush=True)
        return
    kern = r32["kernels"]
    ms = r32["ms_per_step"]
    traffic = load_traffic(w.name, kern)
    step_comp = compulsory_bytes(n, K, B)
    step_pass = sum(v["pass_bytes"] * v["launches_per_step"] for v in kern.values())
    step_traffic = traffic.get("step")
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches_per_step"])
    kd = kern[dom]
    achieved = step_comp / (ms * 1e-3) / 1e9
    line["roofline"] = {
        "bound": "hbm", "kernel": "whole step (one lc_step graph replay)",
        "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
        "traffic": step_traffic,
        "algorithmic_bytes": step_comp,
        "pass_bytes": step_pass,
        "pass_GBps": step_pass / (ms * 1e-3) / 1e9,
        "pass_frac": step_pass / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "traffic_over_algorithmic": step_traffic / step_comp if step_traffic else None,
        "traffic_over_pass": step_traffic / step_pass if step_traffic else None,
        "dominant": {"kernel": dom, "avg_ms": kd["avg_ms"], "step_share": kd["step_share"],
                     "compulsory_GBps": kd["compulsory_GBps"],
                     "compulsory_frac": kd["compulsory_GBps"] / HBM_PEAK_GBPS,
                     "pass_GBps": kd["pass_GBps"], "pass_frac": kd["pass_GBps"] / HBM_PEAK_GBPS,
                     "traffic": traffic.get(dom),
                     "traffic_over_pass": traffic[dom] / kd["pass_bytes"] if dom in traffic else None},
    }
    probe = copy_probe_gbps(torch)
    line["roofline"]["copy_probe_GBps"] = probe
    line["roofline"]["pass_frac_of_copy_probe"] = line["roofline"]["pass_GBps"] / probe
    line["roofline"]["dominant"]["pass_frac_of_copy_probe"] = kd["pass_GBps"] / probe
    line["kernels"] = {k: {"avg_ms": round(v["avg_ms"], 5), "pass_GBps": round(v["pass_GBps"], 1),
                           "step_share": round(v["step_share"], 3),
                           "slices_per_launch": v["slices_per_launch"],
                           "traffic_over_pass": round(traffic[k] / v["pass_bytes"], 3) if k in traffic else None}
                       for k, v in kern.items()}
    line["build_s"] = r32["build_s"]
    line["src_hash"] = src_hash()

    out64 = None
    if not args.no_fp64:
        g64 = [torch.from_numpy(h).cuda() for h in host]
        log("fp64 plain method: build + timed steps")
        r64, out64, plan64 = run_form(lc, torch, [box], g64, lc.LC_PREC_FP64, args.fp64_steps, 1)
        plan64.close()
        del plan64
        log(f"fp64 {r64['ms_per_step']:.3f} ms/step")
        line["fp64_plain"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                              "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "pass_GBps": round(v["pass_GBps"], 1)}
                                          for k, v in r64["kernels"].items()}}
        line["speedup_vs_fp64_plain"] = r32["value"] / r64["value"]
        d = (out32[0].double() - out64[0])
        line["fp32_vs_fp64_gpu"] = {
            "e_max": float(d.abs().max() / out64[0].abs().max()),
            "e_rms": float(d.norm() / out64[0].norm())}
        del g64
    vo = vs_oracle(box, out32[0], out64[0] if out64 is not None else None)
    if vo:
        line["vs_oracle"] = vo
    if "rolling" in extras:
        log("rolling light-cone leg")
        line["rolling"] = rolling_leg(lc, torch, box, g32, max(10, args.steps))
        log("rolling " + ", ".join(f"{m} {line['rolling'][m]['ms_per_observing_step']:.3f}"
                                    for m in ("fused_z", "spectra_3d")) + " ms/observing step")
    del g32, out32, out64
    torch.cuda.empty_cache()
    if "grid512_bands4" in extras:
        line["grid512_bands4"] = bands_leg(lc, torch, max(3, args.steps // 4), 0 if args.no_fp64 else 2)
    if "uneven16" in extras:
        line["uneven16"] = uneven_leg(lc, torch, max(5, args.steps // 2), 0 if args.no_fp64 else 3)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(box, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
