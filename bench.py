#!/usr/bin/env python3
"""Benchmark of the light-cone field on one MI355X.

One step = the whole path over one batch of synthetic input: every slice's
source grid (already resident in HBM) is staged and transformed, and the
field of every band is evaluated (lc_step, replayed from a captured HIP
graph). Kernel construction is precomputation and is timed separately.

Prints ONE JSON line (see the fields below). Default workload: 256^3 grid,
200 Mpc box, 40 slices of 5 Mpc, FP32 form (Kahan slice sum, FP64 mean and
kernels); the plain FP64 method is timed at the same shape for comparison.
"""
import argparse
import hashlib
import json
import math
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


def bytes_model(n, K, B, fused, csz, rsz):
    """Algorithmic bytes per launch of each kernel (FP32: csz=8, rsz=4)."""
    n3 = n ** 3
    spec = n * n * (n // 2 + 1) * csz
    octb = (n // 2 + 1) ** 3 * rsz
    m = {
        "xy_fwd": n3 * rsz + spec,            # fused x + y: read the grid, write the y-transformed spectrum
        "x_fwd": n3 * rsz + spec,             # read the source grid, write the half spectrum
        "col_y_fwd": 2 * spec,                # read + write one spectrum
        "col_y_inv": 2 * spec,
        "x_inv": spec + n3 * rsz,             # read spectrum, write the field
        "yx_inv": spec + n3 * rsz,            # fused inverse y + x (parity layout): read A, write the field
    }
    if fused:
        m["fused_z"] = K * (spec + octb) + B * spec   # every slice + its kernel octant, write A once
    else:
        m["col_z_fwd"] = 2 * spec
        m["mac"] = spec + octb + 2 * spec               # read S^, G^, read-modify-write A
        m["col_z_inv"] = 2 * spec
    return m


def run_form(lc, torch, box, grids, precision, steps, warmup, time_kernels=True):
    K = box.n_slices
    B = len(box.bands)
    n = box.n
    fused = precision == lc.LC_PREC_FP32
    plan = lc.Plan([box], precision=precision, use_graph=True, autotune=fused)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.build_all()
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    odt = torch.float64 if precision == lc.LC_PREC_FP64 else torch.float32
    outs = [torch.empty((n, n, n), dtype=odt, device="cuda") for _ in range(B)]
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
    ms = e0.elapsed_time(e1) / steps
    sched = plan.get_schedule(0)
    res = {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "build_s": t_build,
           "value": n ** 3 * K / (ms * 1e-3), "schedule": sched}
    if time_kernels:
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
        model = bytes_model(n, K, min(B, 2) if fused else B, fused, csz, rsz)
        model["xy_fwd"] *= group
        kern = {}
        for name, kid in ids.items():
            reps = 3 if name == "fused_z" else (2 * K if name != "xy_fwd" else max(3, 2 * K // group))
            t = plan.time_kernel(kid, 0, reps)
            kern[name] = {"avg_ms": t, "launches_per_step": per_step[name],
                          "slices_per_launch": group if name == "xy_fwd" else 1,
                          "alg_bytes": model[name],
                          "GBps": model[name] / (t * 1e-3) / 1e9,
                          "step_share": t * per_step[name] / ms}
        res["kernels"] = kern
    out = [o.double() for o in outs]
    plan.close()
    return res, out


def cpu_baseline(box, seconds):
    """The CPU FP64 oracle (route D, kernel evaluated from its definition)
    on a seeded sample of target cells, all slices; scaled to cell-slices/s."""
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
    return {"value": T * K / t, "unit": "cell-slices/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{T} seeded target cells x all {K} slices, route D (direct periodic summation, "
                      f"kernel from its definition), {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid256", choices=["grid32", "grid128", "grid256"])
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
    w, desc = workload(args.workload)
    box = w.boxes[0]
    n, K = box.n, box.n_slices
    log(f"workload {w.name}: generating dense source grids")
    host = [li.dense_grid(n, c, v) for c, v in box.sources]
    g32 = [torch.from_numpy(h.astype(np.float32)).cuda() for h in host]
    log("fp32 form: build + timed steps")
    r32, out32 = run_form(lc, torch, box, g32, lc.LC_PREC_FP32, args.steps, args.warmup,
                          time_kernels=not args.no_kernel_times)
    log(f"fp32 {r32['ms_per_step']:.3f} ms/step")
    line = {
        "metric": METRIC, "value": r32["value"], "unit": "cell-slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {desc}", "grid": n, "slices": K, "bands": len(box.bands),
                   "form": "FP32 butterflies, Kahan slice sum, FP64 twiddles/kernels/mean",
                   "input": "dense FP32 source grids resident in HBM", "graph": True,
                   "schedule": r32["schedule"]},
    }
    if args.no_kernel_times:
        print(json.dumps(line), flush=True)
        return
    kern = r32["kernels"]
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches_per_step"])
    kd = kern[dom]
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tj = json.load(open(tpath))
            ent = tj.get(f"{w.name}:{dom}")
            if ent and ent.get("src_hash") == src_hash():
                if "bytes_per_slice" in ent:   # kernels launched over several slices
                    traffic = ent["bytes_per_slice"] * kd["slices_per_launch"]
                else:
                    traffic = ent["bytes_per_launch"]
        except Exception:
            traffic = None
    line["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": kd["GBps"], "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": kd["GBps"] / HBM_PEAK_GBPS, "traffic": traffic}
    line["kernels"] = {k: {"avg_ms": round(v["avg_ms"], 5), "GBps": round(v["GBps"], 1),
                           "step_share": round(v["step_share"], 3),
                           "slices_per_launch": v["slices_per_launch"]} for k, v in kern.items()}
    alg_step = n ** 3 * K * 4 + (n // 2 + 1) ** 3 * K * 4 * len(box.bands)
    line["step_alg_GBps"] = alg_step / (r32["ms_per_step"] * 1e-3) / 1e9
    line["build_s"] = r32["build_s"]
    line["src_hash"] = src_hash()

    if not args.no_fp64:
        g64 = [torch.from_numpy(h).cuda() for h in host]
        del g32
        log("fp64 plain method: build + timed steps")
        r64, out64 = run_form(lc, torch, box, g64, lc.LC_PREC_FP64, args.fp64_steps, 1)
        log(f"fp64 {r64['ms_per_step']:.3f} ms/step")
        line["fp64_plain"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                              "kernels": {k: {"avg_ms": round(v["avg_ms"], 5), "GBps": round(v["GBps"], 1)}
                                          for k, v in r64["kernels"].items()}}
        line["speedup_vs_fp64_plain"] = r32["value"] / r64["value"]
        d = (out32[0] - out64[0])
        line["fp32_vs_fp64_gpu"] = {
            "e_max": float(d.abs().max() / out64[0].abs().max()),
            "e_rms": float(d.norm() / out64[0].norm())}
        del g64
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(box, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
