"""Benchmark of the explicit MHD step on one MI355X.

Workload: the 3D stratified MHD box at 256^3 (n = 1.5 polytrope, gamma =
5/3, four pressure scale heights, isobaric 1e-4 density noise, seed field at
beta = 1e6, periodic x/y, reflecting z), SSP-RK2, CFL 0.4.  A step is the
whole hot path: the CFL reduction and the two fused stage kernels
(primitive recovery, van Leer reconstruction, LHLLD fluxes, Contact-CT EMFs,
cell and face updates), with the state resident in HBM.

Printed: one JSON line with zone-updates/s of the FP64 path (`value`), the
roofline of its dominant kernel (the stage kernel), the same for the split
precision path, and the FP64 oracle timed on the host cores on a bounded
sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per zone-update of one SSP-RK2 step: stage 1 reads U^n
# (5 + 3 FP64 = 64 B) and writes U^(1) (64 B); stage 2 reads U^n and U^(1)
# and writes U^(n+1) -> 128 + 192 = 320 B; per stage launch on average 160 B.
BYTES_PER_ZONE_STEP = 320.0
BYTES_PER_ZONE_STAGE = BYTES_PER_ZONE_STEP / 2.0
METRIC = "zone-updates/s (3D MHD 256^3) FP64 vs FP32+learned-EOS; % HBM roofline"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_run(mhd, w, precision, steps, warmup, cfl):
    import torch
    g = mhd.Grid(w.params, precision=precision)
    g.load(w)
    stream = torch.cuda.current_stream()
    g.advance(cfl, warmup)
    g.sync()
    torch.cuda.synchronize()
    # whole-step throughput: device-side dt + both stages, no host round trip
    t0 = time.perf_counter()
    g.advance(cfl, steps)
    g.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # stage-kernel duration with HIP events on the library's stream: a fixed
    # dt so that only the two stage launches run between the events
    dt = g.compute_dt(cfl)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    nrep = max(steps, 4)
    e0.record(stream)
    for _ in range(nrep):
        g.step(dt)
    e1.record(stream)
    e1.synchronize()
    g.sync()
    stage_ms = e0.elapsed_time(e1) / (2.0 * nrep)
    diag = g.diagnostics()
    info = g.launch_info()
    g.close()
    return wall, stage_ms, diag, info


def roofline(ncell, stage_ms):
    achieved = BYTES_PER_ZONE_STAGE * ncell / (stage_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "stage_kernel", "bytes_per_zone_stage": BYTES_PER_ZONE_STAGE}


def cpu_baseline(n, target_s=12.0):
    """The FP64 oracle on the host cores: the same stratified-box workload at
    n^3, as many steps as fit in about target_s seconds (at least one)."""
    from oracle import orc
    from paper_2604_12672_amd import workloads as wl
    w = wl.stratified_box(n)
    o = orc.Oracle(w.params, **w.extras())
    st = w.state()
    o.step(st, o.compute_dt(st, w.cfl))  # warm-up (page-in, thread start)
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(st, o.compute_dt(st, w.cfl))
        steps += 1
        if time.perf_counter() - t0 > target_s:
            break
    el = time.perf_counter() - t0
    return {"value": round(w.ncells * steps / el, 1), "unit": "zone-updates/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"stratified box {n}^3, {steps} SSP-RK2 steps incl. CFL, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="linear grid size")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=96)
    ap.add_argument("--only", choices=["fp64", "split"], default=None)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the halo-exchange design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_12672_amd import mhd
    from paper_2604_12672_amd import workloads as wl
    if not os.path.exists(mhd.LIB_PATH):
        from paper_2604_12672_amd import build
        build.build()
    mhd.load()
    torch.cuda.set_device(0)
    n = args.n
    log(f"bench: building stratified box {n}^3")
    w = wl.stratified_box(n)
    cfl = w.cfl
    res = {}
    for name, prec in (("fp64", mhd.PREC_FP64), ("split", mhd.PREC_SPLIT)):
        if args.only and args.only != name:
            continue
        if name == "split" and args.no_split:
            continue
        log(f"bench: {name} warmup={args.warmup} steps={args.steps}")
        wall, stage_ms, diag, info = gpu_run(mhd, w, prec, args.steps, args.warmup, cfl)
        res[name] = dict(wall=wall, stage_ms=stage_ms, diag=diag, info=info)
        log(f"bench: {name} {wall / args.steps * 1e3:.3f} ms/step, stage {stage_ms:.3f} ms, "
            f"divB {diag['divb_max']:.2e}")
    if args.calib_copy:
        # plain streaming kernel of known size: reads 2^30 bytes, writes 2^30
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("bench: calibration copy of 1 GiB done")
    main_name = "fp64" if "fp64" in res else "split"
    r = res[main_name]
    ms = r["wall"] / args.steps * 1e3
    value = w.ncells * args.steps / r["wall"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "zone-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"stratified MHD box {n}^3 (n=1.5 polytrope, 4 H_P, beta 1e6 "
                               f"seed field, periodic x/y, reflecting z), SSP-RK2, CFL {cfl}, "
                               f"van Leer + LHLLD + Contact-CT, ideal gas, {main_name} path",
                   "cells": w.ncells, "grid": [n, n, n], "precision": main_name,
                   "launch": r["info"]},
        "roofline": roofline(w.ncells, r["stage_ms"]),
        "divb_max": r["diag"]["divb_max"],
    }
    if "split" in res and main_name == "fp64":
        s = res["split"]
        sms = s["wall"] / args.steps * 1e3
        out["split"] = {"value": round(w.ncells * args.steps / s["wall"], 1),
                        "ms_per_step": round(sms, 4), "dtype": "f32 flux/recon/EMF, f64 rest",
                        "speedup_vs_fp64": round(ms / sms, 3),
                        "roofline": roofline(w.ncells, s["stage_ms"]),
                        "divb_max": s["diag"]["divb_max"]}
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle) {args.cpu_n}^3")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
