"""Benchmark of the explicit MHD step on one MI355X.

Headline workload: the 3D stratified MHD box at 256^3 (n = 1.5 polytrope,
gamma = 5/3, four pressure scale heights, isobaric 1e-4 density noise, seed
field at beta = 1e6, periodic x/y, reflecting z), SSP-RK2, CFL 0.4.  A step
is the whole hot path: the CFL reduction and the two fused stage kernels
(primitive recovery, van Leer reconstruction, LHLLD fluxes, Contact-CT EMFs,
cell and face updates), with the state resident in HBM.

Printed: one JSON line with zone-updates/s of the FP64 path (`value`) and the
roofline of its dominant kernel (the stage kernel); the split-precision path
on the same box; the gas+radiation box at 256^3 (FP64 with the previous-T
guess against split precision with the learned guess); the batch EOS
inversion (learned guess against the bracketed solve); the split and FP64
paths' per-field error against the FP64 oracle after 50 steps of the
stratified box with heating and cooling at 128^3; the 384^3 forced
turbulence box (learned guess, split precision); and the FP64 oracle timed
on the host cores on the headline workload (two steps per run, median of
three runs).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per zone of one stage launch (FP64 state, each array
# touched once): stage 1 reads U^n (5 cell + 3 face values = 64 B) and writes
# U^(1) (64 B); stage 2 reads U^n and U^(1) and writes U^(n+1): 128 + 192 =
# 320 B per SSP-RK2 step, 160 B per stage launch on average.  The gas +
# radiation EOS with the previous-step temperature adds that temperature
# read and the solution written (16 B).  The learned guess stores no
# temperature (the guess is recomputed from the state), so its algorithmic
# bytes are the state's alone; the guess array the guess kernel hands to
# the stage is an implementation choice and counts as traffic, not work.
BYTES_STATE_STAGE = 160.0
BYTES_T_STAGE = 16.0
# traffic the stage kernel adds on top (reported beside the roofline): the
# learned guess it reads from the guess kernel's array
BYTES_GUESS_ARRAY = 8.0
METRIC = "zone-updates/s (3D MHD 256^3) FP64 vs FP32+learned-EOS; % HBM roofline"
# the learned guess network 2 -> 64 -> 64 -> 1: multiply-adds per sample, and
# the dense BF16 matrix peak of the chip (TFLOP/s)
MLP_MACS = 2 * 64 + 64 * 64 + 64
BF16_MFMA_PEAK_TFLOPS = 2500.0

# HBM traffic of the stage kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs (average KiB per dispatch over the timed launches), keyed
# by the digest of the kernel sources the counters were taken on.  The
# factors scale the counters to bytes: a plain 1 GiB read + 1 GiB write
# kernel reads FETCH_SIZE = 0.5 GiB and WRITE_SIZE = 1 GiB on this chip.
FETCH_FACTOR = 2.0
WRITE_FACTOR = 1.0
TRAFFIC_KIB = {
    # digest: {path: (fetch KiB, write KiB) per stage dispatch}
    "3f5afaf1e16d1e30": {"fp64": (1363793.3, 1115010.8), "split": (1826299.1, 1218578.1)},
}


# VALU wave instructions per stage dispatch (SQ_INSTS_VALU summed over the
# chip, from profiles/stage_kernel_stratified256_issue_counters.md) for the
# digest of the stage sources.  At the chip's issue rate (1024 SIMDs, one
# wave64 instruction per four cycles, 2.4 GHz) they give the launch's
# instruction-issue floor: the bound the stage kernel actually meets.
VALU_INSTS = {
    "3f5afaf1e16d1e30": {"fp64": 863571147, "split": 596439887},
}
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4.0


# HBM traffic of diff_stage_kernel (FETCH_SIZE, WRITE_SIZE in KiB per
# dispatch, averaged over a super step) for the digest of its sources
RKL2_TRAFFIC_KIB = {
    "53f859047060231e": {"eint": (501489.2, 397803.5), "temp": (502686.9, 266731.5)},
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources each measured kernel is compiled from
STAGE_SOURCES = ("mhd_device.h", "mhd_internal.h", "mhd_kernels.hip")
DIFFUSION_SOURCES = ("mhd_device.h", "mhd_diffusion.hip", "mhd_internal.h")


def code_text(src: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed to one
    space: what the compiler sees, so that an edit of a comment does not
    count as a change of the kernel.  String and character literals are
    kept whole (a comment marker inside one is not a comment)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == "/" and i + 1 < n and src[i + 1] == "/":
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif c == "/" and i + 1 < n and src[i + 1] == "*":
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_digest(names=STAGE_SOURCES):
    """sha256 over the code text (comments and blank space removed) of the
    given HIP sources of the library, first 16 hex digits."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2604_12672_amd", "csrc")
    for name in sorted(names):
        with open(os.path.join(d, name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + code_text(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_bytes(path):
    t = TRAFFIC_KIB.get(kernel_digest(), {}).get(path)
    if t is None:
        return None
    return (t[0] * FETCH_FACTOR + t[1] * WRITE_FACTOR) * 1024.0


def gpu_run(mhd, w, precision, steps, warmup, mlp=None):
    """Whole-step throughput with mhd_advance (device dt, no host round
    trip), then the stage's duration from HIP events on the library's stream
    around fixed-dt steps: only the launches of the stages run between the
    events (the stage kernel, and the per-stage guess or flag kernels where
    the workload has them; timed_kernels names them)."""
    import torch
    guess = mhd.GUESS_MLP if mlp is not None else mhd.GUESS_PREV_T
    g = mhd.Grid(w.params, precision=precision, eos_guess=guess)
    g.load(w, mlp=mlp)
    stream = torch.cuda.current_stream()
    g.advance(w.cfl, warmup)
    g.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(w.cfl, steps)
    g.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    diag = g.diagnostics()
    dt = g.compute_dt(w.cfl)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    nrep = max(min(steps, 50), 4)
    e0.record(stream)
    for _ in range(nrep):
        g.step(dt)
    e1.record(stream)
    e1.synchronize()
    g.sync()
    stage_ms = e0.elapsed_time(e1) / (float(w.params.get("rk_order", 2)) * nrep)
    info = g.launch_info()
    flagged = float(g.shock_flags().mean()) if w.params.get("flatten") else None
    g.close()
    return {"wall": wall, "stage_ms": stage_ms, "diag": diag, "info": info,
            "ms": wall / steps * 1e3, "value": w.ncells * steps / wall, "learned": mlp is not None,
            "flagged": flagged}


def stage_bytes(w, learned):
    # SSP-RK with s stages: the first reads one state, the others two
    s = int(w.params.get("rk_order", 2))
    b = BYTES_STATE_STAGE if s == 2 else (128.0 + 192.0 * (s - 1)) / s
    if w.T is not None and not learned:
        b += BYTES_T_STAGE
    return b


def extra_bytes(w, learned):
    """Bytes per zone and stage the stage kernel moves beyond the
    algorithmic ones: the learned guess it reads (the guess kernel's
    output).  Forcing modes cost 120 B per column and launch (the
    coefficients of the column), under 4 B per zone at 37 planes per
    column segment, and are left out."""
    return BYTES_GUESS_ARRAY if (learned and w.T is not None) else 0.0


def timed_kernels(w, learned):
    """The launches between the HIP events of gpu_run's stage timing: the
    stage kernel, and per stage the learned-guess kernel (learned guess)
    and the pressure and flag passes (shock flattening)."""
    k = ["stage_kernel"]
    if learned and w.T is not None:
        k.append("mlp_guess_kernel")
    if w.params.get("flatten"):
        k += ["shock_pressure_kernel" if not learned else "mlp_guess_kernel (pressure)",
              "shock_flag_kernel"]
    return k


def roofline(w, stage_ms, path, learned=False):
    per_zone = stage_bytes(w, learned)
    per_launch = per_zone * w.ncells
    achieved = per_launch / (stage_ms * 1e-3) / 1e9
    tr = traffic_bytes(path)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if tr is None else round(tr),
           "kernel": "stage_kernel", "stage_ms": round(stage_ms, 4),
           "timed": timed_kernels(w, learned),
           "bytes_per_zone_stage": per_zone, "algorithmic_bytes_per_launch": round(per_launch)}
    xb = extra_bytes(w, learned)
    if xb:
        out["implementation_bytes_per_zone_stage"] = xb
    n = VALU_INSTS.get(kernel_digest(), {}).get(path)
    if n is not None:
        floor_ms = n / VALU_ISSUE_PER_S * 1e3
        out["valu_issue"] = {"wave_insts_per_launch": n, "floor_ms": round(floor_ms, 4),
                             "frac": round(floor_ms / stage_ms, 4)}
    return out


def hbm_target(w, ms, learned=False, frac=0.6):
    """The step against one whose stage launches move their algorithmic bytes
    at `frac` of the HBM peak."""
    stages = int(w.params.get("rk_order", 2))
    t = stages * stage_bytes(w, learned) * w.ncells / (frac * HBM_PEAK_GBS * 1e9) * 1e3
    return {"hbm_fraction": frac, "ms_per_step_at_that_fraction": round(t, 4),
            "ms_per_step": round(ms, 4), "ratio": round(ms / t, 2)}


def newton_stats(w, diag, stages=2):
    """Newton statistics of the last step (all its stages)."""
    return {"newton_steps_per_cell_stage": round(diag["newton_iters"] / (w.ncells * stages), 3),
            "newton_max": diag["newton_max"], "fallback_cell_stages": diag["fallbacks"]}


def eos_bench(mhd, model, n):
    """Batch inversion of n iid (rho, T) samples log-uniform over the
    gas+radiation range: learned guess + Newton polish against the bracketed
    solve, both on the device (HIP events around each call)."""
    import numpy as np
    import torch
    from paper_2604_12672_amd import workloads as wl
    p = wl.gasrad_params(4, 4, 4)
    rho, T = wl.eos_samples(n)
    _, e = wl.gasrad_forward(p, rho, T)
    r = torch.from_numpy(rho).cuda()
    ee = torch.from_numpy(e).cuda()
    out = {}
    for name, guess in (("learned", mhd.GUESS_MLP), ("bracketed", mhd.GUESS_PREV_T)):
        g = mhd.Grid(p, eos_guess=guess)
        if guess == mhd.GUESS_MLP:
            g.set_eos_mlp(model)
        # statistics and guesses from one synchronised call; the rate from
        # asynchronous calls between HIP events on the library's stream
        Td, T0, st = g.eos_solve(r, ee, with_guess=(guess == mhd.GUESS_MLP))
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        scratch = torch.empty_like(r)
        e0.record(stream)
        for _ in range(reps):
            g.eos_solve(r, ee, stats=False, out=scratch)
        e1.record(stream)
        e1.synchronize()
        g.sync()
        ms = e0.elapsed_time(e1) / reps
        g.close()
        Th = Td.cpu().numpy()
        res = {"ms": round(ms, 4), "solves_per_s": round(n / (ms * 1e-3), 1),
               "newton_steps_per_cell": round(st[0] / n, 3), "newton_max": int(st[1]),
               "bracketed_solves": int(st[2]),
               "max_rel_err_vs_exact_T": float(np.max(np.abs(Th - T) / T))}
        if T0 is not None:
            d = np.abs(np.log10(T0.cpu().numpy()) - np.log10(T))
            res["guess_mean_abs_dlog10T"] = float(d.mean())
            res["guess_max_abs_dlog10T"] = float(d.max())
            # the network's matrix work: 4 288 multiply-adds per sample
            # (64 x 64 + 64 x 2 + 64), priced against the BF16 MFMA peak; the
            # timed call also runs the FP64 Newton polish, so this is a lower
            # bound on the rate of the matrix passes themselves
            tf = 2.0 * MLP_MACS * n / (ms * 1e-3) / 1e12
            res["mfma_roofline"] = {"bound": "mfma", "achieved": round(tf, 2),
                                    "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4),
                                    "flop_per_sample": 2 * MLP_MACS,
                                    "note": "network + Newton polish in the timed call"}
        out[name] = res
        log(f"bench: eos {name}: {res}")
    out["speedup_learned_vs_bracketed"] = round(out["bracketed"]["ms"] / out["learned"]["ms"], 3)
    out["samples"] = f"{n} iid (rho, T) log-uniform over [1e-2, 1e2] x [1e5, 1e8] K"
    return out


def _rel_l2(a, b):
    """||a - b|| / ||b||, or ||a|| where the reference field is zero."""
    import numpy as np
    den = float(np.sqrt(np.sum(b * b)))
    num = float(np.sqrt(np.sum((a - b) ** 2)))
    return num / den if den > 0 else num


FIELD_NAMES = [("U", 0, "rho"), ("U", 1, "m_x"), ("U", 2, "m_y"), ("U", 3, "m_z"), ("U", 4, "E"),
               ("Bx", None, "B_x"), ("By", None, "B_y"), ("Bz", None, "B_z")]


def split_error(mhd, n, steps):
    """Per-field rel L2 of the split path (and of the FP64 path) against the
    FP64 oracle after `steps` steps of the stratified box with heating and
    cooling (the 512^3 workload's recipe at n^3, where the oracle takes
    seconds on the host), both GPU paths on the oracle's dt sequence."""
    from oracle import orc
    from paper_2604_12672_amd import workloads as wl
    w = wl.stratified_box(n, heating=True, steps=steps)
    o = orc.Oracle(w.params, **w.extras())
    ref = w.state()
    dts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        dt = o.compute_dt(ref, w.cfl)
        o.step(ref, dt)
        dts.append(dt)
    oracle_s = time.perf_counter() - t0
    res = {}
    for name, prec in (("split", mhd.PREC_SPLIT), ("fp64", mhd.PREC_FP64)):
        g = mhd.Grid(w.params, precision=prec)
        g.load(w)
        for dt in dts:
            g.step(dt)
        out = g.get_state()
        d = g.diagnostics()
        g.close()
        errs = {}
        for key, c, fname in FIELD_NAMES:
            a = out[key] if c is None else out[key][c]
            b = ref[key] if c is None else ref[key][c]
            errs[fname] = _rel_l2(a, b)
        res[name] = {"rel_l2_vs_oracle": errs,
                     "max_rel_l2": max(v for v in errs.values() if v is not None),
                     "divb_max": d["divb_max"]}
    res.update({"grid": [n, n, n], "steps": steps,
                "reference": f"FP64 oracle on the host ({oracle_s:.1f} s), same dt sequence",
                "workload": f"stratified box {n}^3 with heating and cooling (q = 1e-6 of the "
                            f"energy flux in the bottom and top 10 %)"})
    return res


def learned_error(mhd, model, steps):
    """The FP32+learned-EOS step against the FP64 oracle after `steps`
    steps on the workloads with the learned guess: the gas + radiation box
    (config 3's recipe) at 64^3 and the forced Mach-3 turbulence box
    (config 4's recipe) at 48^3, sizes at which the host oracle takes
    seconds; the GPU on the oracle's dt sequence."""
    from oracle import orc
    from paper_2604_12672_amd import workloads as wl
    out = {}
    for name, w in (("gasrad_64", wl.gasrad_box(64)), ("turbulence_48", wl.turbulence_box(48))):
        o = orc.Oracle(w.params, **w.extras())
        ref = w.state()
        dts = []
        t0 = time.perf_counter()
        for _ in range(steps):
            dt = o.compute_dt(ref, w.cfl)
            o.step(ref, dt)
            dts.append(dt)
        oracle_s = time.perf_counter() - t0
        g = mhd.Grid(w.params, precision=mhd.PREC_SPLIT, eos_guess=mhd.GUESS_MLP)
        g.load(w, mlp=model)
        for dt in dts:
            g.step(dt)
        st = g.get_state()
        d = g.diagnostics()
        g.close()
        errs = {}
        for key, c, fname in FIELD_NAMES:
            a = st[key] if c is None else st[key][c]
            b = ref[key] if c is None else ref[key][c]
            errs[fname] = _rel_l2(a, b)
        out[name] = {"steps": steps, "rel_l2_vs_oracle": errs,
                     "max_rel_l2": max(v for v in errs.values() if v is not None),
                     "divb_max": d["divb_max"], "fallback_cell_stages_last_step": d["fallbacks"],
                     "oracle_s": round(oracle_s, 1)}
    out["path"] = "split precision with the learned EOS guess, FP64 oracle on the host as reference"
    return out


# algorithmic bytes per cell of one RKL2 stage j >= 2.  Internal-energy form:
# reads y_(j-1), y_(j-2), y_0, M_0, rho, and T and chi of the previous stage
# (7 x 8 B), writes y_j, T, chi (3 x 8 B).  Temperature form: the stage value
# is T, so it reads y_(j-1), y_(j-2), y_0, M_0, c_v0, rho, chi (7 x 8 B) and
# writes y_j and chi (2 x 8 B).
BYTES_RKL2_STAGE = {0: 80.0, 1: 72.0}


def rkl2_traffic(mode_name):
    t = RKL2_TRAFFIC_KIB.get(kernel_digest(DIFFUSION_SOURCES), {}).get(mode_name)
    if t is None:
        return None
    return (t[0] * FETCH_FACTOR + t[1] * WRITE_FACTOR) * 1024.0


def rkl2_bench(mhd, n):
    """One RKL2 super step of thermal diffusion on the gas+radiation box
    (n^3) with a Kramers-like opacity, dt = 100 parabolic limits (the
    paper's stage count for that ratio), in both forms.  HIP events on the
    library's stream around the asynchronous calls; the stage time is the
    super step of 2s stages over 2s."""
    import torch
    from paper_2604_12672_amd import workloads as wl
    w = wl.config(3, n)
    res = {}
    for name, mode in (("eint", mhd.DIFF_EINT), ("temp", mhd.DIFF_TEMP)):
        g = mhd.Grid(w.params)
        g.load(w)
        g.set_opacity(0.2, alpha=1.0, beta=-3.5)
        dtp = g.parabolic_dt()
        dt = 100.0 * dtp
        s = g.diffuse(dt, 0, mode)  # warm-up, allocation, stage count
        g.sync()
        stream = torch.cuda.current_stream()

        def timed(nst, reps=3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                g.diffuse(dt, nst, mode)
            e1.record(stream)
            e1.synchronize()
            g.sync()
            return e0.elapsed_time(e1) / reps

        ms = timed(s)
        ms2 = timed(2 * s)
        g.close()
        # average stage duration over super steps of 2s stages, the set-up
        # and finishing kernels included (they add about 4 %): the figure a
        # kernel trace of the same calls averages to
        stage_ms = ms2 / (2 * s)
        bpc = BYTES_RKL2_STAGE[mode]
        achieved = bpc * w.ncells / (stage_ms * 1e-3) / 1e9
        tr = rkl2_traffic(name)
        res[name] = {"stages": s, "ms_per_super_step": round(ms, 4),
                     "ms_per_stage": round(stage_ms, 4),
                     "ms_per_added_stage": round((ms2 - ms) / s, 4),
                     "cell_stages_per_s": round(w.ncells / (stage_ms * 1e-3), 1),
                     "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(achieved / HBM_PEAK_GBS, 4),
                                  "traffic": None if tr is None else round(tr),
                                  "kernel": "diff_stage_kernel<%s>" % ("true" if mode == mhd.DIFF_TEMP else "false"),
                                  "bytes_per_cell_stage": bpc}}
        log(f"bench: rkl2 {name}: {s} stages, {ms:.3f} ms per super step, "
            f"{stage_ms:.4f} ms per stage")
    res["workload"] = (f"gas+radiation box {n}^3, kappa = 0.2 rho T^-3.5, one RKL2 super "
                       f"step of 100 parabolic limits")
    return res


def host_cpu():
    """The host CPU the oracle runs on: model name, logical CPUs this
    process may use, and physical cores (distinct core/socket pairs of those
    CPUs, from /proc/cpuinfo)."""
    model, cores = None, set()
    allowed = os.sched_getaffinity(0)
    try:
        proc, phys, core = None, None, None
        with open("/proc/cpuinfo") as f:
            for line in f.read().splitlines() + [""]:
                if not line.strip():
                    if proc is not None and proc in allowed:
                        cores.add((phys, core))
                    proc, phys, core = None, None, None
                    continue
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    proc = int(v)
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif k == "model name" and model is None:
                    model = v
    except OSError:
        pass
    return {"model": model, "logical_cpus_available": len(allowed),
            "physical_cores_available": len(cores) if cores else None}


def cpu_baseline(n, steps=2, runs=3):
    """The FP64 oracle on the host cores on the headline workload (the
    stratified box at n^3): `runs` timed runs of `steps` SSP-RK2 steps each
    (CFL step included), median, after one untimed step; plus one core on a
    48^3 box for scale against per-core CPU figures."""
    import statistics

    from oracle import orc
    from paper_2604_12672_amd import workloads as wl
    w = wl.stratified_box(n)
    o = orc.Oracle(w.params, **w.extras())
    st = w.state()
    o.step(st, o.compute_dt(st, w.cfl))  # warm-up (page-in, thread start)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step(st, o.compute_dt(st, w.cfl))
        times.append(time.perf_counter() - t0)
    el = statistics.median(times)
    threads = orc.num_threads()
    out = {"value": round(w.ncells * steps / el, 1), "unit": "zone-updates/s",
           "cores": threads, "kind": "oracle",
           "sample": (f"stratified box {n}^3 (the headline recipe), {steps} SSP-RK2 steps "
                      f"incl. CFL per run, median of {runs} runs "
                      f"({', '.join(f'{t:.2f}' for t in times)} s), {threads} OpenMP threads"),
           "host": host_cpu()}
    del o, st, w
    orc.set_num_threads(1)
    try:
        w1 = wl.stratified_box(48)
        o1 = orc.Oracle(w1.params, **w1.extras())
        s1 = w1.state()
        o1.step(s1, o1.compute_dt(s1, w1.cfl))
        k1 = 0
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < 4.0:
            o1.step(s1, o1.compute_dt(s1, w1.cfl))
            k1 += 1
        e1 = time.perf_counter() - t1
    finally:
        orc.set_num_threads(threads)
    out["single_core"] = {"value": round(w1.ncells * k1 / e1, 1), "unit": "zone-updates/s",
                          "us_per_cell_step": round(e1 / (w1.ncells * k1) * 1e6, 3),
                          "sample": f"stratified box 48^3, 1 thread, {k1} steps, {e1:.1f} s"}
    return out


def stream_ceiling():
    """Measured copy bandwidth of the device: a 2 GiB torch copy (2 GiB read,
    2 GiB written), best of five, HIP events."""
    import torch
    a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 2 ** 31 / (best * 1e-3) / 1e9


def host_transfer(mhd, w):
    """Seconds to hand the state over from host memory (mhd_set_state with
    host pointers) and back (mhd_get_state to host), for the PCIe-inclusive
    rate; the headline value keeps the state resident in HBM."""
    import torch
    g = mhd.Grid(w.params, precision=mhd.PREC_FP64)
    if w.bg_cc is not None:
        g.set_background(w.bg_cc, w.bg_fz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.set_state(w.U, w.Bx, w.By, w.Bz)
    g.sync()
    t1 = time.perf_counter()
    g.get_state()
    t2 = time.perf_counter()
    g.close()
    return t1 - t0, t2 - t1


def summary(w, r, path):
    return {"value": round(r["value"], 1), "ms_per_step": round(r["ms"], 4),
            "roofline": roofline(w, r["stage_ms"], path, r["learned"]), "divb_max": r["diag"]["divb_max"]}


def turbulence_bench(mhd, model, args):
    """Config 4 (forced MHD turbulence, learned guess, split precision),
    without and with shock flattening."""
    from paper_2604_12672_amd import workloads as wl
    log(f"bench: turbulence box {args.turb_n}^3")
    wt = wl.turbulence_box(args.turb_n)
    tr = gpu_run(mhd, wt, mhd.PREC_SPLIT, args.steps, args.warmup, mlp=model)
    t = dict(summary(wt, tr, "turbulence_split_learned"), **newton_stats(wt, tr["diag"]))
    t["workload"] = (f"forced MHD turbulence {args.turb_n}^3, rms Mach 3, beta 1, "
                     f"gas+radiation, learned guess, split precision")
    log(f"bench: turbulence {tr['ms']:.3f} ms/step, divB {tr['diag']['divb_max']:.2e}")
    # the same run with shock flattening: flags of every stage input
    # (pressure, detector, 5x5x5 dilation), HLL and van Leer where flagged
    wt.params = dict(wt.params, flatten=1)
    tf = gpu_run(mhd, wt, mhd.PREC_SPLIT, args.steps, args.warmup, mlp=model)
    tflat = {
        "value": round(tf["value"], 1), "ms_per_step": round(tf["ms"], 4),
        "overhead_vs_unflattened": round(tf["ms"] / tr["ms"] - 1.0, 4),
        "flagged_fraction_at_end": round(tf["flagged"], 5),
        "divb_max": tf["diag"]["divb_max"],
        "workload": t["workload"] + ", shock flattening (eps_SF 0.2)"}
    log(f"bench: turbulence flattened {tf['ms']:.3f} ms/step, flagged {tf['flagged']:.4f}")
    return t, tflat


def blast_bench(mhd, n, steps, warmup):
    """A pressure-jump box with flattening active where it matters: the
    smooth random box with the pressure raised tenfold in a sphere of radius
    0.25, PPH + SSP-RK3 at CFL 0.4, shock flattening on, FP64 and split."""
    from paper_2604_12672_amd import workloads as wl
    log(f"bench: flattened blast box {n}^3")
    w = wl.smooth_box(n, n, n, blast=(10.0, 0.25))
    w.params = dict(w.params, flatten=1, recon=mhd.RECON_PPH, rk_order=3)
    w.cfl = 0.4
    res = {}
    for name, prec in (("fp64", mhd.PREC_FP64), ("split", mhd.PREC_SPLIT)):
        r = gpu_run(mhd, w, prec, steps, warmup)
        res[name] = {"value": round(r["value"], 1), "ms_per_step": round(r["ms"], 4),
                     "flagged_fraction_at_end": round(r["flagged"], 5),
                     "divb_max": r["diag"]["divb_max"]}
        log(f"bench: blast {name} {r['ms']:.3f} ms/step, flagged {r['flagged']:.4f}")
    res["workload"] = (f"smooth random MHD box {n}^3 with a tenfold pressure sphere "
                       f"(r = 0.25), PPH + SSP-RK3, CFL 0.4, shock flattening")
    return res


# algorithmic bytes per cell of one species-kernel launch with ns species in
# SSP-RK3 (stages 2 and 3 also read the step base): rho X^(s), rho, the three
# face mass fluxes, 2/3 of rho X^n, the flag byte when flattening; rho X out
def species_bytes(ns, rk=3, flat=False):
    base = (rk - 1) / rk
    return 8.0 * ns + 8.0 + 24.0 + base * 8.0 * ns + (1.0 if flat else 0.0) + 8.0 * ns


def species_bench(mhd, n, steps, warmup, ns=12):
    """The paper's production scheme with ns passive species on the
    stratified box: PPH (limited parabola for the fractions) + SSP-RK3 at
    CFL 0.8, FP64 and split; the species kernel's duration from HIP events
    around its own launches is not separable from the stage here, so its
    share is the difference to the same run without species."""
    from paper_2604_12672_amd import workloads as wl
    log(f"bench: {ns} species, stratified box {n}^3, PPH + SSP-RK3")
    w0 = wl.stratified_box(n, cfl=0.8)
    w0.params = dict(w0.params, recon=mhd.RECON_PPH, rk_order=3)
    w = wl.add_species(w0, ns)
    res = {}
    for name, prec in (("fp64", mhd.PREC_FP64), ("split", mhd.PREC_SPLIT)):
        r = gpu_run(mhd, w, prec, steps, warmup)
        r0 = gpu_run(mhd, w0, prec, steps, warmup)
        per_stage = (r["ms"] - r0["ms"]) / 3.0
        ach = species_bytes(ns) * w.ncells / (per_stage * 1e-3) / 1e9
        res[name] = {"value": round(r["value"], 1), "ms_per_step": round(r["ms"], 4),
                     "ms_per_step_without_species": round(r0["ms"], 4),
                     "species_ms_per_stage": round(per_stage, 4),
                     "species_roofline": {"bound": "hbm", "achieved": round(ach, 1),
                                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": round(ach / HBM_PEAK_GBS, 4),
                                          "bytes_per_cell_stage": round(species_bytes(ns), 1),
                                          "note": "species kernel + the stage's mass-flux "
                                                  "writes, from the step-time difference"}}
        log(f"bench: species {name} {r['ms']:.3f} ms/step (without {r0['ms']:.3f})")
    res["workload"] = (f"stratified MHD box {n}^3 with {ns} passive species (smooth random "
                       f"fractions), PPH + SSP-RK3, CFL 0.8")
    res["paper_context"] = ("PPH + LHLLD + SSP-RK3 with 12 species: 1.03 us per cell-step "
                            "on one EPYC 9554 core, about 9.7e5 zone-updates/s per core")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="linear grid size of the headline box")
    ap.add_argument("--only", choices=["fp64", "split", "rkl2", "turbulence", "blast",
                                       "species"],
                    default=None,
                    help="run only this path of the headline box, or only the RKL2 "
                         "diffusion or the turbulence measurement (profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline box only (no gas+radiation, EOS, 512^3, turbulence)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=256)
    ap.add_argument("--eos-n", type=int, default=256 ** 3)
    ap.add_argument("--split-n", type=int, default=128)
    ap.add_argument("--split-steps", type=int, default=50)
    ap.add_argument("--turb-n", type=int, default=384)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_12672_amd import eos_mlp
    from paper_2604_12672_amd import mhd
    from paper_2604_12672_amd import workloads as wl
    if not os.path.exists(mhd.LIB_PATH):
        from paper_2604_12672_amd import build
        build.build()
    mhd.load()
    torch.cuda.set_device(0)
    n = args.n
    if args.only == "turbulence":
        t, tf = turbulence_bench(mhd, eos_mlp.MLPGuess.load(), args)
        print(json.dumps({"turbulence": t, "turbulence_flattened": tf}), flush=True)
        return
    if args.only == "species":
        print(json.dumps({"species": species_bench(mhd, n, args.steps, args.warmup)}),
              flush=True)
        return
    if args.only == "blast":
        print(json.dumps({"blast_flattened": blast_bench(mhd, n, args.steps, args.warmup)}),
              flush=True)
        return
    if args.only == "rkl2":
        print(json.dumps({"rkl2_diffusion": rkl2_bench(mhd, n),
                          "kernel_sources": kernel_digest(DIFFUSION_SOURCES)}), flush=True)
        return
    log(f"bench: stratified box {n}^3 (kernel sources {kernel_digest()})")
    w = wl.stratified_box(n)
    res = {}
    for name, prec in (("fp64", mhd.PREC_FP64), ("split", mhd.PREC_SPLIT)):
        if args.only and args.only != name:
            continue
        log(f"bench: {name} warmup={args.warmup} steps={args.steps}")
        r = gpu_run(mhd, w, prec, args.steps, args.warmup)
        res[name] = r
        log(f"bench: {name} {r['ms']:.3f} ms/step, stage {r['stage_ms']:.3f} ms, "
            f"divB {r['diag']['divb_max']:.2e}")
    if args.calib_copy:
        # plain streaming kernel of known size: reads 2^30 bytes, writes 2^30
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log("bench: calibration copy of 1 GiB done")
    main_name = "fp64" if "fp64" in res else "split"
    r = res[main_name]
    out = {
        "metric": METRIC, "value": round(r["value"], 1), "unit": "zone-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"stratified MHD box {n}^3 (n=1.5 polytrope, 4 H_P, 1e-4 density "
                               f"noise, beta 1e6 seed field, periodic x/y, reflecting z), SSP-RK2, "
                               f"CFL {w.cfl}, van Leer + LHLLD + Contact-CT, ideal gas, "
                               f"{main_name} path",
                   "cells": w.ncells, "grid": [n, n, n], "precision": main_name,
                   "launch": r["info"], "kernel_sources": kernel_digest()},
        "roofline": roofline(w, r["stage_ms"], main_name),
        "divb_max": r["diag"]["divb_max"],
        # the paper's own scaling, on its CPU hardware (context only: one GPU
        # here, no scaling measured)
        "paper_scaling_context": (
            "weak scaling of the MPI CPU code (Sect. 2, code scaling): 64 -> 32768 "
            "Intel Xeon Ice Lake 2.4 GHz cores on HoreKa, parallel efficiency lower by "
            "about 24 % with 32^3 cells per core and about 15 % with 64^3 cells per core"),
    }
    ceil = stream_ceiling()
    out["roofline"]["measured_copy_GBs"] = round(ceil, 1)
    out["roofline"]["frac_of_measured_copy"] = round(out["roofline"]["achieved"] / ceil, 4)
    log(f"bench: device copy ceiling {ceil:.0f} GB/s")
    t_in, t_out = host_transfer(mhd, w)
    out["pcie_inclusive"] = {
        "set_state_host_s": round(t_in, 4), "get_state_host_s": round(t_out, 4),
        "value": round(w.ncells * args.steps / (r["wall"] + t_in + t_out), 1),
        "note": f"{args.steps} steps with the state handed over from and back to host memory"}
    if not args.no_extras and not args.only:
        # the paper's production scheme: PPH reconstruction, SSP-RK3, CFL 0.8
        wp = wl.stratified_box(n, cfl=0.8)
        wp.params = dict(wp.params, recon=mhd.RECON_PPH, rk_order=3)
        log("bench: PPH + SSP-RK3 (CFL 0.8), fp64 and split")
        pp = {}
        for name, prec in (("fp64", mhd.PREC_FP64), ("split", mhd.PREC_SPLIT)):
            r3 = gpu_run(mhd, wp, prec, args.steps, args.warmup)
            pp[name] = summary(wp, r3, "pph_rk3_" + name)
            log(f"bench: pph rk3 {name} {r3['ms']:.3f} ms/step, stage {r3['stage_ms']:.3f} ms")
        pp["workload"] = (f"stratified MHD box {n}^3 as the headline, PPH reconstruction, "
                          f"SSP-RK3, CFL 0.8 (the paper's production scheme)")
        pp["paper_context"] = ("PPH + LHLLD + SSP-RK3 with 12 species: 1.03 us per cell-step "
                               "on one EPYC 9554 core, about 9.7e5 zone-updates/s per core")
        res["pph_rk3"] = pp
        del wp
    if "split" in res and main_name == "fp64":
        s = summary(w, res["split"], "split")
        s["dtype"] = "f32 recon/flux/EMF on deviations, f64 background/accumulation"
        s["speedup_vs_fp64"] = round(r["ms"] / res["split"]["ms"], 3)
        out["split"] = s
    if "pph_rk3" in res:
        out["pph_rk3"] = res["pph_rk3"]
    del w
    if not args.no_extras and not args.only:
        model = eos_mlp.MLPGuess.load()
        # gas + radiation box: plain FP64 step (previous-T guess) against the
        # split step with the learned guess
        log("bench: gas+radiation box 256^3")
        wg = wl.config(3)
        g64 = gpu_run(mhd, wg, mhd.PREC_FP64, args.steps, args.warmup)
        gsp = gpu_run(mhd, wg, mhd.PREC_SPLIT, args.steps, args.warmup)
        gml = gpu_run(mhd, wg, mhd.PREC_SPLIT, args.steps, args.warmup, mlp=model)
        gas = {"fp64_prev_t": dict(summary(wg, g64, "gasrad_fp64"), **newton_stats(wg, g64["diag"])),
               "split_prev_t": dict(summary(wg, gsp, "gasrad_split"), **newton_stats(wg, gsp["diag"])),
               "split_learned": dict(summary(wg, gml, "gasrad_split_learned"),
                                     **newton_stats(wg, gml["diag"])),
               "speedup_split_learned_vs_fp64": round(g64["ms"] / gml["ms"], 3),
               "split_learned_vs_60pct_hbm": hbm_target(wg, gml["ms"], learned=True),
               "learned_guess_kernel": "one MFMA guess kernel per stage (reads U and B, "
                                       "writes the guess array the stage reads)",
               "workload": "gas+radiation box 256^3, log-uniform rho in [1e-2, 1e2] and "
                           "T in [1e5, 1e8] K, beta 1e6, periodic"}
        out["gasrad"] = gas
        log(f"bench: gasrad fp64 {g64['ms']:.3f} ms/step, split {gsp['ms']:.3f}, "
            f"split+learned {gml['ms']:.3f} ms/step")
        del wg
        log("bench: batch EOS inversion")
        out["eos_solve"] = eos_bench(mhd, model, args.eos_n)
        log(f"bench: split error, stratified box {args.split_n}^3 with heating, "
            f"{args.split_steps} steps")
        out["split_error"] = split_error(mhd, args.split_n, args.split_steps)
        log(f"bench: split error vs oracle {out['split_error']['split']['rel_l2_vs_oracle']}")
        log("bench: split + learned against the oracle, gas+radiation 64^3 and turbulence 48^3")
        out["learned_split_error"] = learned_error(mhd, model, args.split_steps)
        out["turbulence"], out["turbulence_flattened"] = turbulence_bench(mhd, model, args)
    if not args.no_extras and not args.only:
        out["blast_flattened"] = blast_bench(mhd, args.n, args.steps, args.warmup)
        out["species"] = species_bench(mhd, args.n, args.steps, args.warmup)
        out["rkl2_diffusion"] = rkl2_bench(mhd, args.n)
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle) {args.cpu_n}^3")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
