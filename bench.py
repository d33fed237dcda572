"""Benchmark: pair evaluations per second of the adaptive-resolution WCSPH
step on one MI355X, FP32 pair arithmetic vs plain FP64, and the batched
serving path.

Main workload (synthetic, seeded): the channel with a circular cylinder (D = 1,
30D x 20D, periodic in y, inflow U = 1 through an inlet buffer with the
characteristic inlet/outlet rule, finest spacing D/100, sizes graded by
C_r = 1.05 per layer, h/dx = 1.2, Re = 100, wall particles inside the
cylinder), ~2e5 particles, with a prescribed background (section 3.3 lets
the reference mass be assigned directly) that follows the fluid's grading.
Before timing, the fluid is adapted four times to the background.  The
configuration lines add the same channel adapted to the background the
library builds from ds_max (3 ceil(ln 64 / ln C_r) = 258 passes of the
background update; its grading is steeper and the fluid ends near 2.5e4
particles), and the oscillating cylinder starting from its built background.  The timed loop is the library's per-iteration schedule
(sph_step, the algorithm of section 3.4): one predict-evaluate-correct step
(two rate evaluations) and the inlet/outlet update per iteration, and every
`--adapt-every` iterations the adaptation (m_ref from the background, split,
merge x3, shift x3, h update).  dt is eq. (timestep) from the library.
One pair evaluation is one ordered pair (i, j != i) with j in N(i),
processed by pass A and pass B in one rate evaluation: a step has 2 (nnz - n)
of them.  Adaptation time is included in the step time.

Prints ONE JSON line; `value` is the FP32 path's pair-evals/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair evals/s per step, FP32 vs FP64 plain; batched-serve p50/p99 step latency"
# Algorithmic work per unit of the two rate passes (the per-term tallies are
# in the design notes): pass A (summation density, beta, p_avg, limited
# shifting, compensated sums) 105 flops per interacting pair and 52 bytes of
# HBM per particle; pass B (EDAC pressure rate, momentum) 125 flops per pair
# and 68 bytes per particle.
PASS_FLOPS_PER_PAIR = {"pass_a": 105, "pass_b": 125}
PASS_BYTES_PER_PARTICLE = {"pass_a": 52, "pass_b": 68}
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
ADAPT_WARM = 4
PROF_EVERY = 4
BG_CAPACITY = 4_000_000


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--adapt-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-evals", type=int, default=20)
    ap.add_argument("--cpu-evals-single", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--serve-arena-gib", type=float, default=4.0)
    ap.add_argument("--serve-skin", type=float, default=0.1,
                    help="list skin of the served simulations (0: a list per evaluation)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the C1 latency and the 1.5e6 / 9.6e5 particle lines")
    ap.add_argument("--schedule", type=str, default=None,
                    help="a_lanes,a_waves,b_lanes,b_unroll,b_waves,list_lanes for the FP32 "
                         "run instead of tuning (for profiled runs)")
    ap.add_argument("--no-tune-cache", action="store_true",
                    help="time the kernel schedules even when the tuning cache holds a pick")
    ap.add_argument("--list-skin", type=float, default=None,
                    help="use this list skin for both precisions instead of timing the "
                         "candidates first (for profiled runs)")
    ap.add_argument("--serve-only", action="store_true",
                    help="for profiled runs: only the serving loop (saturated), printing its "
                         "figures")
    ap.add_argument("--bg-pass-only", action="store_true",
                    help="for profiled runs: build the oscillating cylinder's background and "
                         "time five background passes, printing their figures")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="for hardware-counter runs: a calibration copy of known size, then "
                         "the timed loop's first steps (FP32, --list-skin); prints nothing else")
    return ap.parse_args()


CALIB_BYTES = 1 << 29  # bytes read (and written) by the calibration copy
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rate_passes_channel_traffic.md")
KERNEL_SOURCES = ("paper_2107_01276_amd/csrc/rates.hip", "paper_2107_01276_amd/csrc/sph_device.h",
                  "paper_2107_01276_amd/csrc/sph_internal.h")


def kernel_source_hash():
    """sha256 of the sources the rate passes are compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of each rate pass from the committed counter
    summary, or None when the kernels' sources changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    f = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
             and line.split(": ", 1)[0] in ("kernel_source_sha256", "pass_a_bytes_per_launch",
                                             "pass_b_bytes_per_launch"))
    if f.get("kernel_source_sha256", "").strip() != kernel_source_hash():
        return None
    return {"pass_a": float(f["pass_a_bytes_per_launch"]),
            "pass_b": float(f["pass_b_bytes_per_launch"])}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def procedure_background(SPH, W, s, torch):
    """The background of section 3.3 as the library builds it: a lattice at
    ds_max, then sph_bg_init_passes passes of sph_bg_update around the
    body's solid particles.  Returns the background (host arrays) and what
    the build took."""
    spec = s["spec"]
    ds_max = spec.ds_min * spec.ratio
    bg0 = W.background_lattice(s["domain"], ds_max, 1.2, spec.rho0)
    d = s["domain"]
    cfg = SPH.Config(lo=d.lo, hi=d.hi, periodic=d.periodic, h_lo=0.25 * spec.ds_min,
                     h_hi=2.5 * ds_max, cr=spec.cr, ds_min=spec.ds_min, ds_max=ds_max,
                     bg_mass_q=bg0["mass_q"], mass_q=s["mass_q"])
    ctx = SPH.Context(cfg, BG_CAPACITY)
    B = SPH.Background.from_arrays(bg0, BG_CAPACITY)
    sol = s["kind"] == W.SOLID
    S = SPH.Particles.from_arrays({k: s[k][sol] for k in ("x", "y", "h", "mq")})
    passes = SPH.bg_init_passes(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nsplit = ctx.bg_update(B, S, passes)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    bg = B.numpy()
    bg["mass_q"] = bg0["mass_q"]
    del ctx, B, S
    torch.cuda.empty_cache()
    return bg, {"passes": passes, "n_start": int(bg0["x"].size), "n": int(bg["x"].size),
                "splits": nsplit, "build_ms": ms, "ds_min": spec.ds_min, "ds_max": ds_max,
                "cr": spec.cr}


def fluid_size_ratio(P, W):
    """Largest over smallest fluid spacing sqrt(m / rho0) of the state."""
    st = P.numpy()
    m = st["mq"][st["kind"] == W.FLUID].astype(float)
    return float((m.max() / m.min()) ** 0.5)


def channel_cfg(SPH, s, bg, prec, skin, adapt_every):
    h_hi = max(float(s["h"].max()), float(bg["h"].max()))
    return SPH.config_for(s["domain"], s["params"], float(s["h"].min()), h_hi, precision=prec,
                          mass_q=s["mass_q"], list_skin=skin, n_adapt=adapt_every)


def prepare(SPH, s, bg, prec, capacity, skin, adapt_every):
    cfg = channel_cfg(SPH, s, bg, prec, skin, adapt_every)
    ctx = SPH.Context(cfg, capacity)
    P = SPH.Particles.from_arrays(s, capacity)
    B = SPH.Background.from_arrays(bg, bg["x"].size)
    for _ in range(ADAPT_WARM):
        ctx.adapt(P, B)
    return ctx, P, B


def count_pairs(ctx, P):
    rp, col = ctx.build_neighbors(P)
    return int(col.numel()) - P.n


def run(ctx, P, B, io, steps, warmup, torch):
    """warmup + timed iterations of the schedule (one library call each)."""
    ctx.run(P, warmup, bg=B, io=io)
    torch.cuda.synchronize()
    pairs0 = count_pairs(ctx, P)
    # the rate passes are bracketed with events in the timed region, every
    # PROF_EVERY-th launch (event markers serialise the kernels around them,
    # so sparse sampling keeps the timed work closer to unprofiled)
    ctx.profile(True, kernels=("pass_a", "pass_b"), every=PROF_EVERY)
    ctx.profile_reset()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(ctx.stream)
    ctx.run(P, steps, bg=B, io=io)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = {k: ctx.profile_read(k) for k in ("pass_a", "pass_b", "build", "list")}
    ctx.profile(False)
    pairs1 = count_pairs(ctx, P)
    return ms, prof, 0.5 * (pairs0 + pairs1)


def pmc_sample(SPH, W, torch, skin, adapt_every, sched=None):
    """One plain device copy of CALIB_BYTES (its FETCH_SIZE / WRITE_SIZE give
    the counter-to-bytes factor), then 10 iterations of the timed loop (FP32)
    on the adapted channel: the rate-pass dispatches whose traffic is
    measured."""
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    s = W.channel_cylinder(seed=2)
    bg = W.channel_background(s["spec"], seed=3)
    ctx, P, B = prepare(SPH, s, bg, SPH.SPH_FP32, int(1.6 * s["x"].size), skin, adapt_every)
    if sched:
        ctx.set_schedule(**sched)
    ctx.run(P, 10, bg=B, io=s["io"])
    torch.cuda.synchronize()
    print(json.dumps({"pmc_sample": True, "calib_bytes": CALIB_BYTES, "n": P.n, "skin": skin}))


def parse_schedule(SPH, text):
    vals = [int(v) for v in text.split(",")]
    if len(vals) != len(SPH.SCHEDULE_FIELDS):
        raise SystemExit(f"--schedule needs {len(SPH.SCHEDULE_FIELDS)} integers")
    return dict(zip(SPH.SCHEDULE_FIELDS, vals))


def kernel_names(sched):
    """Device-kernel names of the FP32 rate passes under a schedule."""
    return {"pass_a": f"k_pass_a_f<{sched['a_lanes']}, {sched['a_waves']}>",
            "pass_b": f"k_pass_b_f<true, {sched['b_lanes']}, {sched['b_unroll']}, "
                      f"{sched['b_waves']}>"}


def roofline_line(r32, traffic, sched):
    """Roofline of the rate pass with the larger share of the FP32 step,
    from its live-measured average launch time and the algorithmic work."""
    per = {}
    for k in ("pass_a", "pass_b"):
        ms, nl = r32["prof"][k]
        if nl:
            per[k] = ms / nl
    dom = max(per, key=lambda k: per[k])
    avg = per[dom]
    flops = PASS_FLOPS_PER_PAIR[dom] * r32["pairs"]
    byts = PASS_BYTES_PER_PARTICLE[dom] * r32["n"]
    achieved = flops / (avg * 1e-3) / 1e12
    intensity = flops / byts
    ridge = PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBPS * 1e9)
    alu = intensity >= ridge
    roof = {"bound": "alu" if alu else "hbm", "kernel": kernel_names(sched)[dom],
            "achieved": achieved if alu else byts / (avg * 1e-3) / 1e9,
            "peak": PEAK_FP32_TFLOPS if alu else PEAK_HBM_GBPS,
            "unit": "TFLOP/s" if alu else "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic[dom] if traffic else None
    roof.update({"avg_launch_ms": avg, "flops_per_launch": flops, "flops_per_pair":
                 PASS_FLOPS_PER_PAIR[dom], "algorithmic_bytes_per_launch": byts,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "avg_launch_ms_both": per})
    if traffic:
        roof["hbm_GBps"] = traffic[dom] / (avg * 1e-3) / 1e9
        roof["hbm_frac"] = roof["hbm_GBps"] / PEAK_HBM_GBPS
        roof["traffic_over_algorithmic"] = traffic[dom] / byts
    return roof


def serving_bench(SPH, W, args):
    """Continuous batching of periodic Taylor-Green requests (particle counts
    log-uniform in [2e3, 2e5], Re uniform in [100, 1000], each with its own
    dt, FP32) over a fixed arena, every pool step one batched step of the
    whole resident set.  Saturated: every request present at t = 0, admitted
    as the arena frees up (the pool's throughput).  Open loop: a calibration
    run (the first 32 requests, all present at t = 0, 10 steps) measures the
    saturated completion rate, and the requests then arrive as a Poisson
    process at 0.8 of it (latency under load)."""
    from paper_2107_01276_amd import serving
    reqs = W.serving_requests(n_req=args.serve_requests, seed=4, rate=1.0)
    built = {}

    def make(req):
        key = (req["side"], req["seed"])
        if key not in built:
            st = W.tgv(req["side"], seed=req["seed"], re=req["re"])
            cfg = SPH.config_for(st["domain"], st["params"], float(st["h"].min()),
                                 float(st["h"].max()), precision=SPH.SPH_FP32,
                                 mass_q=st["mass_q"], list_skin=args.serve_skin, lean=1, list_k=64)
            built[key] = (cfg, st, SPH.timestep(cfg))
        return built[key]

    for r in reqs:
        make(r)
    arena = int(args.serve_arena_gib * (1 << 30))
    sat = serving.serve([dict(r, arrival=0.0) for r in reqs], make, arena, steps=args.serve_steps)
    ncal = min(32, len(reqs))
    cal = [dict(r, arrival=0.0) for r in reqs[:ncal]]
    c = serving.serve(cal, make, arena, steps=10)
    rate = 0.8 * ncal / c["wall_s"] * 10.0 / args.serve_steps
    for r in reqs:
        r["arrival"] = r["arrival"] / rate
    res = serving.serve(reqs, make, arena, steps=args.serve_steps)
    res["arrival_rate_per_s"] = rate
    res["particles_total"] = int(sum(make(r)[1]["x"].size for r in reqs))
    res["saturated"] = sat
    res["list_skin"] = args.serve_skin
    return res


def config_lines(SPH, W, torch):
    """The other configurations: C1 (2,500-particle Taylor-Green, FP64, 100
    steps, one simulation's latency), the 1.5e6-particle wake-refined 1:250
    channel (PEC steps with the characteristic inlet/outlet, both
    precisions), the channel adapted to the background the library builds
    from ds_max (the build timed; FP32 and FP64 steps), and the oscillating
    cylinder (9.6e5 particles generated, adapted to its built background;
    the whole loop: body motion and a background pass every step,
    adaptation every 10 steps, inlet/outlet update)."""
    out = {}
    # C1
    s = W.tgv(50, seed=1)
    cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                         precision=SPH.SPH_FP64, mass_q=s["mass_q"], list_skin=0.0)
    ctx = SPH.Context(cfg, s["x"].size)
    P = SPH.Particles.from_arrays(s)
    ctx.run(P, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run(P, 100)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    pairs = count_pairs(ctx, P)
    out["c1_tgv_2500_fp64"] = {"ms_per_step": t * 10.0, "run_100_steps_ms": t * 1e3,
                               "pair_evals_per_s": 2.0 * pairs * 100 / t, "n_particles": P.n}
    del ctx, P
    # C3 snapshot: the wake-refined channel
    s = W.channel_wake()
    for name, prec in (("fp32", SPH.SPH_FP32), ("fp64", SPH.SPH_FP64)):
        cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                             precision=prec, mass_q=s["mass_q"], list_skin=0.3, lean=0)
        # inlet copies are appended as fluid leaves the inlet zone
        cap = int(1.05 * s["x"].size)
        ctx = SPH.Context(cfg, cap)
        P = SPH.Particles.from_arrays(s, cap)
        ctx.run(P, 2, io=s["io"])
        torch.cuda.synchronize()
        pairs = count_pairs(ctx, P)
        steps = 10
        t0 = time.perf_counter()
        ctx.run(P, steps, io=s["io"])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[f"c3_wake_channel_{name}"] = {"n_particles": P.n, "ms_per_step": t * 1e3 / steps,
                                          "pair_evals_per_s": 2.0 * pairs * steps / t}
        del ctx, P
        torch.cuda.empty_cache()
    # C2 on the background the library builds from ds_max
    s = W.channel_cylinder(seed=2)
    bg, bgi = procedure_background(SPH, W, s, torch)
    # the m_ref lookup builds the background's cells in the same context
    cap = max(int(1.6 * s["x"].size), bg["x"].size)
    line = {"background": bgi, "n_particles_generated": int(s["x"].size)}
    for name, prec, steps in (("fp32", SPH.SPH_FP32, 40), ("fp64", SPH.SPH_FP64, 40)):
        ctx, P, B = prepare(SPH, s, bg, prec, cap, 0.2, 10)
        n_ad, ratio = P.n, fluid_size_ratio(P, W)
        ctx.run(P, 5, bg=B, io=s["io"])
        torch.cuda.synchronize()
        pairs = count_pairs(ctx, P)
        t0 = time.perf_counter()
        ctx.run(P, steps, bg=B, io=s["io"])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        line[name] = {"n_particles_adapted": n_ad, "n_particles": P.n, "fluid_size_ratio": ratio,
                      "ms_per_step": t * 1e3 / steps, "pair_evals_per_s": 2.0 * pairs * steps / t}
        del ctx, P, B
        torch.cuda.empty_cache()
    out["c2_channel_procedure_background"] = line
    del bg
    # C5: the oscillating cylinder, whole loop
    s = W.oscillating_cylinder()
    mo = s["motion"]
    bg, bg5 = procedure_background(SPH, W, s, torch)
    cap = int(1.5 * s["x"].size)
    h_hi = max(float(s["h"].max()), float(bg["h"].max()))
    cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()), h_hi,
                         precision=SPH.SPH_FP32, mass_q=s["mass_q"], list_skin=0.3, n_adapt=10,
                         n_bg=1, cr=s["spec"].cr, ds_min=s["spec"].ds_min,
                         ds_max=s["spec"].ds_min * s["spec"].ratio, bg_mass_q=bg["mass_q"])
    # the context also runs the per-step background pass: room for both sets
    bcap = max(cap, int(1.2 * bg["x"].size))
    ctx = SPH.Context(cfg, bcap)
    P = SPH.Particles.from_arrays(s, cap)
    B = SPH.Background.from_arrays(bg, bcap)
    sol = s["kind"] == W.SOLID
    S = SPH.Particles.from_arrays({k: s[k][sol] for k in ("x", "y", "h", "mq")})
    dt = SPH.timestep(cfg)
    y0, t_sim = 0.0, 0.0
    n_gen = P.n
    for _ in range(ADAPT_WARM):
        ctx.adapt(P, B)
    n_ad = P.n
    # one background pass alone (the loop runs one every step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.bg_update(B, S, 1)
    torch.cuda.synchronize()
    bg_pass_ms = (time.perf_counter() - t0) * 1e3

    def advance(k):
        nonlocal y0, t_sim
        for _ in range(k):
            y1, vel, acc = W.body_motion(t_sim + dt, mo["amp"], mo["period"])
            ctx.move_solids(P, (0.0, y1 - y0), (0.0, vel), (0.0, acc))
            S.y[:S.n] += (y1 - y0)
            ctx.run(P, 1, bg=B, solids=S, io=s["io"])
            y0, t_sim = y1, t_sim + dt

    advance(2)
    torch.cuda.synchronize()
    n0 = P.n
    steps = 10
    t0 = time.perf_counter()
    advance(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["c5_oscillating_cylinder_fp32"] = {"n_particles_generated": n_gen,
                                           "n_particles_adapted": n_ad,
                                           "n_particles_start": n0, "n_particles_end": P.n,
                                           "ms_per_step": t * 1e3 / steps,
                                           "background_pass_ms": bg_pass_ms,
                                           "background_n_start": bg5["n"],
                                           "background_n": B.n, "background": bg5}
    del ctx, P, B
    torch.cuda.empty_cache()
    return out


def cpu_baseline(SPH, W, s, dt, n0, args):
    import oracle
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                     hdx=s["params"]["hdx"], mass_q=s["mass_q"])
    dom = oracle.Dom(s["domain"].lo, s["domain"].hi, s["domain"].periodic)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    legs = {}
    o = None
    for label, threads, evals in (("all_cores", cores, args.cpu_evals),
                                  ("single_thread", 1, args.cpu_evals_single)):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        opairs = 0
        for _ in range(evals):
            o = oracle.rates_k(dom, prm, s, dt, io=s["params"]["io_ref"], scales=False)
            opairs += int(o["nnb"].sum()) - n0
        t = time.perf_counter() - t0
        legs[label] = {"value": opairs / t, "threads": threads, "evals": evals, "seconds": t}
    oracle.set_threads(cores)
    cpu = {"value": legs["all_cores"]["value"], "unit": "pair-evals/s", "cores": cores,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{args.cpu_evals} rate evaluations (neighbour search + boundary pass + "
                     f"pass A + pass B, FP64, OpenMP over rows on {cores} threads) of the "
                     f"initial {n0}-particle channel state; single-thread leg: "
                     f"{args.cpu_evals_single} evaluations",
           "seconds": legs["all_cores"]["seconds"], "single_thread": legs["single_thread"]}
    return cpu


def rates_errors(SPH, s, dt, n0, torch):
    """The GPU paths' rates on the initial channel state against the
    oracle's, per field: normwise, the largest per-particle error relative
    to the oracle's sum of term magnitudes, and max |error| / max |value|."""
    import numpy as np

    import oracle
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                     hdx=s["params"]["hdx"], mass_q=s["mass_q"])
    dom = oracle.Dom(s["domain"].lo, s["domain"].hi, s["domain"].periodic)
    o = oracle.rates_k(dom, prm, s, dt, io=s["params"]["io_ref"])
    rerr = {"state": f"initial {n0}-particle channel state, one evaluation"}
    for name, prec in (("fp32", SPH.SPH_FP32), ("fp64", SPH.SPH_FP64)):
        cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()),
                             float(s["h"].max()), precision=prec, mass_q=s["mass_q"])
        r = SPH.Context(cfg, n0).rates(SPH.Particles.from_arrays(s), dt)
        e = {}
        for k in oracle.RATE_FIELDS:
            a = r[k].cpu().numpy()
            b = o[k]
            e[k] = {"norm": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)),
                    "cond": oracle.cond_error(a, b, o["scale"][k]),
                    "maxabs": float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))}
        rerr[name] = e
    return rerr



def progress(msg):
    """One line per finished phase on stderr, so a long run shows where it is."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2107_01276_amd as SPH
    import workloads as W

    torch.cuda.set_device(0)
    if args.pmc_sample:
        pmc_sample(SPH, W, torch, args.list_skin if args.list_skin is not None else 0.3,
                   args.adapt_every, parse_schedule(SPH, args.schedule) if args.schedule else None)
        return
    if args.serve_only:
        from paper_2107_01276_amd import serving
        reqs = W.serving_requests(n_req=args.serve_requests, seed=4, rate=1.0)
        built = {}

        def make(req):
            key = (req["side"], req["seed"])
            if key not in built:
                st = W.tgv(req["side"], seed=req["seed"], re=req["re"])
                cfg = SPH.config_for(st["domain"], st["params"], float(st["h"].min()),
                                     float(st["h"].max()), precision=SPH.SPH_FP32,
                                     mass_q=st["mass_q"], list_skin=args.serve_skin, lean=1, list_k=64)
                built[key] = (cfg, st, SPH.timestep(cfg))
            return built[key]

        res = serving.serve([dict(r, arrival=0.0) for r in reqs], make,
                            int(args.serve_arena_gib * (1 << 30)), steps=args.serve_steps)
        print(json.dumps({"serve_only": True, "saturated": res}))
        return
    if args.bg_pass_only:
        s = W.oscillating_cylinder()
        bg, info = procedure_background(SPH, W, s, torch)
        spec, d = s["spec"], s["domain"]
        cfg = SPH.Config(lo=d.lo, hi=d.hi, periodic=d.periodic, h_lo=0.25 * spec.ds_min,
                         h_hi=2.5 * spec.ds_min * spec.ratio, cr=spec.cr, ds_min=spec.ds_min,
                         ds_max=spec.ds_min * spec.ratio, bg_mass_q=bg["mass_q"],
                         mass_q=s["mass_q"])
        bcap = int(1.2 * bg["x"].size)
        ctx = SPH.Context(cfg, bcap)
        B = SPH.Background.from_arrays(bg, bcap)
        sol = s["kind"] == W.SOLID
        S = SPH.Particles.from_arrays({k: s[k][sol] for k in ("x", "y", "h", "mq")})
        ms = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.bg_update(B, S, 1)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
        print(json.dumps({"bg_pass_only": True, "build": info, "pass_ms": ms, "n": B.n}))
        return
    s = W.channel_cylinder(seed=2)
    bg = W.channel_background(s["spec"], seed=3)
    n0 = s["x"].size
    cap = int(1.6 * n0)
    dt = SPH.timestep(channel_cfg(SPH, s, bg, SPH.SPH_FP32, 0.0, args.adapt_every))

    # list schedule picked by timing the step loop itself (untimed here)
    from paper_2107_01276_amd import tune

    def maker(prec):
        def make(skin):
            ctx, P, B = prepare(SPH, s, bg, prec, cap, skin, args.adapt_every)
            return {"ctx": ctx, "P": P, "B": B}
        return make

    def run_steps(st, k):
        st["ctx"].run(st["P"], k, bg=st["B"], io=s["io"])

    tuning = {}
    results = {}
    for name, prec, steps in (("fp32", SPH.SPH_FP32, args.steps),
                              ("fp64", SPH.SPH_FP64, args.fp64_steps)):
        if args.list_skin is None:
            tuning[name] = tune.tune_list_skin(maker(prec), run_steps,
                                               steps=2 * max(args.adapt_every, 10))
        else:
            tuning[name] = {"best": args.list_skin, "ms_per_step": None}
        if name == "fp32" and args.schedule:
            sched_tuning = {"schedule": parse_schedule(SPH, args.schedule), "source": "--schedule"}
        elif name == "fp32":
            # kernel schedules timed on a copy of the same loop, then set on
            # the fresh context that is timed
            tc, tP, tB = prepare(SPH, s, bg, prec, cap, tuning[name]["best"], args.adapt_every)
            sched_tuning = tune.tune_schedule(
                tc, lambda k: tc.run(tP, k, bg=tB, io=s["io"]), n=tP.n, precision=name,
                use_cache=not args.no_tune_cache)
            del tc, tP, tB
            torch.cuda.empty_cache()
        ctx, P, B = prepare(SPH, s, bg, prec, cap, tuning[name]["best"], args.adapt_every)
        if name == "fp32":
            ctx.set_schedule(**sched_tuning["schedule"])
        n_adapted = P.n
        ratio = fluid_size_ratio(P, W)
        ms, prof, pairs = run(ctx, P, B, s["io"], steps, args.warmup, torch)
        ms_step = ms / steps
        results[name] = {"ms_per_step": ms_step, "pairs": pairs, "n": P.n, "prof": prof,
                         "pair_evals_per_s": 2.0 * pairs / (ms_step * 1e-3),
                         "n_adapted": n_adapted, "size_ratio": ratio}
        progress(f"{name}: {ms_step:.4f} ms/step over {steps} steps, n={P.n}")
        del ctx, P, B
        torch.cuda.empty_cache()

    r32 = results["fp32"]
    roof = roofline_line(r32, measured_traffic(), sched_tuning["schedule"])

    serve = None
    if not args.no_serve:
        serve = serving_bench(SPH, W, args)
        torch.cuda.empty_cache()
        progress("serving done")

    configs = None if args.no_configs else config_lines(SPH, W, torch)
    progress("config lines done")

    cpu = None
    rerr = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(SPH, W, s, dt, n0, args)
        progress("cpu baseline done")
        rerr = rates_errors(SPH, s, dt, n0, torch)

    out = {
        "metric": METRIC,
        "value": r32["pair_evals_per_s"],
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "channel 30D x 20D with cylinder, D/100, graded by C_r 1.05 per "
                               "5 rows (1:64 cap), Re 100, adapt every 10 steps to a prescribed "
                               "background, characteristic inlet/outlet",
                   "n_particles": r32["n"], "n_particles_generated": n0,
                   "n_particles_adapted": r32["n_adapted"],
                   "fluid_size_ratio": r32["size_ratio"], "pairs_per_eval": r32["pairs"],
                   "adapt_every": args.adapt_every, "dt": dt},

        "fp64": {"value": results["fp64"]["pair_evals_per_s"],
                 "ms_per_step": results["fp64"]["ms_per_step"], "steps": args.fp64_steps},
        "fp32_over_fp64": r32["pair_evals_per_s"] / results["fp64"]["pair_evals_per_s"],
        "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in r32["prof"].items() if v[1]},
        "kernel_launches": {k: v[1] for k, v in r32["prof"].items() if v[1]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rates_error_vs_oracle": rerr,
        "serving": serve,
        "serving_saturated_over_fp64_plain": (
            serve["saturated"]["pair_evals_per_s"] / results["fp64"]["pair_evals_per_s"]
            if serve else None),
        "configs": configs,
        "list_skin_tuning": tuning,
        "schedule_tuning": sched_tuning,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
