"""Benchmark: pair evaluations per second of the adaptive-resolution WCSPH
step on one MI355X, FP32 pair arithmetic vs plain FP64.

Workload (synthetic, seeded): the channel with a circular cylinder (D = 1,
30D x 20D, periodic in y, inflow U = 1 through an inlet buffer, outlet
buffer, finest spacing D/100, sizes graded by C_r = 1.05 per layer up to
64 D/100, h/dx = 1.2, Re = 100, wall particles inside the cylinder), ~2e5
particles, with a prescribed background (section 3.3) that sets the
reference mass.  Every step is followed by the inlet/outlet update.  Before
timing, the fluid is adapted four times to the background.  A step is one
predict-evaluate-correct step (two rate evaluations); every `--adapt-every`
steps the fluid reference mass is looked up from the background and the
fluid is split, merged three times, shifted three times and given new h.
One pair evaluation is one ordered pair (i, j != i) with j in N(i),
processed by pass A and pass B in one rate evaluation: a step has
2 (nnz - n) of them.  Adaptation time is included in the step time.

Prints ONE JSON line; `value` is the FP32 path's pair-evals/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair evals/s per step, FP32 vs FP64 plain; batched-serve p50/p99 step latency"
# Floating-point operations of the pass-B pair term (EDAC pressure rate and
# momentum, eqs. edac:sph and mom-sph) per interacting ordered pair, counted
# in the kernel as written: two kernel-gradient evaluations, the averaged
# gradient, the harmonic EDAC viscosity, the diffusion and viscous
# denominators, the pressure term and the accumulations.
PASS_B_FLOPS_PER_PAIR = 79
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
ADAPT_WARM = 4
PROF_EVERY = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--adapt-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-evals", type=int, default=40)
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=100)
    ap.add_argument("--serve-arena-gib", type=float, default=4.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--list-skin", type=float, default=None,
                    help="use this list skin for both precisions instead of timing the "
                         "candidates first (for profiled runs)")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="for hardware-counter runs: a calibration copy of known size, then a "
                         "few FP32 rate evaluations of the channel; prints nothing else")
    return ap.parse_args()


CALIB_BYTES = 1 << 29  # bytes read (and written) by the calibration copy
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_b_channel_traffic.md")
KERNEL_SOURCES = ("paper_2107_01276_amd/csrc/rates.hip", "paper_2107_01276_amd/csrc/sph_device.h")


def serving_bench(SPH, W, args):
    """Continuous batching of periodic Taylor-Green requests (particle counts
    log-uniform in [2e3, 2e5], Re uniform in [100, 1000], each with its own
    dt, FP32) over a fixed arena.  A calibration run (the first 32 requests,
    all present at t = 0, 10 steps) measures the saturated completion rate;
    the requests then arrive as a Poisson process at 0.8 of it."""
    from paper_2107_01276_amd import serving
    reqs = W.serving_requests(n_req=args.serve_requests, seed=4, rate=1.0)
    built = {}

    def make(req):
        key = (req["side"], req["seed"])
        if key not in built:
            st = W.tgv(req["side"], seed=req["seed"], re=req["re"])
            cfg = SPH.config_for(st["domain"], st["params"], float(st["h"].min()),
                                 float(st["h"].max()), precision=SPH.SPH_FP32,
                                 mass_q=st["mass_q"], list_skin=0.0, lean=1)
            built[key] = (cfg, st, st["dt"])
        return built[key]

    for r in reqs:
        make(r)
    arena = int(args.serve_arena_gib * (1 << 30))
    ncal = min(32, len(reqs))
    cal = [dict(r, arrival=0.0) for r in reqs[:ncal]]
    c = serving.serve(cal, make, arena, args.serve_streams, steps=10)
    rate = 0.8 * ncal / c["wall_s"] * 10.0 / args.serve_steps
    for r in reqs:
        r["arrival"] = r["arrival"] / rate
    res = serving.serve(reqs, make, arena, args.serve_streams, steps=args.serve_steps)
    res["arrival_rate_per_s"] = rate
    res["particles_total"] = int(sum(make(r)[1]["x"].size for r in reqs))
    return res


def pass_b_source_hash():
    """sha256 of the source pass B is compiled from: its body and kernels,
    the pair-arithmetic helpers, lane-group size and pass-B tuning macros
    above them in rates.hip, and the device header."""
    import hashlib
    rates = open(os.path.join(ROOT, KERNEL_SOURCES[0])).read()
    k0 = rates.index("#define PASS_B_PARAMS(T)")
    k1 = rates.index("\n}\n", rates.index("void k_pass_b<float, false>", k0))
    h0 = rates.index("#define RATES_FP_CONTRACT")
    h1 = rates.index("template <typename T>\nstruct RatesBufs", h0)
    g0 = rates.index("#define RGB ")
    g1 = rates.index("#define RATES_FP_CONTRACT")
    h = hashlib.sha256()
    h.update(rates[g0:g1].encode())
    h.update(rates[h0:h1].encode())
    h.update(rates[k0:k1].encode())
    with open(os.path.join(ROOT, KERNEL_SOURCES[1]), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per pass-B launch from the committed counter summary, or
    None when the kernel's source changed since the counters were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "kernel_source_sha256: ")))
    if fields.get("kernel_source_sha256", "").strip() != pass_b_source_hash():
        return None
    return float(fields["traffic_bytes_per_launch"])


def pmc_sample(SPH, W, torch):
    """One plain device copy of CALIB_BYTES (its FETCH_SIZE / WRITE_SIZE give
    the counter-to-bytes factor), then 4 FP32 rate evaluations of the
    channel (the pass-B dispatches whose traffic is measured)."""
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    s = W.channel_cylinder(seed=2)
    cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                         precision=SPH.SPH_FP32, mass_q=s["mass_q"])
    ctx = SPH.Context(cfg, s["x"].size)
    P = SPH.Particles.from_arrays(s)
    for _ in range(4):
        ctx.rates(P, s["dt"])
    torch.cuda.synchronize()
    print(json.dumps({"pmc_sample": True, "calib_bytes": CALIB_BYTES, "n": P.n}))


def count_pairs(ctx, P):
    rp, col = ctx.build_neighbors(P)
    return int(col.numel()) - P.n


def prepare(SPH, W, s, bg, prec, capacity, skin=0.1):
    h_hi = max(float(s["h"].max()), float(bg["h"].max()))
    cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()), h_hi, precision=prec,
                         mass_q=s["mass_q"], list_skin=skin)
    ctx = SPH.Context(cfg, capacity)
    P = SPH.Particles.from_arrays(s, capacity)
    B = SPH.Background.from_arrays(bg, bg["x"].size)
    for _ in range(ADAPT_WARM):
        ctx.adapt(P, B)
    return ctx, P, B


def advance(st, nsteps, dt, io, adapt_every):
    """nsteps of the timed loop: steps with the inlet/outlet update after each
    (one library call per run of steps), and an adaptation every
    `adapt_every` steps.  st holds ctx, P, B and the step counter k."""
    left = nsteps
    while left > 0:
        k = left if not adapt_every else min(left, adapt_every - st["k"] % adapt_every)
        if io is not None:
            st["ctx"].step_inout(st["P"], dt, k, io)
        else:
            st["ctx"].step(st["P"], dt, k)
        st["k"] += k
        left -= k
        if adapt_every and st["k"] % adapt_every == 0:
            st["ctx"].adapt(st["P"], st["B"])


def run(ctx, P, B, dt, steps, warmup, adapt_every, torch, io=None):
    st = {"ctx": ctx, "P": P, "B": B, "k": 0}
    advance(st, warmup, dt, io, adapt_every)
    torch.cuda.synchronize()
    pairs0 = count_pairs(ctx, P)
    # only the roofline kernel is bracketed with events in the timed region,
    # every PROF_EVERY-th launch (event markers serialise the kernels around
    # them, so sparse sampling keeps the timed work closer to unprofiled)
    ctx.profile(True, kernels=("pass_b",), every=PROF_EVERY)
    ctx.profile_reset()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(ctx.stream)
    advance(st, steps, dt, io, adapt_every)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = {k: ctx.profile_read(k) for k in ("pass_a", "pass_b", "build", "list")}
    ctx.profile(False)
    pairs1 = count_pairs(ctx, P)
    return ms, prof, 0.5 * (pairs0 + pairs1)


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
        pmc_sample(SPH, W, torch)
        return
    s = W.channel_cylinder(seed=2)
    bg = W.channel_background(s["spec"], seed=3)
    n0 = s["x"].size
    dt = s["dt"]
    cap = int(1.6 * n0)

    # list schedule picked by timing the step loop itself (untimed here)
    from paper_2107_01276_amd import tune

    def maker(prec):
        def make(skin):
            ctx, P, B = prepare(SPH, W, s, bg, prec, cap, skin)
            return {"ctx": ctx, "P": P, "B": B, "k": 0}
        return make

    def run_steps(st, k):
        advance(st, k, dt, s["io"], args.adapt_every)

    tuning = {}
    results = {}
    for name, prec, steps in (("fp32", SPH.SPH_FP32, args.steps),
                              ("fp64", SPH.SPH_FP64, args.fp64_steps)):
        if args.list_skin is None:
            tuning[name] = tune.tune_list_skin(maker(prec), run_steps,
                                               steps=2 * max(args.adapt_every, 10))
        else:
            tuning[name] = {"best": args.list_skin, "ms_per_step": None}
        ctx, P, B = prepare(SPH, W, s, bg, prec, cap, tuning[name]["best"])
        ms, prof, pairs = run(ctx, P, B, dt, steps, args.warmup, args.adapt_every, torch, s["io"])
        ms_step = ms / steps
        results[name] = {"ms_per_step": ms_step, "pairs": pairs, "n": P.n, "prof": prof,
                         "pair_evals_per_s": 2.0 * pairs / (ms_step * 1e-3)}
        del ctx, P, B
        torch.cuda.empty_cache()

    r32 = results["fp32"]
    ms_b, nb = r32["prof"]["pass_b"]
    avg_b = ms_b / max(nb, 1)
    flops = PASS_B_FLOPS_PER_PAIR * r32["pairs"]
    achieved = flops / (avg_b * 1e-3) / 1e12
    traffic = measured_traffic()
    roof = {"bound": "alu", "kernel": "k_pass_b<float>", "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic, "avg_launch_ms": avg_b, "flops_per_launch": flops,
            "flops_per_pair": PASS_B_FLOPS_PER_PAIR}
    if traffic is not None:
        gbs = traffic / (avg_b * 1e-3) / 1e9
        roof["hbm_GBps"] = gbs
        roof["hbm_frac"] = gbs / PEAK_HBM_GBPS

    serve = None
    if not args.no_serve:
        serve = serving_bench(SPH, W, args)
        torch.cuda.empty_cache()

    cpu = None
    rerr = None
    if not args.no_cpu_baseline:
        import oracle
        prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                         hdx=s["params"]["hdx"], mass_q=s["mass_q"])
        dom = oracle.Dom(s["domain"].lo, s["domain"].hi, s["domain"].periodic)
        t0 = time.perf_counter()
        opairs = 0
        for _ in range(args.cpu_evals):
            o = oracle.rates_k(dom, prm, s, dt, io=s["params"]["io_ref"])
            opairs += int(o["nnb"].sum()) - n0
        t = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": opairs / t, "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_evals} rate evaluations (neighbour search + boundary pass + "
                         f"pass A + pass B, FP64, OpenMP over rows) of the initial "
                         f"{n0}-particle channel state",
               "seconds": t}
        # the GPU paths' rates on the same state against the oracle's:
        # normwise relative error per field
        rerr = {"state": f"initial {n0}-particle channel state, one evaluation"}
        for name, prec in (("fp32", SPH.SPH_FP32), ("fp64", SPH.SPH_FP64)):
            cfg = SPH.config_for(s["domain"], s["params"], float(s["h"].min()),
                                 float(s["h"].max()), precision=prec, mass_q=s["mass_q"])
            r = SPH.Context(cfg, n0).rates(SPH.Particles.from_arrays(s), dt)
            rerr[name] = {k: float(torch.linalg.norm(r[k].cpu() - torch.as_tensor(o[k])) /
                                   max(float(torch.linalg.norm(torch.as_tensor(o[k]))), 1e-300))
                          for k in ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")}

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
        "config": {"workload": "channel with cylinder, D/100, 1:64 cap, C_r 1.05, Re 100, "
                               "adapt every 10 steps from a prescribed background",
                   "n_particles": r32["n"], "pairs_per_eval": r32["pairs"],
                   "adapt_every": args.adapt_every},
        "fp64": {"value": results["fp64"]["pair_evals_per_s"],
                 "ms_per_step": results["fp64"]["ms_per_step"], "steps": args.fp64_steps},
        "fp32_over_fp64": r32["pair_evals_per_s"] / results["fp64"]["pair_evals_per_s"],
        "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in r32["prof"].items() if v[1]},
        "kernel_launches": {k: v[1] for k, v in r32["prof"].items() if v[1]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rates_error_vs_oracle": rerr,
        "serving": serve,
        "list_skin_tuning": tuning,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
