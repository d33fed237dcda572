"""Benchmark: pair evaluations per second of the adaptive-resolution WCSPH
step on one MI355X, FP32 pair arithmetic vs plain FP64.

Workload: the channel with a circular cylinder (D = 1, 30D x 20D, periodic in
y, finest spacing D/100, sizes graded by C_r = 1.05 per layer, h/dx = 1.2,
Re = 100), ~2e5 particles, synthetic and seeded.  A step is one
predict-evaluate-correct step: two neighbour builds, two pass-A and two
pass-B evaluations and the integrator, with the fluid adapted (split, merge,
shift, h update) every `--adapt-every` steps when the library supports it.
One pair evaluation is one ordered pair (i, j != i) with j in N(i),
processed by pass A and pass B in one rate evaluation; a step has
2 (nnz - n) of them.

Prints ONE JSON line.  `value` is the FP32 path's pair-evals/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair evals/s per step, FP32 vs FP64 plain; batched-serve p50/p99 step latency"
# Algorithmic work of the pass-B pair term (EDAC pressure rate + momentum),
# per interacting ordered pair, counted from eqs. (edac:sph) and (mom-sph)
# as evaluated: two kernel-gradient evaluations, the averaged gradient, the
# Cleary harmonic viscosity, the diffusion and viscous denominators, the
# pressure term and four compensated/plain accumulations.
PASS_B_FLOPS_PER_PAIR = 79
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-evals", type=int, default=2)
    return ap.parse_args()


def count_pairs(ctx, P):
    rp, col = ctx.build_neighbors(P)
    return int(col.numel()) - P.n


def timed_steps(ctx, P, dt, steps, warmup, torch):
    for _ in range(warmup):
        ctx.step(P, dt, 1)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_reset()
    s = ctx.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        ctx.step(P, dt, 1)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = {k: ctx.profile_read(k) for k in ("pass_a", "pass_b", "build", "list")}
    ctx.profile(False)
    return ms, prof


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2107_01276_amd as SPH
    import workloads as W

    torch.cuda.set_device(0)
    s = W.channel_cylinder(seed=2)
    n = s["x"].size
    dt = s["dt"]
    h = s["h"]

    def make(prec):
        cfg = SPH.config_for(s["domain"], s["params"], float(h.min()), float(h.max()),
                             precision=prec, mass_q=s["mass_q"])
        return SPH.Context(cfg, n)

    results = {}
    for name, prec, steps in (("fp32", SPH.SPH_FP32, args.steps), ("fp64", SPH.SPH_FP64, args.fp64_steps)):
        ctx = make(prec)
        P = SPH.Particles.from_arrays(s)
        pairs0 = count_pairs(ctx, P)
        ms, prof = timed_steps(ctx, P, dt, steps, args.warmup, torch)
        pairs1 = count_pairs(ctx, P)
        pairs = 0.5 * (pairs0 + pairs1)
        ms_step = ms / steps
        results[name] = {"ms_per_step": ms_step, "pairs": pairs,
                         "pair_evals_per_s": 2.0 * pairs / (ms_step * 1e-3), "prof": prof,
                         "n": P.n}
        del ctx, P
        torch.cuda.empty_cache()

    r32 = results["fp32"]
    ms_b, nb = r32["prof"]["pass_b"]
    avg_b = ms_b / max(nb, 1)
    flops = PASS_B_FLOPS_PER_PAIR * r32["pairs"]
    achieved = flops / (avg_b * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": "pass_b<float>", "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": None, "avg_launch_ms": avg_b,
            "flops_per_launch": flops}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                         hdx=s["params"]["hdx"], mass_q=s["mass_q"])
        dom = oracle.Dom(s["domain"].lo, s["domain"].hi, s["domain"].periodic)
        t0 = time.perf_counter()
        opairs = 0
        for _ in range(args.cpu_evals):
            o = oracle.rates(dom, prm, s["x"], s["y"], s["u"], s["v"], s["p"], s["h"], s["m"], dt)
            opairs += o["col"].size - n
        t = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": opairs / t, "unit": "pair-evals/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_evals} full rate evaluations (neighbour build + pass A + "
                         f"pass B, FP64) of the {n}-particle channel state",
               "seconds": t}

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
        "config": {"workload": "channel-cylinder D/100 graded C_r=1.05 (30Dx20D, Re=100, h/dx=1.2)",
                   "n_particles": n, "pairs_per_eval": r32["pairs"], "adapt_every": None},
        "fp64": {"value": results["fp64"]["pair_evals_per_s"],
                 "ms_per_step": results["fp64"]["ms_per_step"], "steps": args.fp64_steps},
        "fp32_over_fp64": r32["pair_evals_per_s"] / results["fp64"]["pair_evals_per_s"],
        "kernel_ms": {k: (v[0] / max(v[1], 1)) for k, v in r32["prof"].items()},
        "kernel_launches": {k: v[1] for k, v in r32["prof"].items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
