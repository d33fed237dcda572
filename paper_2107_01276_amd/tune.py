"""Autotuning of the launch schedules.

Two things are tuned on the caller's own workload, because the best choice
depends on the flow and on the device:

* the neighbour-list skin: the rate passes reuse a list built with a skin
  while every particle has moved less than 1.5 skin h (the exact predicate
  is re-applied, so results do not depend on the skin).  A larger skin means
  fewer list builds but longer rows in every evaluation.  `tune_list_skin`
  times the step loop for each candidate skin on fresh copies of the state.

* the kernel schedules compiled into the library (sph_set_schedule): lanes
  per particle, the waves per SIMD the register allocation must allow, and
  the row entries loaded ahead, for each FP32 rate pass and the list build.
  `tune_schedule` times each kernel's variants with the library's own event
  timers on the live loop, one kernel at a time, and keeps the fastest.
  The live state keeps changing (list rebuilds, adaptations), so each
  variant is timed over windows long enough to hold whole cycles of both, in
  rounds that interleave the variants, and ranked by its median window.
  Results are cached per device, precision and particle-count bucket
  (powers of two) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

import torch

CANDIDATES = (0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.5)

# the variants of each kernel, as fields of the schedule
KERNEL_FIELDS = {"pass_a": ("a_lanes", "a_waves"),
                 "pass_b": ("b_lanes", "b_unroll", "b_waves"),
                 "list": ("list_lanes",)}


def tune_list_skin(make, run_steps, steps: int = 20, warmup: int = 2, candidates=CANDIDATES):
    """make(skin) -> state (fresh, with its own context); run_steps(state, k)
    advances it k steps (the loop to be timed, adaptation included).
    Returns {"best": skin, "ms_per_step": {skin: ms}}."""
    times = {}
    for skin in candidates:
        st = make(skin)
        run_steps(st, warmup)
        stream = st["ctx"].stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        run_steps(st, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        times[skin] = e0.elapsed_time(e1) / steps
        del st
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    return {"best": best, "ms_per_step": times}


def _variants(fields):
    from paper_2107_01276_amd import SCHEDULE_CHOICES
    out = [{}]
    for f in fields:
        out = [dict(v, **{f: c}) for v in out for c in SCHEDULE_CHOICES[f]]
    return out


def cache_key(n: int, precision: str) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    bucket = int(math.floor(math.log2(max(n, 1))))
    return f"{dev}|{precision}|2^{bucket}"


def default_cache_path() -> str:
    return os.environ.get("SPH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2107_01276_amd",
                                       "schedules.json"))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_schedule(ctx, run_steps, n: int, precision: str = "fp32", steps: int = 20,
                  rounds: int = 3, warmup: int = 1, cache_path: str | None = None,
                  use_cache: bool = True):
    """Picks the context's launch schedule.  run_steps(k) advances the live
    state k steps (its loop must launch the kernels being tuned; the list
    build runs only when the list is rebuilt, so a kernel with no launch in
    the timed steps keeps its current variant).  Each kernel's variants are
    timed in turn, the others held at their current choice, from the
    library's per-launch event timers.  The pick is set on ctx and returned
    as {"schedule": ..., "source": "cache" | "tuned", "key": ...,
    "ms_per_launch": {kernel: {variant: ms}}}."""
    path = cache_path or default_cache_path()
    key = cache_key(n, precision)
    data = _load(path) if use_cache else {}
    if key in data:
        ctx.set_schedule(**data[key]["schedule"])
        return {"schedule": ctx.schedule, "source": "cache", "key": key,
                "ms_per_launch": data[key].get("ms_per_launch", {})}
    times = {}
    for kern, fields in KERNEL_FIELDS.items():
        before = {f: ctx.schedule[f] for f in fields}
        samples = {}
        for _ in range(rounds):
            for v in _variants(fields):
                ctx.set_schedule(**v)
                run_steps(warmup)
                ctx.profile(True, kernels=(kern,), every=1)
                ctx.profile_reset()
                run_steps(steps)
                if torch.cuda.is_available():
                    torch.cuda.synchronize()
                ms, launches = ctx.profile_read(kern)
                ctx.profile(False)
                if launches:
                    samples.setdefault(",".join(str(v[f]) for f in fields), []).append(ms / launches)
        per = {k: sorted(v)[len(v) // 2] for k, v in samples.items()}
        if per:
            best = min(per, key=per.get)
            ctx.set_schedule(**dict(zip(fields, (int(x) for x in best.split(",")))))
        else:
            ctx.set_schedule(**before)  # not launched in the timed steps: unchanged
        times[kern] = per
    sched = ctx.schedule
    if use_cache:
        data[key] = {"schedule": sched, "ms_per_launch": times}
        _store(path, data)
    return {"schedule": sched, "source": "tuned", "key": key, "ms_per_launch": times}
