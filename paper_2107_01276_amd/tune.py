"""Autotuning of the neighbour-list schedule.

The rate passes reuse a neighbour list built with a skin while every
particle has moved less than 1.5 skin h (the exact predicate is re-applied,
so results do not depend on the skin).  A larger skin means fewer list
builds but longer rows in every evaluation; the best value depends on the
flow (speeds, adaptation cadence) and on the device.  `tune_list_skin`
times the caller's own step loop for each candidate skin on fresh copies of
the state and returns the fastest.
"""
from __future__ import annotations

import torch

CANDIDATES = (0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.5)


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
