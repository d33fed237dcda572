"""Continuous-batching request loop over the serving pool (sph_pool_*).

Requests arrive over wall-clock time.  Between pool steps the loop admits,
in arrival order, every request that has arrived and fits the pool (a free
range of particle slots and cell tables; admission stops at the first that
does not, so that a large request is not starved), advances every resident
simulation by one step with one batched step of the whole resident set,
and retires the simulations that finished their steps; their ranges take
the next arrivals.  Every pool step gives each resident simulation a step
latency: the device time of that batched step.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import Particles, Pool


def serve(requests, make_state, arena_bytes: int, max_sims: int = 512, steps: int = 100,
          on_done=None):
    """requests: dicts with at least "arrival" (seconds from the start).
    make_state(req) -> (Config, state dict for Particles.from_arrays, dt).
    on_done(req, pool, sim_id) is called before a finished simulation is
    retired (e.g. to read its state).  Returns latency and throughput
    statistics."""
    pool = Pool(arena_bytes, max_sims)
    order = sorted(range(len(requests)), key=lambda k: requests[k]["arrival"])
    waiting = collections.deque()
    resident = {}
    lat = []
    step_ms = []
    pair_evals = 0
    done = 0
    peak_resident = 0
    peak_particles = 0
    head = None  # (req, Particles, cfg, dt) of the first waiting request
    t0 = time.perf_counter()
    nxt = 0
    busy = 0.0
    while nxt < len(order) or waiting or head is not None or resident:
        now = time.perf_counter() - t0
        while nxt < len(order) and requests[order[nxt]]["arrival"] <= now:
            waiting.append(requests[order[nxt]])
            nxt += 1
        while head is not None or waiting:
            if head is None:
                req = waiting.popleft()
                cfg, st, dt = make_state(req)
                head = (req, Particles.from_arrays(st), cfg, dt)
            req, P, cfg, dt = head
            sid = pool.admit(cfg, P, dt)
            if sid is None:
                break
            req["admitted"] = time.perf_counter() - t0
            resident[sid] = [req, steps]
            head = None
        if not resident:
            if head is not None:
                raise RuntimeError("a request does not fit the empty pool")
            if nxt < len(order):
                time.sleep(max(0.0, requests[order[nxt]]["arrival"] - (time.perf_counter() - t0)))
            continue
        info = pool.info()
        peak_resident = max(peak_resident, len(resident))
        peak_particles = max(peak_particles, info["particles"])
        tb = time.perf_counter()
        pool.step(1)
        busy += time.perf_counter() - tb
        ms = pool.info()["last_step_ms"]
        step_ms.append(ms)
        lat.extend([ms] * len(resident))
        for sid in list(resident):
            resident[sid][1] -= 1
            if resident[sid][1] == 0:
                if on_done is not None:
                    on_done(resident[sid][0], pool, sid)
                resident[sid][0]["finished"] = time.perf_counter() - t0
                pool.retire(sid)
                pair_evals += pool.stats(sid, pairs=True)["pair_evals"]
                del resident[sid]
                done += 1
    wall = time.perf_counter() - t0
    pool.close()
    lat = np.asarray(lat)
    gpu_s = float(np.sum(step_ms)) * 1e-3
    return {
        "requests": done,
        "steps_per_request": steps,
        "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
        "pair_evals": int(pair_evals),
        "wall_s": wall,
        "busy_s": busy,
        "gpu_s": gpu_s,
        "pool_steps": len(step_ms),
        "pair_evals_per_s": pair_evals / wall if wall > 0 else None,
        "pair_evals_per_gpu_s": pair_evals / gpu_s if gpu_s > 0 else None,
        "peak_resident": peak_resident,
        "peak_particles": int(peak_particles),
        "arena_bytes": int(arena_bytes),
    }
