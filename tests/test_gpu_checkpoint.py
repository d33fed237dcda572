"""Checkpoint and resume through the C ABI (sph_export / sph_import): the
round trip is bit-exact, a run resumed in a fresh context steps exactly as
the uninterrupted one (bit for bit with list_skin 0, in both precisions),
and bad checkpoints are refused before anything is written."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import ctx_for, lib, particles

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind")


def _case():
    s = W.wall_box(nx=16, ny=16, layers=3, jitter=0.1, seed=41)
    rng = np.random.default_rng(42)
    n = s["x"].size
    fl = s["kind"] == W.FLUID
    s["u"] = np.where(fl, 0.2 * rng.standard_normal(n), 0.0)
    s["v"] = np.where(fl, 0.1 * rng.standard_normal(n), 0.0)
    s["p"] = np.where(fl, 1.0 - s["y"], 0.0)
    s["rho"] = 1.0 + 0.01 * rng.standard_normal(n)
    s["params"] = {"rho0": 1.0, "cs": 10.0, "nu": 0.05, "hdx": 1.2}
    return s


def test_round_trip_bitexact():
    P = lib()
    s = _case()
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=2 * s["x"].size)
    ps = particles(P, s, capacity=2 * s["x"].size)
    buf = ctx.export(ps, step=123, time=0.0456)
    assert buf.size == ctx.lib.sph_export_bytes(ps.n)
    q = particles(P, {"x": np.zeros(1), "y": np.zeros(1), "h": np.ones(1),
                      "mq": np.ones(1, np.int64)}, capacity=2 * s["x"].size)
    step, t = ctx.import_(q, buf)
    assert (step, t) == (123, 0.0456) and q.n == ps.n
    a, b = ps.numpy(), q.numpy()
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("skin", [0.0, 0.1])
def test_resume(prec, skin):
    P = lib()
    s = _case()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    dt = 2e-4
    print(f"[ckpt] prec={prec} skin={skin}", flush=True)
    c1 = ctx_for(P, s, pr, body_force=(0.0, -1.0), list_skin=skin)
    p1 = particles(P, s)
    c1.step(p1, dt, 20)
    c2 = ctx_for(P, s, pr, body_force=(0.0, -1.0), list_skin=skin)
    p2 = particles(P, s)
    c2.step(p2, dt, 10)
    buf = c2.export(p2, step=10, time=10 * dt)
    del c2, p2
    c3 = ctx_for(P, s, pr, body_force=(0.0, -1.0), list_skin=skin)
    p3 = particles(P, {"x": np.zeros(1), "y": np.zeros(1), "h": np.ones(1),
                       "mq": np.ones(1, np.int64)}, capacity=s["x"].size)
    step, t = c3.import_(p3, buf)
    assert step == 10 and t == 10 * dt
    c3.step(p3, dt, 10)
    a, b = p1.numpy(), p3.numpy()
    for k in ("x", "y", "u", "v", "p", "rho"):
        if skin == 0.0:
            assert np.array_equal(a[k], b[k]), k
        else:
            d = float(np.max(np.abs(a[k] - b[k])) / max(np.max(np.abs(a[k])), 1e-300))
            assert d < (1e-12 if prec == "fp64" else 1e-5), (k, d)


def test_import_rejections_leave_state():
    P = lib()
    s = _case()
    n = s["x"].size
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=n)
    ps = particles(P, s, capacity=n)
    good = ctx.export(ps)
    small = particles(P, {"x": np.zeros(3), "y": np.zeros(3), "h": np.ones(3),
                          "mq": np.ones(3, np.int64)}, capacity=n // 2)
    before = small.numpy()

    def refused(buf, code, target=small):
        with pytest.raises(P.SphError) as e:
            ctx.import_(target, buf)
        assert e.value.code == code
        after = target.numpy()
        for k in before:
            assert np.array_equal(before[k], after[k]), k

    refused(good, P.SPH_E_CAPACITY)                       # n above the capacity
    bad = good.copy(); bad[0] = ord("X"); refused(bad, P.SPH_E_INVAL)     # magic
    refused(good[:100], P.SPH_E_INVAL)                    # truncated
    few = ctx.export(particles(P, {k: s[k][:10] for k in ("x", "y", "h", "u", "v", "p", "rho",
                                                          "mq", "kind", "mref")}))
    nanbuf = few.copy()
    nanbuf[64 + 8 * 10 * 4 + 8 * 3:64 + 8 * 10 * 4 + 8 * 4] = np.frombuffer(
        np.array([math.nan]).tobytes(), np.uint8)       # p of particle 3
    refused(nanbuf, P.SPH_E_NONFINITE)
    other = ctx_for(P, dict(s, mass_q=s["mass_q"] * 2), P.SPH_FP64, capacity=n)
    with pytest.raises(P.SphError) as e:                   # another mass quantum
        other.import_(particles(P, s, capacity=n), good)
    assert e.value.code == P.SPH_E_INVAL
    ctx.import_(small, few)                               # a valid one still works
    assert small.n == 10
