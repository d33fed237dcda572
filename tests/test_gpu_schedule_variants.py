"""Every launch-schedule variant compiled into the library (sph_set_schedule:
lanes per particle, waves per SIMD and row entries loaded ahead of the FP32
rate passes, lanes of the list build) gives FP32 rates within the FP32
tolerance of the oracle: on variable-h fluid whose longest rows exceed the
list width (the cell-walk branch), and on fluid between walls (the solid
ghost-velocity kernels).  Combinations that are not compiled in are refused
and leave the schedule as it was."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, lib, odom, particles, with_fields

pytestmark = pytest.mark.gpu

PRM = {"rho0": 1.0, "cs": 10.0, "nu": 0.01, "hdx": 1.2}


def _clustered():
    s = with_fields(W.clustered_varh(3000, seed=8, h_lo=0.006, ratio=16), seed=8)
    return s, {"list_k": 48}, None


def _wall():
    s = W.wall_box(nx=24, ny=20, layers=3, jitter=0.1, seed=21)
    rng = np.random.default_rng(22)
    fl = s["kind"] == W.FLUID
    n = s["x"].size
    s["u"] = np.where(fl, 0.3 * np.sin(2 * np.pi * s["x"]) + 0.05 * rng.standard_normal(n), 0.0)
    s["v"] = np.where(fl, 0.2 * np.cos(2 * np.pi * s["x"]) * s["y"], 0.0)
    s["p"] = np.where(fl, 1.0 - 2.0 * s["y"] + 0.01 * rng.standard_normal(n), 0.0)
    s["rho"] = 1.0 + 0.01 * rng.standard_normal(n)
    s["params"] = dict(PRM)
    s["m"] = s["mq"] * s["mass_q"]
    return s, {"body_force": (0.0, -2.0)}, (0.0, -2.0)


def _oracle(s, body, dt):
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                     hdx=s["params"]["hdx"], mass_q=s["mass_q"],
                     fx=body[0] if body else 0.0, fy=body[1] if body else 0.0)
    if "kind" in s:
        return oracle.rates_k(odom(s["domain"]), prm, s, dt)
    return oracle.rates(odom(s["domain"]), prm, s["x"], s["y"], s["u"], s["v"], s["p"], s["h"],
                        s["mq"] * s["mass_q"], dt)


def _variants(P):
    ch = P.SCHEDULE_CHOICES
    a = [dict(a_lanes=g, a_waves=w) for g in ch["a_lanes"] for w in ch["a_waves"]]
    b = [dict(b_lanes=g, b_unroll=u, b_waves=w) for g in ch["b_lanes"]
         for u in ch["b_unroll"] for w in ch["b_waves"]]
    lst = [dict(list_lanes=g) for g in ch["list_lanes"]]
    return a + b + lst


@pytest.mark.parametrize("case", ["clustered", "wall"])
def test_every_variant_vs_oracle(case):
    P = lib()
    s, kw, body = _clustered() if case == "clustered" else _wall()
    dt = 1e-4
    o = _oracle(s, body, dt)
    ctx = ctx_for(P, s, P.SPH_FP32, **kw)
    assert ctx.schedule == P.DEFAULT_SCHEDULE
    print(f"[variants] case={case} n={s['x'].size}", flush=True)
    for v in _variants(P):
        ctx.set_schedule(**P.DEFAULT_SCHEDULE)
        sc = ctx.set_schedule(**v)
        r = ctx.rates(particles(P, s), dt)
        check_rates(r, o, "fp32", f"{case} {sc}")
        assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])


def test_schedule_rejections():
    P = lib()
    s, kw, _ = _clustered()
    ctx = ctx_for(P, s, P.SPH_FP32)
    before = ctx.schedule
    for bad in ({"a_lanes": 3}, {"a_waves": 2}, {"b_lanes": 8}, {"b_unroll": 3},
                {"b_waves": 6}, {"list_lanes": 16}, {"a_lanes": 0}):
        with pytest.raises(P.SphError) as e:
            ctx.set_schedule(**bad)
        assert e.value.code == P.SPH_E_INVAL and "not compiled in" in str(e.value), bad
        assert ctx.schedule == before
