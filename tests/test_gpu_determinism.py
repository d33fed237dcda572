"""Determinism: the whole loop (steps with walls and the characteristic
inlet/outlet, the inlet/outlet update, adaptation against a background)
run twice from the same state in fresh contexts gives the same bits, in
both precisions.  No sum in the path depends on the order in which atomics
land (the boundary list's order and the shift maximum do not change any
value)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dt_of, lib

pytestmark = pytest.mark.gpu


def _run(P, prec):
    spec = W.ChannelSpec(length=4.0, height=4.0, cyl_x=1.5, ds_min=0.02, ratio=8, io_layers=4)
    s = W.channel_cylinder(spec, seed=5)
    bg = W.channel_background(spec, seed=6)
    cap = 4 * s["x"].size
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(bg["h"].max()),
                       precision=prec, mass_q=s["mass_q"], list_skin=0.2)
    ctx = P.Context(cfg, cap)
    ps = P.Particles.from_arrays(s, cap)
    B = P.Background.from_arrays(bg, cap)
    ctx.adapt(ps, B)
    for _ in range(2):
        ctx.step_inout(ps, dt_of(s), 10, s["io"])
        ctx.adapt(ps, B)
    return ps.numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_run_twice_same_bits(prec):
    P = lib()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    a = _run(P, pr)
    b = _run(P, pr)
    print(f"[determinism] prec={prec} n={a['x'].size}", flush=True)
    assert a["x"].size == b["x"].size
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind"):
        assert np.array_equal(a[k], b[k]), k
