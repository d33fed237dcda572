"""sph_step runs the per-iteration schedule of section 3.4 (background
update every n_bg iterations, adaptation every n_adapt, then the step and
the inlet/outlet update) inside the library.  Its result equals, bit for
bit, the separate calls made in the same order from Python."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import lib

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind")


def _same(a, b, tag):
    assert a.n == b.n, (tag, a.n, b.n)
    ga, gb = a.numpy(), b.numpy()
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), (tag, k)


def test_channel_schedule_equals_separate_calls():
    """The benchmark's channel: adaptation every 10 iterations against a
    prescribed background, inlet/outlet update after every step, 25
    iterations from iteration 0 in one call; the same from Python as runs of
    steps with the inlet/outlet update and adaptations between them."""
    P = lib()
    s = W.channel_cylinder(seed=2)
    bg = W.channel_background(s["spec"], seed=3)
    cap = int(1.6 * s["x"].size)
    print(f"[schedule] channel n={s['x'].size}", flush=True)

    def make():
        cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()),
                           max(float(s["h"].max()), float(bg["h"].max())), precision=P.SPH_FP32,
                           mass_q=s["mass_q"], list_skin=0.3, n_adapt=10)
        ctx = P.Context(cfg, cap)
        ps = P.Particles.from_arrays(s, cap)
        B = P.Background.from_arrays(bg, bg["x"].size)
        ctx.adapt(ps, B)
        return cfg, ctx, ps, B

    cfg, ctx, ps, B = make()
    dt = P.timestep(cfg)
    assert dt == pytest.approx(oracle.dt_for(s), rel=4e-16)
    d = ctx.run(ps, 25, bg=B, io=s["io"], diag=True)
    assert ctx.iteration == 25 and d["n"] == ps.n
    _, c2, p2, B2 = make()
    for k in (10, 10, 5):
        c2.step_inout(p2, dt, k, s["io"])
        if k == 10:
            c2.adapt(p2, B2)
    _same(ps, p2, "channel")
    assert d["mq_total"] == int(p2.numpy()["mq"].sum())


def test_zone_schedule_with_background_updates():
    """The zone-refined Taylor-Green lattice with its markers as the solids:
    a background pass every 5 iterations and an adaptation every 10, for 22
    iterations starting at iteration 3 (the counter carries across calls),
    against the separate calls."""
    P = lib()
    s = W.tgv_zone(50)
    bp, bg0, dom = s["bg_params"], s["background"], s["domain"]
    cap = 8 * s["x"].size

    def make():
        cfg = P.Config(lo=dom.lo, hi=dom.hi, periodic=dom.periodic, h_lo=0.003, h_hi=0.05,
                       cr=bp["cr"], ds_min=bp["ds_min"], ds_max=bp["ds_max"],
                       bg_mass_q=bg0["mass_q"], mass_q=s["mass_q"], hdx=1.0, nu=s["params"]["nu"],
                       list_skin=0.0, n_adapt=10, n_bg=5, bg_passes=1, dt=2e-4)
        ctx = P.Context(cfg, cap)
        B = P.Background.from_arrays(bg0, cap)
        M = P.Particles.from_arrays({"x": s["markers"]["x"], "y": s["markers"]["y"],
                                     "h": s["markers"]["h"],
                                     "mq": np.ones(s["markers"]["x"].size, np.int64)})
        ctx.bg_update(B, M, P.bg_init_passes(cfg))
        ps = P.Particles.from_arrays(dict(s), cap)
        ctx.adapt(ps, B)
        return ctx, ps, B, M

    ctx, ps, B, M = make()
    print(f"[schedule] zone n={ps.n} bg={B.n}", flush=True)
    ctx.iteration = 3
    ctx.run(ps, 10, bg=B, solids=M)
    ctx.run(ps, 12, bg=B, solids=M)
    assert ctx.iteration == 25
    c2, p2, B2, M2 = make()
    for it in range(3, 25):
        if it % 5 == 0:
            c2.bg_update(B2, M2, 1)
        if it % 10 == 0:
            c2.adapt(p2, B2)
        c2.step(p2, 2e-4, 1)
    assert B.n == B2.n
    _same(ps, p2, "zone")
