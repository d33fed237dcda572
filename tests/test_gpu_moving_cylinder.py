"""A cylinder oscillating across the stream, y_c = 0.5 D sin(2 pi t / 5)
(1:100, Re = 200, D/400, 9.6e5 particles at full size): the prescribed
body motion (sph_move_solids) with the wall acceleration of eq. (bc-pre),
steps, the background following the body (one pass per step, section 3.3)
and the adaptation against the oracle on a small channel, and at full size
the rates of every particle after the body has moved, plus a run of the
whole loop that keeps the mass ledger and the body's position exact."""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, dt_of, lib, odom, particles, rel_norm

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")


def _prm(s):
    return oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"], hdx=s["params"]["hdx"],
                      mass_q=s["mass_q"])


def _solids(P, s, g=None):
    g = s if g is None else g
    sol = g["kind"] == W.SOLID
    return P.Particles.from_arrays({"x": g["x"][sol], "y": g["y"][sol], "h": g["h"][sol],
                                    "mq": np.ones(int(sol.sum()), np.int64)}), \
        {"x": g["x"][sol], "y": g["y"][sol], "h": g["h"][sol]}


def _compare_bg(gb, ob, tag):
    assert np.array_equal(gb["mask"], ob["mask"]) and np.array_equal(gb["mq"], ob["mq"]), tag
    for k in ("ds", "mref"):
        assert np.allclose(gb[k], ob[k], rtol=1e-12, atol=0), (tag, k)
    for k in ("x", "y", "h"):
        assert float(np.max(np.abs(gb[k] - ob[k]))) < 1e-12, (tag, k)


def test_moving_cylinder_small_vs_oracle():
    P = lib()
    spec = W.ChannelSpec(length=4.0, height=4.0, cyl_x=2.0, ds_min=0.02, ratio=8, re=200.0,
                         io_layers=0)
    s = W.oscillating_cylinder(spec)
    s["m"] = s["mq"] * s["mass_q"]
    mo = s["motion"]
    d = odom(s["domain"])
    n = s["x"].size
    dt = dt_of(s)
    print(f"[osc-small] n={n} dt={dt}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=4 * n, cr=spec.cr, ds_min=spec.ds_min,
                  ds_max=spec.ds_min * spec.ratio)
    ps = particles(P, s, capacity=4 * n)
    o = dict(s)
    t = 0.0
    y0 = 0.0
    for k in range(5):
        y1, vel, acc = W.body_motion(t + 2 * dt, mo["amp"], mo["period"])
        dy = y1 - y0
        ctx.move_solids(ps, (0.0, dy), (0.0, vel), (0.0, acc))
        ctx.step(ps, dt, 2)
        o = oracle.move_solids(d, o, (0.0, dy), (0.0, vel))
        o = oracle.step_k(d, _prm(s), o, dt, 2, aw=(0.0, acc))
        t += 2 * dt
        y0 = y1
    g = ps.numpy()
    sol = g["kind"] == W.SOLID
    assert np.array_equal(g["y"][sol], o["y"][sol]) and np.array_equal(g["v"][sol], o["v"][sol])
    for k in ("x", "y", "u", "v", "p", "rho"):
        e = rel_norm(g[k], o[k])
        print(f"[osc-small] {k} {e:.2e}", flush=True)
        assert e < 1e-10, (k, e)
    # the background follows the moved body: one pass, both sides
    bg = W.channel_background(spec)
    bp = oracle.BgPrm(cr=spec.cr, ds_min=spec.ds_min, ds_max=spec.ds_min * spec.ratio,
                      mass_q=bg["mass_q"])
    S, sd = _solids(P, s, g)
    ob, onsplit = oracle.bg_update(d, bp, bg, sd, 1, cap=4 * n)
    c2 = P.Context(P.config_for(s["domain"], s["params"], float(s["h"].min()), float(bg["h"].max()),
                                mass_q=s["mass_q"], cr=spec.cr, ds_min=spec.ds_min,
                                ds_max=spec.ds_min * spec.ratio, bg_mass_q=bg["mass_q"]), 4 * n)
    B = P.Background.from_arrays(bg, 4 * n)
    nsplit = c2.bg_update(B, S, 1)
    assert nsplit == onsplit and B.n == ob["x"].size
    _compare_bg(B.numpy(), ob, "moved body")
    # adaptation of the stepped state against the oracle's background
    st = {k: np.asarray(o[k]).copy() for k in ("x", "y", "u", "v", "p", "rho", "h", "kind")}
    st["mq"] = s["mq"].copy()
    st["mref"] = oracle.mref_lookup(d, st["x"], st["y"], st["h"], ob["x"], ob["y"], ob["h"],
                                    ob["mref"])
    oa, oinfo = oracle.adapt(d, _prm(s), st, cap=4 * n)
    pa = P.Particles.from_arrays(dict(st), 4 * n)
    ainfo = c2.adapt(pa, P.Background.from_arrays(ob, 4 * n))
    print(f"[osc-small] adapt gpu split={ainfo['n_split']} merged={ainfo['merged']}; "
          f"oracle split={oinfo['n_split']} merged={oinfo['merged']}", flush=True)
    assert ainfo["n_split"] == oinfo["n_split"] and ainfo["merged"] == oinfo["merged"]
    ga = pa.numpy()
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind"):
        assert np.array_equal(ga[k], oa[k]), k


def test_moving_cylinder_full_size():
    P = lib()
    s = W.oscillating_cylinder()
    s["m"] = s["mq"] * s["mass_q"]
    spec, mo = s["spec"], s["motion"]
    d = odom(s["domain"])
    n = s["x"].size
    print(f"[osc] n={n}", flush=True)
    # the body at a quarter period: displaced by the amplitude, at rest, decelerating
    yq, vq, aq = W.body_motion(0.25 * mo["period"], mo["amp"], mo["period"])
    o = oracle.move_solids(d, s, (0.0, yq), (0.0, vq))
    r_o = oracle.rates_k(d, _prm(s), o, dt_of(s), aw=(0.0, aq), io=s["params"]["io_ref"])
    for prec, name in ((P.SPH_FP64, "fp64"), (P.SPH_FP32, "fp32")):
        ctx = ctx_for(P, s, prec)
        ps = particles(P, s)
        ctx.move_solids(ps, (0.0, yq), (0.0, vq), (0.0, aq))
        r = ctx.rates(ps, dt_of(s))
        assert np.array_equal(r["nnb"].cpu().numpy(), r_o["nnb"])
        check_rates(r, r_o, name, "oscillating cylinder")
    # the whole loop on the FP32 path: body motion and a background pass
    # every step, adaptation every 10 steps, inlet/outlet zones updated
    bg = W.channel_background(spec)
    cap = 2 * n
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(bg["h"].max()),
                       precision=P.SPH_FP32, mass_q=s["mass_q"], cr=spec.cr, ds_min=spec.ds_min,
                       ds_max=spec.ds_min * spec.ratio, bg_mass_q=bg["mass_q"])
    ctx = P.Context(cfg, cap)
    ps = P.Particles.from_arrays(s, cap)
    B = P.Background.from_arrays(bg, cap)
    sol0 = s["kind"] == W.SOLID
    ys = s["y"][sol0].copy()
    M0 = int(s["mq"].sum())
    dt, t, y0 = dt_of(s), 0.0, 0.0
    steps = 20
    ctx.adapt(ps, B)
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        y1, vel, acc = W.body_motion(t + dt, mo["amp"], mo["period"])
        ctx.move_solids(ps, (0.0, y1 - y0), (0.0, vel), (0.0, acc))
        ys = ys + (y1 - y0)
        ctx.step_inout(ps, dt, 1, s["io"])
        S, _ = _solids(P, s, ps.numpy())
        ctx.bg_update(B, S, 1)
        if k % 10 == 0:
            ctx.adapt(ps, B)
        t += dt
        y0 = y1
    el = time.perf_counter() - t0
    g = ps.numpy()
    sol = g["kind"] == W.SOLID
    print(f"[osc] loop {steps} steps {1e3 * el / steps:.2f} ms/step (with host copies of the "
          f"solids), n={ps.n}, mass change={int(g['mq'].sum()) - M0}", flush=True)
    assert np.array_equal(np.sort(g["y"][sol]), np.sort(ys))
    assert np.all(np.isfinite(g["u"])) and np.all(np.isfinite(g["p"]))
