"""The Gresho-Chan vortex (section 4.2) on the GPU: rates against the oracle
on the exact steady state, the centripetal closed form, one adaptation with
the refined-region background bit-exact against the oracle (m_ref lookup,
split, merges, shifts, h update), and a run with and without adaptation
against the exact steady solution (the vortex must stay steady: L1 velocity
error, maximum speed, mass exactly conserved, angular momentum)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, dt_of, lib, odom, particles, rel_norm

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")


def _prm(s):
    return oracle.Prm(rho0=1.0, cs=10.0, nu=0.0, hdx=1.0, mass_q=s["mass_q"])


def _jittered(s, seed=3):
    """The same vortex on a lattice jittered by 2% of the spacing (on the
    exact lattice the shift is rounding noise, so its parity would be
    meaningless), with the closed-form fields at the moved positions."""
    rng = np.random.default_rng(seed)
    d = s["domain"]
    dx = (d.hi[0] - d.lo[0]) / math.sqrt(s["x"].size)
    out = dict(s)
    out["x"] = d.lo[0] + np.mod(s["x"] + 0.02 * dx * rng.standard_normal(s["x"].size) - d.lo[0],
                                d.hi[0] - d.lo[0])
    out["y"] = d.lo[1] + np.mod(s["y"] + 0.02 * dx * rng.standard_normal(s["y"].size) - d.lo[1],
                                d.hi[1] - d.lo[1])
    out["u"], out["v"], out["p"], _ = W.gresho_chan_fields(out["x"], out["y"])
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rates_vs_oracle_and_centripetal(prec):
    P = lib()
    s0 = W.gresho_chan(40)
    s = _jittered(s0)
    print(f"[gresho] rates n={s['x'].size} prec={prec}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64 if prec == "fp64" else P.SPH_FP32)
    r = ctx.rates(particles(P, s), dt_of(s))
    o = oracle.rates(odom(s["domain"]), _prm(s), s["x"], s["y"], s["u"], s["v"], s["p"], s["h"],
                     s["mq"] * s["mass_q"], dt_of(s))
    assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])
    check_rates(r, o, prec, "gresho")
    # the centripetal acceleration of the exact steady state, on the lattice
    r = ctx.rates(particles(P, s0), dt_of(s0))
    x, y = s0["x"], s0["y"]
    r2 = np.maximum(x * x + y * y, 1e-300)
    _, _, _, uphi = W.gresho_chan_fields(x, y)
    ax, ay = -uphi ** 2 * x / r2, -uphi ** 2 * y / r2
    du, dv = r["dudt"].cpu().numpy(), r["dvdt"].cpu().numpy()
    err = (np.abs(du - ax) + np.abs(dv - ay)).sum() / (np.abs(ax) + np.abs(ay)).sum()
    assert err < 0.04, err


def test_adapt_with_background_bitexact():
    P = lib()
    nx = 40
    s = W.gresho_chan(nx)
    bg = W.gresho_chan_background(nx)
    n = s["x"].size
    cap = 8 * n
    q = s["mass_q"]
    dom = s["domain"]
    print(f"[gresho] adapt n={n} nb={bg['x'].size}", flush=True)
    st = {k: s[k].copy() for k in ("x", "y", "u", "v", "p", "rho", "h", "mq", "kind")}
    st["mref"] = oracle.mref_lookup(odom(dom), st["x"], st["y"], st["h"], bg["x"], bg["y"], bg["h"],
                                    bg["mref"])
    o, oinfo = oracle.adapt(odom(dom), oracle.Prm(mass_q=q, hdx=1.0), st, cap=cap)
    cfg = P.Config(lo=dom.lo, hi=dom.hi, periodic=dom.periodic, h_lo=float(s["h"].min()) * 0.5,
                   h_hi=float(bg["h"].max()), precision=P.SPH_FP64, hdx=1.0, mass_q=q)
    ctx = P.Context(cfg, cap)
    ps = P.Particles.from_arrays(dict(s), cap)
    info = ctx.adapt(ps, P.Background.from_arrays(bg, bg["x"].size))
    g = ps.numpy()
    print(f"[gresho] gpu n={ps.n} split={info['n_split']} merged={info['merged']} "
          f"oracle n={o['x'].size} split={oinfo['n_split']} merged={oinfo['merged']}", flush=True)
    assert info["n_split"] > 0
    assert info["n_split"] == oinfo["n_split"] and info["merged"] == oinfo["merged"]
    assert ps.n == o["x"].size
    assert np.array_equal(info["origin"].cpu().numpy(), oinfo["origin"])
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mref"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["mq"], o["mq"]) and g["mq"].sum() == s["mq"].sum()


def _run(P, nx, adaptive, T):
    s = W.gresho_chan(nx)
    bg = W.gresho_chan_background(nx) if adaptive else None
    hmin = float(s["h"].min()) * (math.sqrt(0.5) if adaptive else 1.0)
    hmax = max(float(s["h"].max()) * 1.5, float(bg["h"].max()) if adaptive else 0.0)
    cfg = P.config_for(s["domain"], s["params"], 0.9 * hmin, hmax, precision=P.SPH_FP64,
                       mass_q=s["mass_q"], list_skin=0.1)
    cap = 8 * s["x"].size
    ctx = P.Context(cfg, cap)
    ps = P.Particles.from_arrays(s, cap)
    B = P.Background.from_arrays(bg, bg["x"].size) if adaptive else None

    def angmom(g):
        m = g["mq"] * s["mass_q"]
        return float(np.sum(m * (g["x"] * g["v"] - g["y"] * g["u"])))

    g0 = ps.numpy()
    L0, M0 = angmom(g0), int(g0["mq"].sum())
    dt = 0.25 * hmin / (1.0 + s["params"]["cs"])
    nsteps = int(round(T / dt))
    if adaptive:
        ctx.adapt(ps, B)
    k = 0
    while k < nsteps:
        kk = min(10, nsteps - k)
        ctx.step(ps, dt, kk)
        k += kk
        if adaptive:
            ctx.adapt(ps, B)
    g = ps.numpy()
    u, v, _, _ = W.gresho_chan_fields(g["x"], g["y"])
    return {"n": int(ps.n), "l1": float(np.mean(np.hypot(g["u"] - u, g["v"] - v))),
            "umax": float(np.max(np.hypot(g["u"], g["v"]))), "mass": int(g["mq"].sum()) - M0,
            "dL": (angmom(g) - L0) / L0}


def test_steady_vortex_with_and_without_adaptation():
    P = lib()
    plain = _run(P, 50, False, 0.3)
    adapt = _run(P, 50, True, 0.3)
    print(f"[gresho] plain {plain} adaptive {adapt}", flush=True)
    for r in (plain, adapt):
        assert r["mass"] == 0
        assert r["l1"] < 0.015
        assert 0.95 < r["umax"] < 1.05
        assert abs(r["dL"]) < 3e-3
    assert adapt["n"] > plain["n"]                # the inner region was refined
    assert adapt["l1"] < 1.5 * plain["l1"] + 2e-3  # and costs little accuracy
