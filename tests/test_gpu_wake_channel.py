"""The channel at the 1:250 ratio (D/250, Re = 1000) with its wake refined
by the vorticity criterion, at full size (1.5e6 particles): the neighbour
lists of every particle bit-exact with the oracle, the rates of every
particle within 1e-12 (FP64) and 1e-5 (FP32), the vorticity, the
solution-driven background update (k = 0.1, section 3.3) and one
adaptation against that background bit-exact."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, dt_of, lib, odom, particles, rel_norm

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")


@pytest.fixture(scope="module")
def wake():
    s = W.channel_wake()
    s["m"] = s["mq"] * s["mass_q"]
    return s


def _prm(s):
    return oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"], hdx=s["params"]["hdx"],
                      mass_q=s["mass_q"])


def test_wake_channel_neighbors_and_rates(wake):
    P = lib()
    s = wake
    d = odom(s["domain"])
    print(f"[wake] n={s['x'].size} levels={np.unique(s['h']).size}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64)
    rp, col = ctx.build_neighbors(particles(P, s))
    orp, ocol = oracle.neighbors(d, s["x"], s["y"], s["h"])
    print(f"[wake] nnz gpu={col.numel()} oracle={ocol.size}", flush=True)
    assert np.array_equal(rp.cpu().numpy(), orp) and np.array_equal(col.cpu().numpy(), ocol)
    del rp, col, orp, ocol
    o = oracle.rates_k(d, _prm(s), s, dt_of(s), io=s["params"]["io_ref"])
    for prec, name in ((P.SPH_FP64, "fp64"), (P.SPH_FP32, "fp32")):
        c = ctx if prec == P.SPH_FP64 else ctx_for(P, s, prec)
        r = c.rates(particles(P, s), dt_of(s))
        assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])
        check_rates(r, o, name, "wake channel")


def test_wake_channel_solution_background_and_adapt(wake):
    P = lib()
    s = wake
    d = odom(s["domain"])
    spec = s["spec"]
    n = s["x"].size
    bg = W.channel_background(spec)
    kind = s["kind"]
    sol = kind == W.SOLID
    solids = {"x": s["x"][sol], "y": s["y"][sol], "h": s["h"][sol]}
    k_frac, passes = 0.1, 1
    print(f"[wake-bg] n={n} nb={bg['x'].size}", flush=True)
    rp, col = oracle.neighbors(d, s["x"], s["y"], s["h"])
    om = oracle.vorticity(d, s["x"], s["y"], s["u"], s["v"], s["h"], s["m"], s["rho"], rp, col)
    del rp, col
    cap = 2 * n
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(bg["h"].max()),
                       precision=P.SPH_FP64, mass_q=s["mass_q"], cr=spec.cr, ds_min=spec.ds_min,
                       ds_max=spec.ds_min * spec.ratio, bg_mass_q=bg["mass_q"])
    ctx = P.Context(cfg, cap)
    F = P.Particles.from_arrays(s, cap)
    w = ctx.vorticity(F).cpu().numpy()
    ew = float(np.linalg.norm(w - om) / np.linalg.norm(om))
    print(f"[wake-bg] vorticity rel err {ew:.2e}", flush=True)
    assert ew < 1e-12
    aom = np.abs(om)
    thresh = k_frac * aom[kind == W.FLUID].max()
    phi = oracle.shepard_to_bg(d, bg["x"], bg["y"], bg["h"], s["x"], s["y"], s["h"], aom, kind=kind)
    bp = oracle.BgPrm(cr=spec.cr, ds_min=spec.ds_min, ds_max=spec.ds_min * spec.ratio,
                      mass_q=bg["mass_q"])
    ob, onsplit = oracle.bg_update(d, bp, bg, solids, passes, cap=cap, phi=phi, phi_thresh=thresh)
    B = P.Background.from_arrays(bg, cap)
    S = P.Particles.from_arrays({"x": solids["x"], "y": solids["y"], "h": solids["h"],
                                 "mq": np.ones(int(sol.sum()), np.int64)})
    info = ctx.bg_update_solution(B, S, F, k_frac, passes)
    gb = B.numpy()
    print(f"[wake-bg] gpu nb={B.n} splits={info['nsplit']} marked={(gb['mask'] == 3).sum()}; "
          f"oracle nb={ob['x'].size} splits={onsplit} marked={(ob['mask'] == 3).sum()}", flush=True)
    assert (ob["mask"] == 3).sum() > 0 and onsplit > 0
    assert info["nsplit"] == onsplit and B.n == ob["x"].size
    assert np.array_equal(gb["mask"], ob["mask"]) and np.array_equal(gb["mq"], ob["mq"])
    for k in ("ds", "mref"):
        assert np.allclose(gb[k], ob[k], rtol=1e-12, atol=0), k
    for k in ("x", "y", "h"):
        assert float(np.max(np.abs(gb[k] - ob[k]))) < 1e-12, k
    # one adaptation against the oracle's background on both sides
    st = {k: s[k].copy() for k in ("x", "y", "u", "v", "p", "rho", "h", "mq", "kind")}
    st["mref"] = oracle.mref_lookup(d, st["x"], st["y"], st["h"], ob["x"], ob["y"], ob["h"],
                                    ob["mref"])
    o, oinfo = oracle.adapt(d, _prm(s), st, cap=cap)
    ps = P.Particles.from_arrays(s, cap)
    ainfo = ctx.adapt(ps, P.Background.from_arrays(ob, cap))
    print(f"[wake-adapt] gpu n={ps.n} split={ainfo['n_split']} merged={ainfo['merged']}; "
          f"oracle n={o['x'].size} split={oinfo['n_split']} merged={oinfo['merged']}", flush=True)
    assert ainfo["n_split"] == oinfo["n_split"] and ainfo["merged"] == oinfo["merged"]
    assert sum(oinfo["merged"]) > 0
    assert np.array_equal(ainfo["origin"].cpu().numpy(), oinfo["origin"])
    g = ps.numpy()
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind"):
        assert np.array_equal(g[k], o[k]), k
