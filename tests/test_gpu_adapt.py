"""GPU parity of the adaptation path against the oracle, through the C ABI:
split / merge x3 / shift x3 / h update index maps (origin, satellite flag,
counts) bit-exact, and the double-precision fields bit-exact as well (both
sides evaluate the same operations in the same order); background m_ref
lookup bit-exact; background update: counts, masks and positions exact,
sizes within 1e-12 (the geometric mean goes through log/exp)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import lib, odom

pytestmark = pytest.mark.gpu

ADAPT_FIELDS = ("x", "y", "u", "v", "p", "rho", "h", "mref")


def _inner_refine(nx=30, seed=2, frac=0.5, hdx=1.0, jitter=0.05):
    s = W.tgv(nx, seed=seed, hdx=hdx, jitter=jitter)
    m = s["m"][0]
    inner = (s["x"] > 0.1) & (s["x"] < 0.5) & (s["y"] > 0.1) & (s["y"] < 0.5)
    st = {k: s[k].copy() for k in ("x", "y", "u", "v", "p", "h", "mq", "kind")}
    st["rho"] = 1.0 + 0.01 * np.sin(2 * np.pi * s["x"]) * np.cos(2 * np.pi * s["y"])
    st["mref"] = np.where(inner, frac * m, m)
    return st, s


def _light_cloud(nx=24, seed=5):
    s = W.tgv(nx, seed=seed)
    rng = np.random.default_rng(seed)
    n = s["x"].size
    st = {k: s[k].copy() for k in ("x", "y", "u", "v", "p", "h", "kind")}
    st["mq"] = (s["mq"] * rng.uniform(0.2, 0.6, n)).astype(np.int64)
    st["h"] = s["h"] * rng.uniform(0.8, 1.6, n)
    st["mref"] = np.full(n, s["m"][0])
    st["rho"] = np.ones(n)
    return st, s


def _run_gpu_adapt(P, st, q, dom, hdx, capacity, h_hi):
    cfg = P.Config(lo=dom.lo, hi=dom.hi, periodic=dom.periodic, h_lo=float(st["h"].min()) * 0.5,
                   h_hi=h_hi, precision=P.SPH_FP64, hdx=hdx, mass_q=q)
    ctx = P.Context(cfg, capacity)
    ps = P.Particles.from_arrays(st, capacity)
    info = ctx.adapt(ps)
    return ps, info


@pytest.mark.parametrize("case", ["inner_half", "inner_quarter", "light_cloud"])
def test_adapt_bitexact(case):
    P = lib()
    if case == "light_cloud":
        st, s = _light_cloud()
        hdx = 1.0
    else:
        st, s = _inner_refine(frac=0.5 if case == "inner_half" else 0.25)
        hdx = 1.0
    q = s["mass_q"]
    dom = s["domain"]
    n = st["x"].size
    cap = 7 * n + 16
    print(f"[adapt] case={case} n={n}", flush=True)
    o, oinfo = oracle.adapt(odom(dom), oracle.Prm(mass_q=q, hdx=hdx), st, cap=cap)
    ps, info = _run_gpu_adapt(P, st, q, dom, hdx, cap, float(st["h"].max()) * 2)
    g = ps.numpy()
    print(f"[adapt] gpu n={ps.n} split={info['n_split']} merged={info['merged']} "
          f"oracle n={o['x'].size} split={oinfo['n_split']} merged={oinfo['merged']}", flush=True)
    assert info["n_split"] == oinfo["n_split"] and info["merged"] == oinfo["merged"]
    assert ps.n == o["x"].size
    assert np.array_equal(info["origin"].cpu().numpy(), oinfo["origin"])
    assert np.array_equal(info["sat"].cpu().numpy(), oinfo["sat"])
    assert np.array_equal(g["mq"], o["mq"]) and g["mq"].sum() == st["mq"].sum()
    mism = {k: int(np.sum(g[k] != o[k])) for k in ADAPT_FIELDS}
    maxd = {k: float(np.max(np.abs(g[k] - o[k]))) for k in ADAPT_FIELDS}
    print(f"[adapt] mismatches={mism} maxdiff={maxd}", flush=True)
    for k in ADAPT_FIELDS:
        assert mism[k] == 0, (k, mism[k], maxd[k])


def test_adapt_capacity_two_phase():
    P = lib()
    st, s = _inner_refine(nx=16, frac=0.25)
    n = st["x"].size
    cap = n + 10
    cfg = P.Config(h_lo=float(st["h"].min()) * 0.5, h_hi=float(st["h"].max()) * 2,
                   mass_q=s["mass_q"], precision=P.SPH_FP64)
    ctx = P.Context(cfg, cap)
    ps = P.Particles.from_arrays(st, cap)
    before = ps.numpy()
    info = ctx.adapt(ps)
    assert info.get("error") == P.SPH_E_CAPACITY
    assert info["n_required"] == n + 6 * info["n_split"] > cap
    after = ps.numpy()
    assert ps.n == n
    for k in before:
        assert np.array_equal(before[k], after[k]), k


def test_mref_lookup_bitexact():
    P = lib()
    a = W.random_varh(3000, seed=31, h_lo=0.004, ratio=3)
    b = W.random_varh(800, seed=32, h_lo=0.01, ratio=2)
    bm = np.random.default_rng(1).uniform(1, 2, 800)
    exp = oracle.mref_lookup(odom(a["domain"]), a["x"], a["y"], a["h"], b["x"], b["y"], b["h"], bm)
    cfg = P.Config(h_lo=0.004, h_hi=0.02)
    ctx = P.Context(cfg, 3000)
    st = {"x": a["x"], "y": a["y"], "h": a["h"], "mq": np.ones(3000, np.int64)}
    ps = P.Particles.from_arrays(st)
    bg = P.Background.from_arrays({"x": b["x"], "y": b["y"], "h": b["h"], "ds": b["h"],
                                   "mref": bm, "mask": np.zeros(800, np.int32),
                                   "mq": np.ones(800, np.int64)})
    ctx.mref_lookup(ps, bg)
    assert np.array_equal(ps.mref[:3000].cpu().numpy(), exp)


def test_background_square():
    """Background initialisation around a unit square (section 3.3 example):
    ds 0.1 -> 0.4, C_r = 1.2, 24 passes."""
    P = lib()
    dom = W.Domain((-4.0, -4.0), (4.0, 4.0), (False, False))
    bg = W.background_lattice(dom, 0.4, 1.2, 1.0)
    sol = W.square_solid(0.0, 0.0, 1.0, 0.1, 1.2, layers=3)
    passes = 24
    bp = oracle.BgPrm(cr=1.2, ds_min=0.1, ds_max=0.4, mass_q=bg["mass_q"])
    ob, onsplit = oracle.bg_update(odom(dom), bp, bg, sol, passes, cap=50000)
    cfg = P.Config(lo=dom.lo, hi=dom.hi, periodic=dom.periodic, h_lo=0.05, h_hi=0.8, cr=1.2,
                   ds_min=0.1, ds_max=0.4, bg_mass_q=bg["mass_q"], mass_q=bg["mass_q"])
    ctx = P.Context(cfg, 50000)
    B = P.Background.from_arrays(bg, 50000)
    S = P.Particles.from_arrays({"x": sol["x"], "y": sol["y"], "h": sol["h"],
                                 "mq": np.ones(sol["x"].size, np.int64)})
    nsplit = ctx.bg_update(B, S, passes)
    gb = B.numpy()
    print(f"[bg] gpu n={B.n} splits={nsplit} oracle n={ob['x'].size} splits={onsplit}", flush=True)
    assert nsplit == onsplit and B.n == ob["x"].size
    assert np.array_equal(gb["mask"], ob["mask"]) and np.array_equal(gb["mq"], ob["mq"])
    for k in ("ds", "mref"):
        assert np.allclose(gb[k], ob[k], rtol=1e-12, atol=0), k
    for k in ("x", "y", "h"):
        d = float(np.max(np.abs(gb[k] - ob[k])))
        print(f"[bg] {k} maxdiff={d}", flush=True)
        assert d < 1e-12, k


def test_vorticity_vs_oracle():
    P = lib()
    s = W.tgv(40, seed=9)
    rng = np.random.default_rng(9)
    s["rho"] = 1.0 + 0.01 * rng.standard_normal(s["x"].size)
    ctx = P.Context(P.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                                 mass_q=s["mass_q"]), s["x"].size)
    w = ctx.vorticity(P.Particles.from_arrays(s)).cpu().numpy()
    rp, col = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"])
    o = oracle.vorticity(odom(s["domain"]), s["x"], s["y"], s["u"], s["v"], s["h"],
                         s["mq"] * s["mass_q"], s["rho"], rp, col)
    err = float(np.linalg.norm(w - o) / np.linalg.norm(o))
    print(f"[vorticity] rel err {err:.2e}", flush=True)
    assert err < 1e-12


def test_background_solution_adaptivity():
    """Section 3.3, solution adaptivity: |vorticity| of a Taylor-Green field
    carried to a coarse background; background particles above half the
    maximum are refined to ds_min and the rest graded by C_r."""
    P = lib()
    s = W.tgv(40, seed=10)
    dom = s["domain"]
    bg = W.background_lattice(dom, 0.2, 1.2, 1.0)
    k_frac, passes = 0.5, 10
    rho = np.ones(s["x"].size)
    m = s["mq"] * s["mass_q"]
    rp, col = oracle.neighbors(odom(dom), s["x"], s["y"], s["h"])
    om = np.abs(oracle.vorticity(odom(dom), s["x"], s["y"], s["u"], s["v"], s["h"], m, rho, rp, col))
    phi = oracle.shepard_to_bg(odom(dom), bg["x"], bg["y"], bg["h"], s["x"], s["y"], s["h"], om)
    thresh = k_frac * om.max()
    empty = {"x": np.zeros(0), "y": np.zeros(0), "h": np.zeros(0)}
    bp = oracle.BgPrm(cr=1.2, ds_min=0.025, ds_max=0.2, mass_q=bg["mass_q"])
    ob, onsplit = oracle.bg_update(odom(dom), bp, bg, empty, passes, cap=40000, phi=phi,
                                   phi_thresh=thresh)
    cfg = P.Config(lo=dom.lo, hi=dom.hi, periodic=dom.periodic, h_lo=float(s["h"].min()), h_hi=0.5,
                   cr=1.2, ds_min=0.025, ds_max=0.2, bg_mass_q=bg["mass_q"], mass_q=s["mass_q"])
    ctx = P.Context(cfg, 40000)
    B = P.Background.from_arrays(bg, 40000)
    S = P.Particles.from_arrays({"x": np.zeros(0), "y": np.zeros(0), "h": np.zeros(0),
                                 "mq": np.zeros(0, np.int64)}, capacity=1)
    F = P.Particles.from_arrays(s)
    info = ctx.bg_update_solution(B, S, F, k_frac, passes)
    gb = B.numpy()
    print(f"[bg-sol] gpu n={B.n} splits={info['nsplit']} oracle n={ob['x'].size} "
          f"splits={onsplit} max|w| gpu={info['omega_max']:.12g} oracle={om.max():.12g}", flush=True)
    assert info["omega_max"] == pytest.approx(om.max(), rel=1e-12)
    assert onsplit > 0 and (ob["mask"] == 3).sum() > 0
    assert info["nsplit"] == onsplit and B.n == ob["x"].size
    assert np.array_equal(gb["mask"], ob["mask"]) and np.array_equal(gb["mq"], ob["mq"])
    for k in ("ds", "mref"):
        assert np.allclose(gb[k], ob[k], rtol=1e-12, atol=0), k
    for k in ("x", "y", "h"):
        assert float(np.max(np.abs(gb[k] - ob[k]))) < 1e-12, k
