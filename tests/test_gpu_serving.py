"""GPU tests of the serving pool (sph_pool_*) through the C ABI.  The pool
advances every resident simulation with one batched step (one launch per
kernel for all of them) captured into a graph.  A simulation's result is
the same bit for bit alone, in a mix (other sizes, Reynolds numbers and
time steps, FP32 and FP64 together, an open box with variable h, others
admitted and retired mid-run) and stepped eagerly by sph_pec on a lean
context with the same list; the FP64 and FP32 pool paths follow the oracle;
admission by free ranges refuses and later accepts; the pair counter
matches the neighbour count."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import dt_of, lib, odom, rel_norm, with_fields

pytestmark = pytest.mark.gpu

KEYS = ("x", "y", "u", "v", "p", "rho")


def _tgv(P, nx, seed, re, prec, skin=0.0):
    s = W.tgv(nx, seed=seed, re=re)
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                       precision=prec, mass_q=s["mass_q"], list_skin=skin, lean=1, list_k=64)
    return s, cfg


def _varh(P, prec, skin=0.0):
    """An open box with a 1:4 smoothing-length range (several levels)."""
    s = with_fields(W.random_varh(1800, seed=41, h_lo=0.012, ratio=4, periodic=(False, False)),
                    seed=41)
    s["dt"] = 1e-4
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                       precision=prec, mass_q=s["mass_q"], list_skin=skin, lean=1, list_k=64)
    return s, cfg


def _read(P, pool, sid, n):
    Q = P.Particles(n)
    pool.read(sid, Q)
    return Q.numpy()


def _eager(P, s, cfg, nsteps):
    ctx = P.Context(cfg, s["x"].size)
    E = P.Particles.from_arrays(s)
    ctx.step(E, dt_of(s), nsteps)
    return E.numpy()


@pytest.mark.parametrize("skin", [0.0, 0.05])
def test_alone_vs_mix_vs_eager(skin):
    """With no list skin every evaluation rebuilds every simulation's list;
    with a skin each simulation keeps its list until one of its particles
    moved too far (rebuilds within the first steps here), whatever the other
    residents do: either way a simulation's state is the same bits alone,
    in the mix (across a change of the resident set) and in a context."""
    P = lib()
    s, cfg = _tgv(P, 40, 31, 100.0, P.SPH_FP32, skin)
    n = s["x"].size
    v, vcfg = _varh(P, P.SPH_FP64, skin)
    others = [_tgv(P, nx, sd, re, pr, skin) for nx, sd, re, pr in
              ((70, 32, 400.0, P.SPH_FP32), (25, 33, 900.0, P.SPH_FP64), (55, 34, 250.0, P.SPH_FP32))]
    print(f"[pool] alone vs mix n={n} skin={skin}", flush=True)
    alone = P.Pool(1 << 28, max_sims=8)
    a = alone.admit(cfg, P.Particles.from_arrays(s), dt_of(s))
    mix = P.Pool(1 << 28, max_sims=8)
    ids = [mix.admit(c, P.Particles.from_arrays(o), dt_of(o)) for o, c in others[:2]]
    m = mix.admit(cfg, P.Particles.from_arrays(s), dt_of(s))
    mv = mix.admit(vcfg, P.Particles.from_arrays(v), dt_of(v))
    assert a is not None and m is not None and mv is not None and all(i is not None for i in ids)
    for k in range(5):
        alone.step(1)
        mix.step(1)
        if k == 2:
            # the resident set changes mid-run: one retired, one admitted
            mix.retire(ids[0])
            o, c = others[2]
            ids.append(mix.admit(c, P.Particles.from_arrays(o), dt_of(o)))
            assert ids[-1] is not None
        ga, gm = _read(P, alone, a, n), _read(P, mix, m, n)
        ge = _eager(P, s, cfg, k + 1)
        for key in KEYS:
            assert np.array_equal(ga[key], gm[key]), (k, key)
            assert np.array_equal(ga[key], ge[key]), (k, key)
    # the open variable-h FP64 simulation in the mix against its eager run
    gv, ev = _read(P, mix, mv, v["x"].size), _eager(P, v, vcfg, 5)
    for key in KEYS:
        assert np.array_equal(gv[key], ev[key]), key
    alone.step(10)
    mix.step(10)
    ga, gm = _read(P, alone, a, n), _read(P, mix, m, n)
    for key in KEYS:
        assert np.array_equal(ga[key], gm[key]), key
    st = mix.stats(m, pairs=True)
    assert st["steps"] == 15 and st["last_ms"] > 0 and st["pair_evals"] > 0
    alone.close()
    mix.close()


@pytest.mark.parametrize("prec,skin", [("fp64", 0.0), ("fp32", 0.0), ("fp64", 0.05), ("fp32", 0.05)])
def test_pool_follows_oracle(prec, skin):
    """Ten pool steps of a periodic Taylor-Green vortex (alone, and beside
    another simulation) against the oracle's trajectory, per particle:
    positions (minimum image) and u, v, p, rho relative to their largest
    magnitude.  FP64 within 1e-12, FP32 within 2e-6 (the FP32 rates are
    within about 1e-6 of the FP64 ones per particle, integrated over ten
    steps of dt = 4.5e-4).  With a list skin the simulation keeps its list
    across steps and rebuilds it when its particles moved too far."""
    P = lib()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    s, cfg = _tgv(P, 30, 35, 100.0, pr, skin)
    o2, c2 = _tgv(P, 45, 36, 600.0, P.SPH_FP32, skin)
    pool = P.Pool(1 << 27, max_sims=4)
    other = pool.admit(c2, P.Particles.from_arrays(o2), dt_of(o2))
    sid = pool.admit(cfg, P.Particles.from_arrays(s), dt_of(s))
    assert other is not None and sid is not None
    pool.step(10)
    g = _read(P, pool, sid, s["x"].size)
    o = oracle.step(oracle.Dom(), oracle.Prm(mass_q=s["mass_q"], nu=s["params"]["nu"]), s, dt_of(s), 10)
    tol = 1e-12 if prec == "fp64" else 2e-6
    errs = {}
    for k in ("x", "y"):
        d = g[k] - o[k]
        d = d - np.round(d)
        errs[k] = float(np.abs(d).max() / np.sqrt(1.0 / s["x"].size))
    for k in ("u", "v", "p", "rho"):
        errs[k] = float(np.abs(g[k] - o[k]).max() / np.abs(o[k]).max())
    print(f"[pool-oracle] {prec} skin={skin} {errs}", flush=True)
    for k, e in errs.items():
        assert e < tol, (k, e)
    pool.close()


def test_admission_by_free_ranges():
    P = lib()
    s, cfg = _tgv(P, 50, 36, 100.0, P.SPH_FP32)
    n = s["x"].size
    fp = P.footprint(cfg, n)
    assert fp > n * 500
    pool = P.Pool(16 << 20, max_sims=64)
    info0 = pool.info()
    cap = info0["slots_total"]
    k_fit = cap // n
    assert k_fit >= 2
    Pn = P.Particles.from_arrays(s)
    ids = [pool.admit(cfg, Pn, dt_of(s)) for _ in range(k_fit)]
    assert all(i is not None for i in ids)
    info = pool.info()
    assert info["resident"] == k_fit and info["particles"] == k_fit * n
    assert info["slots_used"] == k_fit * n
    assert pool.admit(cfg, Pn, dt_of(s)) is None          # full: SPH_E_AGAIN
    assert pool.info()["resident"] == k_fit               # nothing changed
    pool.step(2)
    pool.retire(ids[0])
    c = pool.admit(cfg, Pn, dt_of(s))                      # the freed range is reused
    assert c is not None
    pool.step(1)
    assert pool.stats(ids[1])["steps"] == 3 and pool.stats(c)["steps"] == 1
    for i in ids[1:] + [c]:
        pool.retire(i)
    info = pool.info()
    assert info["resident"] == 0 and info["slots_used"] == 0 and info["tables_used"] == 0
    assert info["largest_free"] == info["slots_total"]   # ranges coalesced
    # a simulation with boundary particles is refused (the pool is fluid only)
    w = W.wall_box(nx=12, ny=12, layers=3)
    wcfg = P.config_for(w["domain"], {"rho0": 1.0, "cs": 10.0, "nu": 0.01, "hdx": 1.0},
                        float(w["h"].min()), float(w["h"].max()), mass_q=w["mass_q"])
    ps = P.Particles.from_arrays(dict(w, u=np.zeros(w["x"].size), v=np.zeros(w["x"].size),
                                      p=np.zeros(w["x"].size)))
    c = ps.c()
    import ctypes
    sid = ctypes.c_int32(-1)
    rc = pool.lib.sph_pool_admit(pool._h, ctypes.byref(wcfg.c()), ctypes.byref(c), 1e-4,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 ctypes.byref(sid))
    assert rc == P.SPH_E_INVAL
    pool.close()


def test_pair_counter():
    P = lib()
    s, cfg = _tgv(P, 45, 37, 100.0, P.SPH_FP64)
    n = s["x"].size
    rp, col = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"])
    pairs0 = col.size - n
    pool = P.Pool(1 << 27, max_sims=4)
    sid = pool.admit(cfg, P.Particles.from_arrays(s), dt_of(s))
    pool.step(1)
    pe = pool.stats(sid, pairs=True)["pair_evals"]
    # the first evaluation sees exactly the initial pairs; the half step moves
    # particles by far less than a spacing
    assert abs(pe - 2 * pairs0) <= 2e-3 * pe
    pool.retire(sid)
    assert pool.stats(sid, pairs=True)["pair_evals"] == pe
    pool.close()
