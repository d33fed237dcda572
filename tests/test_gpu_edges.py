"""Degenerate inputs through the C ABI against the oracle: the empty set and
a single particle (rates, PEC steps, adaptation, diagnostics), coincident
particles (r = 0 pairs other than the self pair) and isolated particles
(no neighbour inside the support, so beta <= 0 and the scaled sums drop)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, lib, rel_norm

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")
H = 0.05
DOM = W.Domain((0.0, 0.0), (1.0, 1.0), (True, True))
Q = W.mass_quantum(1.05 * 0.01)


def _set(x, y, seed=0):
    n = len(x)
    rng = np.random.default_rng(seed)
    mq = W.quantize_mass(np.full(n, 0.0025), Q)
    return {"x": np.asarray(x, float), "y": np.asarray(y, float), "h": np.full(n, H),
            "u": 0.2 * rng.standard_normal(n), "v": 0.2 * rng.standard_normal(n),
            "p": 0.3 + 0.1 * rng.standard_normal(n), "rho": np.ones(n), "mq": mq,
            "mref": np.full(n, 0.0025), "kind": np.zeros(n, np.int32), "m": mq * Q}


def _ctx(P, prec, cap=64):
    cfg = P.Config(lo=DOM.lo, hi=DOM.hi, periodic=DOM.periodic, h_lo=H / 3, h_hi=H,
                   precision=prec, mass_q=Q, nu=0.01)
    return P.Context(cfg, cap)


def _compare_rates(P, prec, s):
    ctx = _ctx(P, prec)
    r = ctx.rates(P.Particles.from_arrays(s, 64), 1e-4)
    o = oracle.rates(oracle.Dom(DOM.lo, DOM.hi, DOM.periodic), oracle.Prm(mass_q=Q, nu=0.01),
                     s["x"], s["y"], s["u"], s["v"], s["p"], s["h"], s["m"], 1e-4)
    n = s["x"].size
    assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])
    for k in FIELDS:
        a = r[k].cpu().numpy()
        assert a.shape == (n,) and np.all(np.isfinite(a)), k
    if n:
        # a field of all zeros (no interacting pair) must be matched exactly
        check_rates(r, o, "fp64" if prec == P.SPH_FP64 else "fp32", f"edges n={n}",
                    tol={"norm": np.inf})
        for k in FIELDS:
            if not np.any(o[k]):
                assert not np.any(r[k].cpu().numpy()), k
    return r


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_empty_and_single(prec):
    P = lib()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    d = oracle.Dom(DOM.lo, DOM.hi, DOM.periodic)
    for n in (0, 1):
        s = _set([0.5] * n, [0.5] * n)
        print(f"[edges] prec={prec} n={n}", flush=True)
        r = _compare_rates(P, pr, s)
        if n == 1:
            assert r["beta"].cpu().numpy()[0] <= 0.0 and r["dpdt"].cpu().numpy()[0] == 0.0
        # steps
        ctx = _ctx(P, pr)
        ps = P.Particles.from_arrays(s, 64)
        ctx.step(ps, 1e-4, 3)
        o = oracle.step(d, oracle.Prm(mass_q=Q, nu=0.01), s, 1e-4, 3)
        g = ps.numpy()
        for k in ("x", "y", "u", "v", "p"):
            assert g[k].shape == (n,) and np.allclose(g[k], o[k], rtol=1e-12, atol=0), k
        dg = ctx.diagnostics(ps)
        assert dg["n"] == n and dg["mq_total"] == int(s["mq"].sum())
        # adaptation: a single particle heavier than 1.05 m_ref splits into seven
        st = dict(s, mref=np.full(n, 0.0025 / 8))
        ctx = _ctx(P, pr)
        ps = P.Particles.from_arrays(st, 64)
        info = ctx.adapt(ps)
        oa, oinfo = oracle.adapt(d, oracle.Prm(mass_q=Q, nu=0.01), st, cap=64)
        assert ps.n == oa["x"].size == 7 * n and info["n_split"] == oinfo["n_split"] == n
        g = ps.numpy()
        for k in ("x", "y", "h", "mq", "mref"):
            assert np.array_equal(g[k], oa[k]), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coincident_and_isolated(prec):
    P = lib()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    # a small lattice, two particles on top of each other inside it, a
    # coincident pair far from it, and isolated particles
    g = (np.arange(6) + 0.5) * (0.6 * H)
    X, Y = np.meshgrid(g + 0.1, g + 0.1, indexing="ij")
    x = list(X.ravel()) + [0.15, 0.6, 0.6, 0.85, 0.4]
    y = list(Y.ravel()) + [0.15, 0.6, 0.6, 0.15, 0.85]
    x[7], y[7] = x[8], y[8]  # two lattice particles coincide
    s = _set(x, y, seed=3)
    print(f"[edges] coincident/isolated prec={prec} n={len(x)}", flush=True)
    r = _compare_rates(P, pr, s)
    beta = r["beta"].cpu().numpy()
    assert np.all(beta[-2:] <= 0.0)          # isolated: only the self pair
    assert np.all(r["dpdt"].cpu().numpy()[-2:] == 0.0)
