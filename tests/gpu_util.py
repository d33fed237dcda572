"""Shared helpers of the GPU parity tests (load the HIP library, move
workload dicts to device, compare against the oracle)."""
import numpy as np

import oracle
import workloads as W


def dt_of(s):
    """The time step of a workload (oracle.dt_for: eq. timestep from its
    h_min and U unless it names a dt)."""
    return oracle.dt_for(s)


def lib():
    import paper_2107_01276_amd as P
    P.load_library()
    return P


def odom(d):
    return oracle.Dom(tuple(d.lo), tuple(d.hi), tuple(d.periodic))


def ctx_for(P, s, precision, capacity=None, h=None, **kw):
    h = s["h"] if h is None else h
    cfg = P.config_for(s["domain"], s.get("params", {"rho0": 1.0, "cs": 10.0, "nu": 0.01, "hdx": 1.0}),
                       float(np.min(h)), float(np.max(h)), precision=precision,
                       mass_q=s.get("mass_q", 2.0 ** -60), **kw)
    return P.Context(cfg, capacity or len(s["x"]))


def particles(P, s, capacity=None):
    d = dict(s)
    if "mq" not in d:
        d["mq"] = np.ones(len(d["x"]), np.int64)
    return P.Particles.from_arrays(d, capacity)


def rel_norm(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def csr_np(rp, col):
    return rp.cpu().numpy(), col.cpu().numpy()


def with_fields(s, seed=0):
    """Adds smooth velocity/pressure/mass fields to a position set."""
    rng = np.random.default_rng(seed)
    x, y = s["x"], s["y"]
    n = x.size
    out = dict(s)
    out["u"] = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.01 * rng.standard_normal(n)
    out["v"] = -np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
    out["p"] = 0.3 * np.cos(2 * np.pi * x) + 0.1 * rng.standard_normal(n)
    m = 2.0 * s["h"] ** 2  # mass ~ rho0 dx^2 with h ~ dx
    q = W.mass_quantum(1.05 * m.max() * 2)
    out["mq"] = W.quantize_mass(m, q)
    out["mass_q"] = q
    out["m"] = out["mq"] * q
    out["params"] = {"rho0": 1.0, "cs": 10.0, "nu": 0.01, "hdx": 1.0}
    return out


RATE_FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")
# Bounds of the rate parity tests.  Normwise: ||a - b||_2 / ||b||_2 per
# field.  Per particle (condition-aware): max_i |a_i - b_i| / s_i, with s_i the
# oracle's sum of the magnitudes of the terms b_i adds up (oracle.rate_scales).
# FP64 pair arithmetic: both 1e-12.  FP32 pair arithmetic: the target's 1e-5
# normwise; per particle 1e-5 as well, which leaves room for about 160 ulp
# (2^-24) of the terms: a pair term takes some 10-20 roundings, and the
# quintic's derivative loses up to a factor 10 to cancellation at the
# distances of split children (q ~ 0.4), while every sum is compensated.
TOL = {"fp64": {"norm": 1e-12, "cond": 1e-12}, "fp32": {"norm": 1e-5, "cond": 1e-5}}


def rate_errors(r, o, fields=RATE_FIELDS):
    """Per field: normwise relative error, the condition-aware per-particle
    error against o["scale"], and max |a - b| / max |b|."""
    out = {}
    for k in fields:
        a = r[k].cpu().numpy() if hasattr(r[k], "cpu") else np.asarray(r[k])
        b = np.asarray(o[k], np.float64)
        mb = float(np.abs(b).max()) if b.size else 0.0
        mx = float(np.abs(a - b).max()) if b.size else 0.0
        out[k] = {"norm": rel_norm(a, b), "cond": oracle.cond_error(a, b, o["scale"][k]),
                  "maxabs": mx / mb if mb > 0 else mx}
    return out


def check_rates(r, o, prec, label="", fields=RATE_FIELDS, tol=None):
    """Asserts the normwise and per-particle bounds of TOL[prec] on every
    field; prints the errors first."""
    t = dict(TOL[prec])
    if tol:
        t.update(tol)
    e = rate_errors(r, o, fields)
    worst = {k: (f"{v['norm']:.2e}", f"{v['cond']:.2e}") for k, v in e.items()}
    print(f"[rates] {label} {prec} (norm, cond) {worst}", flush=True)
    for k, v in e.items():
        assert v["norm"] < t["norm"], (label, prec, k, "norm", v["norm"])
        assert v["cond"] < t["cond"], (label, prec, k, "cond", v["cond"])
    return e
