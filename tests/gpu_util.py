"""Shared helpers of the GPU parity tests (load the HIP library, move
workload dicts to device, compare against the oracle)."""
import numpy as np

import oracle
import workloads as W


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
