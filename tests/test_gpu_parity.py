"""GPU parity of the HIP hot path against the FP64 CPU oracle, through the
C ABI: neighbour lists bit-exact, rates within the stated tolerances
(FP64 pair arithmetic: 1e-12, FP32 pair arithmetic: 1e-5, both normwise per
field and per particle against the oracle's sum of term magnitudes), PEC
steps against the oracle's trajectory."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, csr_np, ctx_for, dt_of, lib, odom, particles, rel_norm, with_fields

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")


def _neighbor_case(name):
    if name == "periodic":
        return W.random_varh(3000, seed=101, h_lo=0.004, ratio=8)
    if name == "open":
        return W.random_varh(3000, seed=102, h_lo=0.004, ratio=8, periodic=(False, False))
    if name == "clustered":
        return W.clustered_varh(4000, seed=103)
    if name == "ratio64":
        return W.clustered_varh(4000, seed=104, h_lo=0.002, ratio=64)
    if name == "tgv":
        return W.tgv(50, seed=1)
    raise KeyError(name)


@pytest.mark.parametrize("case", ["periodic", "open", "clustered", "ratio64", "tgv"])
def test_neighbors_bitexact(case):
    P = lib()
    s = _neighbor_case(case)
    print(f"[neighbors] case={case} n={s['x'].size}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    rp, col = csr_np(*ctx.build_neighbors(ps))
    orp, ocol = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"])
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)


def test_neighbors_edge_cases():
    P = lib()
    # empty, single particle, particles on cell boundaries and at the period
    base = W.random_varh(10, seed=5, h_lo=0.05, ratio=1.0)
    ctx = ctx_for(P, base, P.SPH_FP64, capacity=64)
    for xs, ys in (([], []), ([0.5], [0.5]), ([0.0, 0.15, 0.3, 0.999999], [0.0, 0.0, 0.0, 0.5])):
        s = {"x": np.array(xs, float), "y": np.array(ys, float),
             "h": np.full(len(xs), 0.05), "domain": base["domain"]}
        ps = particles(P, s, capacity=64)
        rp, col = csr_np(*ctx.build_neighbors(ps))
        orp, ocol = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"], "brute")
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    # capacity: too small a CSR buffer is reported, required size returned
    s = W.random_varh(50, seed=6, h_lo=0.05, ratio=1.0)
    ps = particles(P, s, capacity=64)
    with pytest.raises(P.SphError) as e:
        ctx.build_neighbors(ps, nnz_cap=10)
    assert e.value.code == P.SPH_E_CAPACITY


# Particle counts around the neighbour sort's tile of 2,048 keys (one
# workgroup per tile and digit pass): below, at and just past a tile, and a
# ragged count of several tiles.
@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 6145])
def test_neighbors_sort_tile_counts(n):
    P = lib()
    s = W.random_varh(n, seed=300 + n % 97, h_lo=0.006, ratio=4)
    print(f"[neighbors] tile counts n={n}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64)
    rp, col = csr_np(*ctx.build_neighbors(particles(P, s)))
    orp, ocol = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"])
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


def test_neighbors_sort_skewed_digits():
    """Most keys in a few digit buckets: 11,000 of 12,000 particles packed in
    a square of side 0.05 (one level, a handful of level-0 cells, so every
    sort pass sees long runs of equal digits across several tiles), the rest
    with larger h in a band beyond the reach of the square."""
    P = lib()
    rng = np.random.default_rng(311)
    nd, ns = 11000, 1000
    x = np.concatenate([0.4 + 0.05 * rng.random(nd), 0.7 + 0.3 * rng.random(ns)])
    y = np.concatenate([0.6 + 0.05 * rng.random(nd), rng.random(ns)])
    h = np.concatenate([np.full(nd, 0.0006), 0.02 * np.exp(rng.uniform(0, 1, ns))])
    s = {"x": x, "y": y, "h": h, "domain": W.Domain((0.0, 0.0), (1.0, 1.0), (True, True))}
    ctx = ctx_for(P, s, P.SPH_FP64)
    rp, col = csr_np(*ctx.build_neighbors(particles(P, s)))
    orp, ocol = oracle.neighbors(odom(s["domain"]), s["x"], s["y"], s["h"])
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


def _rates_case(name):
    if name == "tgv":
        s = W.tgv(50, seed=1)
        s["params"] = dict(s["params"])
        return s
    if name == "varh":
        return with_fields(W.random_varh(2500, seed=7, h_lo=0.01, ratio=4), seed=7)
    if name == "clustered":
        return with_fields(W.clustered_varh(3000, seed=8, h_lo=0.006, ratio=16), seed=8)
    raise KeyError(name)


def _oracle_rates(s, dt):
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                     hdx=s["params"]["hdx"], mass_q=s["mass_q"])
    return oracle.rates(odom(s["domain"]), prm, s["x"], s["y"], s["u"], s["v"], s["p"], s["h"],
                        s["mq"] * s["mass_q"], dt)


@pytest.mark.parametrize("case", ["tgv", "varh", "clustered"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rates_vs_oracle(case, prec):
    P = lib()
    s = _rates_case(case)
    dt = 1e-4
    precision = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    print(f"[rates] case={case} prec={prec} n={s['x'].size}", flush=True)
    ctx = ctx_for(P, s, precision)
    r = ctx.rates(particles(P, s), dt)
    o = _oracle_rates(s, dt)
    assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])
    check_rates(r, o, prec, case)


def test_list_reuse_after_moves():
    """The rate passes reuse a neighbour list built with a skin while every
    particle moved less than the allowance, and rebuild otherwise.  Rates
    must match the oracle after a small move (list reused), after a move
    larger than the allowance (list rebuilt) and after changing h."""
    P = lib()
    s = _rates_case("clustered")
    ctx = ctx_for(P, s, P.SPH_FP64)
    rng = np.random.default_rng(3)
    dt = 1e-4
    for label, scale in (("initial", 0.0), ("small", 0.02), ("large", 0.6), ("small2", 0.02)):
        s = dict(s)
        jit = scale * s["h"]
        s["x"] = s["x"] + rng.uniform(-jit, jit)
        s["y"] = s["y"] + rng.uniform(-jit, jit)
        lo, hi = s["domain"].lo, s["domain"].hi
        s["y"] = lo[1] + np.mod(s["y"] - lo[1], hi[1] - lo[1])
        s["x"] = np.clip(s["x"], lo[0], np.nextafter(hi[0], lo[0]))
        r = ctx.rates(particles(P, s), dt)
        o = _oracle_rates(s, dt)
        assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"]), label
        check_rates(r, o, "fp64", label)
    s = dict(s)
    s["h"] = s["h"] * 1.05
    r = ctx.rates(particles(P, s), dt)
    o = _oracle_rates(s, dt)
    assert np.array_equal(r["nnb"].cpu().numpy(), o["nnb"])


def test_pec_steps_vs_oracle():
    """Periodic Taylor-Green, 50x50, Re = 100, 20 PEC steps in FP64."""
    P = lib()
    s = W.tgv(50, seed=1)
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    print("[step] tgv 50x50 fp64 20 steps", flush=True)
    ctx.step(ps, dt_of(s), 20)
    g = ps.numpy()
    o = oracle.step(oracle.Dom(), oracle.Prm(mass_q=s["mass_q"]), s, dt_of(s), 20)
    for k in ("x", "y"):
        d = g[k] - o[k]
        d = d - np.round(d)
        assert np.abs(d).max() < 1e-12
    for k in ("u", "v", "p", "rho"):
        assert rel_norm(g[k], o[k]) < 1e-11, k


def test_tgv_decay_gpu_fp32():
    """Closed-form check on the GPU: kinetic energy of the periodic vortex
    decays as exp(-16 pi^2 t / Re) over 100 PEC steps (section 4.1)."""
    P = lib()
    s = W.tgv(50, seed=1)
    ctx = ctx_for(P, s, P.SPH_FP32)
    ps = particles(P, s)
    ke0 = ctx.diagnostics(ps)["ke"]
    ctx.step(ps, dt_of(s), 100)
    d = ctx.diagnostics(ps)
    T = 100 * dt_of(s)
    assert d["ke"] / ke0 == pytest.approx(math.exp(-16 * math.pi ** 2 * T / 100), rel=1e-3)
    assert d["mq_total"] == int(s["mq"].sum())


def test_channel_full_size_sampled():
    """Channel with a cylinder at its full size (~2e5 particles, 9 h levels):
    CSR rows of a seeded sample match brute force exactly; FP32 and FP64
    rates match the oracle within tolerance on every particle."""
    P = lib()
    s = W.channel_cylinder(seed=2)
    n = s["x"].size
    print(f"[channel] n={n}", flush=True)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(n, 200, replace=False))
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    rp, col = csr_np(*ctx.build_neighbors(ps))
    d = odom(s["domain"])
    orp, ocol = oracle.cross_neighbors(d, s["x"][sample], s["y"][sample], s["h"][sample],
                                       s["x"], s["y"], s["h"], "brute")
    for k, i in enumerate(sample):
        assert np.array_equal(col[rp[i]:rp[i + 1]], ocol[orp[k]:orp[k + 1]])
    dt = dt_of(s)
    # the cylinder's solid particles take the wall boundary pass of section 2.2
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                     hdx=s["params"]["hdx"], mass_q=s["mass_q"])
    # and its inlet/outlet particles the characteristic rule
    o = oracle.rates_k(odom(s["domain"]), prm, s, dt, io=s["params"]["io_ref"])
    for prec, name in ((P.SPH_FP64, "fp64"), (P.SPH_FP32, "fp32")):
        c2 = ctx_for(P, s, prec)
        r = c2.rates(particles(P, s), dt)
        check_rates(r, o, name, "channel")
