"""GPU parity of the boundary particles (section 2.2) through the C ABI:
the wall/inlet/outlet boundary pass and the rates that use it against the
oracle (FP64 pair arithmetic 1e-12, FP32 1e-5, normwise per field), PEC
steps with walls and open boundaries against the oracle's trajectory, the
inlet/outlet update bit-exact, and the Couette start-up against its series
solution on the FP32 path."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, lib, odom, particles, rel_norm

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")
PRM = {"rho0": 1.0, "cs": 10.0, "nu": 0.05, "hdx": 1.2}


def _wall_case():
    s = W.wall_box(nx=24, ny=20, layers=3, jitter=0.1, seed=21)
    rng = np.random.default_rng(22)
    fl = s["kind"] == W.FLUID
    n = s["x"].size
    s["u"] = np.where(fl, 0.3 * np.sin(2 * np.pi * s["x"]) + 0.05 * rng.standard_normal(n), 0.0)
    s["v"] = np.where(fl, 0.2 * np.cos(2 * np.pi * s["x"]) * s["y"], 0.0)
    s["u"][(~fl) & (s["y"] > 0.5)] = 0.4       # top wall slides
    s["p"] = np.where(fl, 1.0 - 2.0 * s["y"] + 0.01 * rng.standard_normal(n), 0.0)
    s["rho"] = 1.0 + 0.01 * rng.standard_normal(n)
    s["params"] = dict(PRM)
    s["m"] = s["mq"] * s["mass_q"]
    return s


def _io_case():
    s = W.inout_strip(nx=30, ny=12, n_in=5, n_out=5, jitter=0.1, seed=23)
    rng = np.random.default_rng(24)
    n = s["x"].size
    fl = s["kind"] == W.FLUID
    s["u"] = np.where(fl, 1.0 + 0.05 * rng.standard_normal(n), s["u"])
    s["v"] = np.where(fl, 0.05 * rng.standard_normal(n), 0.0)
    s["p"] = np.where(fl, 0.1 * np.sin(np.pi * s["x"]), 0.0)
    s["params"] = dict(PRM)
    s["m"] = s["mq"] * s["mass_q"]
    return s


def _prm(s, body=(0.0, 0.0)):
    return oracle.Prm(rho0=1.0, cs=PRM["cs"], nu=PRM["nu"], hdx=PRM["hdx"], mass_q=s["mass_q"],
                      fx=body[0], fy=body[1])


IO_REF = (1.0, 0.0, 0.05)


def _io_kw(case):
    """Library and oracle arguments of the inlet/outlet rule of a case."""
    if case == "inout_char":
        return {"io_mode": 1, "io_ref": IO_REF}, IO_REF
    return {}, None


@pytest.mark.parametrize("case", ["wall", "inout", "inout_char"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_boundary_rates_vs_oracle(case, prec):
    P = lib()
    s = _wall_case() if case == "wall" else _io_case()
    body = (0.0, -2.0) if case == "wall" else (0.0, 0.0)
    kw, io = _io_kw(case)
    dt = 1e-4
    precision = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    print(f"[boundary] case={case} prec={prec} n={s['x'].size}", flush=True)
    ctx = ctx_for(P, s, precision, body_force=body, **kw)
    ps = particles(P, s)
    r = ctx.rates(ps, dt)
    o = oracle.rates_k(odom(s["domain"]), _prm(s, body), s, dt, io=io)
    check_rates(r, o, prec, case)
    # the boundary values written into the state (double in both paths)
    st = ps.numpy()
    for k, ok in (("p", "p_bc"), ("u", "u_bc"), ("v", "v_bc")):
        assert rel_norm(st[k], o[ok]) < 1e-13, k


@pytest.mark.parametrize("case", ["wall", "inout", "inout_char"])
def test_boundary_steps_vs_oracle(case):
    P = lib()
    s = _wall_case() if case == "wall" else _io_case()
    body = (0.0, -2.0) if case == "wall" else (0.0, 0.0)
    kw, io = _io_kw(case)
    dt = 2e-4
    print(f"[boundary-steps] case={case} n={s['x'].size}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64, body_force=body, **kw)
    ps = particles(P, s)
    ctx.step(ps, dt, 10)
    g = ps.numpy()
    o = oracle.step_k(odom(s["domain"]), _prm(s, body), s, dt, 10, io=io)
    for k in ("x", "y", "u", "v", "p", "rho"):
        e = rel_norm(g[k], o[k])
        print(f"[boundary-steps] {k} {e:.2e}", flush=True)
        assert e < 1e-10, (k, e)
    assert np.array_equal(g["kind"], o["kind"])


def test_inout_bitexact_and_capacity():
    P = lib()
    s = W.inout_strip(nx=30, ny=12, n_in=5, n_out=5, jitter=0.3, seed=25)
    rng = np.random.default_rng(26)
    s["x"] = s["x"] + rng.uniform(0.0, 0.6 * s["dx"] * 3, s["x"].size)
    s["p"] = rng.standard_normal(s["x"].size)
    s["params"] = dict(PRM)
    n = s["x"].size
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=2 * n)
    # capacity two-phase: a set whose capacity cannot take the copies
    ps_small = particles(P, s, capacity=n)
    before = ps_small.numpy()
    oo, oorig, ocnt = oracle.inout(s["io"], s, cap=2 * n)
    if ocnt["appended"] > ocnt["deleted"]:
        info = ctx.inout(ps_small, s["io"])
        assert info.get("error") == P.SPH_E_CAPACITY
        assert info["n_required"] == n + ocnt["appended"] - ocnt["deleted"]
        after = ps_small.numpy()
        for k in before:
            assert np.array_equal(before[k], after[k]), k
    ps = particles(P, s, capacity=2 * n)
    info = ctx.inout(ps, s["io"])
    assert "error" not in info
    g = ps.numpy()
    assert np.array_equal(info["origin"].cpu().numpy(), oorig)
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mref", "mq", "kind"):
        assert np.array_equal(g[k], oo[k]), k
    assert info["appended"] == ocnt["appended"] and info["deleted"] == ocnt["deleted"]
    assert info["to_outlet"] == ocnt["to_outlet"]


def test_couette_startup_fp32():
    P = lib()
    s = W.wall_box(nx=10, ny=10, layers=4, jitter=0.0, hdx=1.2)
    U, nu = 1.0, 0.5
    s["u"] = np.where((s["kind"] == W.SOLID) & (s["y"] > 0.5), U, 0.0)
    s["params"] = {"rho0": 1.0, "cs": 10.0, "nu": nu, "hdx": 1.2}
    dt = oracle.timestep(1.2 * s["dx"], U, 10.0, nu)
    ctx = ctx_for(P, s, P.SPH_FP32)
    ps = particles(P, s)
    ctx.step(ps, dt, 100)
    g = ps.numpy()
    fl = g["kind"] == W.FLUID
    T = 100 * dt
    y = g["y"][fl]
    ref = U * y / s["H"]
    for k in range(1, 400):
        ref = ref + 2 * U / (k * np.pi) * (-1) ** k * np.sin(k * np.pi * y / s["H"]) * np.exp(
            -k * k * np.pi ** 2 * nu * T / s["H"] ** 2)
    err = np.abs(g["u"][fl] - ref).max()
    print(f"[couette] fp32 max error vs series {err:.2e}", flush=True)
    assert err < 0.01


@pytest.mark.parametrize("skin", [0.02, 0.1, 0.3])
def test_step_inout_equals_separate_calls(skin):
    """sph_step_inout: the same state as sph_step + sph_inout called step by
    step (bit for bit), with the counters summed and the origin maps
    composed, over enough steps for inlet particles to enter the fluid.
    sph_step_inout enqueues its steps as guarded runs; the skins make the
    list expire at predicted and corrected positions at different steps, and
    the inlet crossings move slots, so every way a run stops is taken."""
    P = lib()
    s = _io_case()
    s["u"] = np.where(s["kind"] == W.INLET, 1.0, s["u"])
    dt = 2e-3
    nsteps = 40
    n = s["x"].size
    cap = 2 * n
    print(f"[step_inout] skin={skin}", flush=True)
    ctx_a = ctx_for(P, s, P.SPH_FP64, capacity=cap, list_skin=skin)
    A = particles(P, s, capacity=cap)
    comp = np.arange(n)
    tot = {"appended": 0, "deleted": 0, "to_outlet": 0}
    for _ in range(nsteps):
        ctx_a.step(A, dt, 1)
        info = ctx_a.inout(A, s["io"])
        for k in tot:
            tot[k] += info[k]
        comp = comp[info["origin"].cpu().numpy()]
    ctx_b = ctx_for(P, s, P.SPH_FP64, capacity=cap, list_skin=skin)
    B = particles(P, s, capacity=cap)
    ib = ctx_b.step_inout(B, dt, nsteps, s["io"])
    print(f"[step_inout] n {A.n} {B.n} counts {tot} {ib}", flush=True)
    assert tot["appended"] > 0
    assert A.n == B.n
    for k in tot:
        assert ib[k] == tot[k], k
    assert np.array_equal(ib["origin"].cpu().numpy(), comp)
    ga, gb = A.numpy(), B.numpy()
    for k in ("x", "y", "u", "v", "p", "rho", "h", "mq", "kind"):
        assert np.array_equal(ga[k], gb[k]), k


@pytest.mark.parametrize("rule", [0, 1])
def test_pulse_reflection_fp32(rule):
    """An acoustic pulse (p' = -rho0 c u', running upstream) in a flowing
    strip, U = 1, c = 10, on the FP32 path: with the characteristic
    inlet/outlet it leaves the channel (under 3% of its energy stays);
    with the inlet velocity held (rule 0) more than a third reflects."""
    P = lib()
    nx, ny = 80, 16
    s = W.inout_strip(nx=nx, ny=ny, n_in=6, n_out=6, U=1.0)
    L = nx * s["dx"]
    fl = s["kind"] == W.FLUID
    pp = 0.5 * np.exp(-((s["x"] - 0.5 * L) / (0.08 * L)) ** 2) * fl
    s["p"] = pp.copy()
    s["u"] = 1.0 - pp / 10.0
    s["params"] = {"rho0": 1.0, "cs": 10.0, "nu": 0.002, "hdx": 1.2}
    kw = {"io_mode": 1, "io_ref": (1.0, 0.0, 0.0)} if rule == 1 else {}
    ctx = ctx_for(P, s, P.SPH_FP32, **kw)
    ps = particles(P, s)
    dt = 0.25 * s["h"][0] / 11.0
    nsteps = int(0.35 / dt)
    print(f"[pulse] rule={rule} n={s['x'].size} steps={nsteps}", flush=True)
    ctx.step(ps, dt, nsteps)
    g = ps.numpy()
    mid = (g["kind"] == W.FLUID) & (g["x"] > 0.1 * L) & (g["x"] < 0.9 * L)
    ratio = float(np.sum(g["p"][mid] ** 2)) / float(np.sum(pp ** 2))
    print(f"[pulse] rule={rule} energy left {ratio:.4f}", flush=True)
    if rule == 1:
        assert ratio < 0.03
    else:
        assert ratio > 0.3
