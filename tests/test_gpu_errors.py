"""Argument checks of the C ABI: invalid configurations are refused at
creation, and calls with missing arrays, non-finite values or sizes beyond
the capacity return SPH_E_INVAL (or SPH_E_CAPACITY) without touching the
state.  Every case here is refused on the host before any kernel runs."""
import ctypes as C
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import ctx_for, lib, particles

pytestmark = pytest.mark.gpu


def test_config_rejections():
    P = lib()
    base = dict(lo=(0.0, 0.0), hi=(1.0, 1.0), periodic=(1, 1), h_lo=0.01, h_hi=0.02)
    bad = ({"io_mode": 2}, {"io_ref": (math.nan, 0.0, 0.0)}, {"io_mode": 1, "cs": 0.0},
           {"hi": (0.0, 1.0)}, {"h_lo": 0.0}, {"list_skin": 1.5}, {"precision": 7},
           {"wall_accel": (math.inf, 0.0)}, {"merge_iters": 9}, {"lean": 2}, {"n_adapt": -1},
           {"n_bg": -2}, {"dt": -1e-4}, {"sol_k": math.nan}, {"bg_passes": -1},
           {"csr_k": -1}, {"csr_k": 70000})
    for b in bad:
        with pytest.raises(P.SphError) as e:
            P.Context(P.Config(**{**base, **b}), 16)
        assert e.value.code == P.SPH_E_INVAL, b
    P.Context(P.Config(**base, io_mode=1, io_ref=(1.0, 0.0, 0.0)), 16)  # a valid one


def test_call_rejections_leave_state():
    P = lib()
    s = W.wall_box(nx=8, ny=8, layers=2, jitter=0.1)
    s["u"] = np.zeros(s["x"].size)
    s["v"] = np.zeros(s["x"].size)
    s["p"] = np.zeros(s["x"].size)
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    before = ps.numpy()
    D2 = C.c_double * 2
    # non-finite body motion
    with pytest.raises(P.SphError) as e:
        ctx.move_solids(ps, (math.nan, 0.0), (0.0, 0.0))
    assert e.value.code == P.SPH_E_INVAL
    # no kind array: moving the solids and the body force need it
    c = ps.c()
    c.kind = None
    assert ctx.lib.sph_move_solids(ctx._h, C.byref(c), D2(0.1, 0.0), D2(0.0, 0.0),
                                   D2(0.0, 0.0)) == P.SPH_E_INVAL
    f = (C.c_double * 8)()
    assert ctx.lib.sph_body_force(ctx._h, C.byref(c), f) == P.SPH_E_INVAL
    # n beyond the capacity, and a step with dt <= 0
    c = ps.c()
    c.n = c.capacity + 1
    assert ctx.lib.sph_pec(ctx._h, C.byref(c), 1e-4, 1) == P.SPH_E_INVAL
    assert ctx.lib.sph_step(ctx._h, C.byref(c), None, None, None, 1, None) == P.SPH_E_INVAL
    with pytest.raises(P.SphError) as e:
        ctx.step(ps, 0.0, 1)
    assert e.value.code == P.SPH_E_INVAL
    # the schedule: a background update every n_bg iterations needs the solids
    c2 = P.Context(dataclasses.replace(ctx.cfg, n_bg=5), ps.capacity)
    bgd = W.background_lattice(s["domain"], 0.25, 1.2, 1.0)
    assert bgd["x"].size <= ps.capacity
    B = P.Background.from_arrays(bgd, ps.capacity)
    with pytest.raises(P.SphError) as e:
        c2.run(ps, 1, bg=B)
    assert e.value.code == P.SPH_E_INVAL
    after = ps.numpy()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    # a valid call still works and moves the solids only
    ctx.move_solids(ps, (0.125, 0.0), (0.5, 0.0))
    g = ps.numpy()
    sol = g["kind"] == W.SOLID
    assert np.all(g["u"][sol] == 0.5) and np.array_equal(g["y"], before["y"])
    assert np.array_equal(g["x"][~sol], before["x"][~sol])


def test_nonfinite_state_reported():
    """A NaN or infinite value anywhere in the state (set from the host; no
    step runs on it) makes the diagnostics return SPH_E_NONFINITE, with the
    sums still written; a finite state passes."""
    P = lib()
    s = W.wall_box(nx=8, ny=8, layers=2, jitter=0.1)
    n = s["x"].size
    s["u"] = np.zeros(n)
    s["v"] = np.zeros(n)
    s["p"] = np.zeros(n)
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    d = ctx.diagnostics(ps)
    assert d["n"] == n and math.isfinite(d["ke"])
    for field, val in (("p", math.nan), ("u", math.inf), ("rho", math.nan), ("h", -math.inf)):
        q = particles(P, dict(s, **{field: np.where(np.arange(n) == 5, val, s.get(field, np.ones(n)))}))
        with pytest.raises(P.SphError) as e:
            ctx.diagnostics(q)
        assert e.value.code == P.SPH_E_NONFINITE, field


def test_ledger_overflow_reported():
    """The diagnostics sum the mass ledger in checked int64: quanta whose
    total does not fit are reported (SPH_E_INVAL) instead of wrapping; a
    total just below 2^63 is summed exactly.  Only the reduction runs."""
    P = lib()
    s = W.tgv(8, seed=2)
    n = s["x"].size
    ctx = ctx_for(P, s, P.SPH_FP64)
    ps = particles(P, s)
    big = (2 ** 63 - 1) // n
    ps.mq[:n] = big
    d = ctx.diagnostics(ps)
    assert d["mq_total"] == big * n
    ps.mq[:n] = 2 ** 62
    with pytest.raises(P.SphError) as e:
        ctx.diagnostics(ps)
    assert e.value.code == P.SPH_E_INVAL and "ledger" in str(e.value)


def test_background_update_rejections():
    """A background update refuses solids beyond the context capacity or
    without positions, before any kernel runs."""
    P = lib()
    bg = W.background_lattice(W.Domain((0.0, 0.0), (1.0, 1.0), (True, True)), 0.1, 1.2, 1.0)
    cfg = P.Config(lo=(0.0, 0.0), hi=(1.0, 1.0), periodic=(1, 1), h_lo=0.01, h_hi=0.2, cr=1.2,
                   ds_min=0.05, ds_max=0.1, bg_mass_q=bg["mass_q"])
    ctx = P.Context(cfg, 200)
    B = P.Background.from_arrays(bg, 200)
    big = P.Particles.from_arrays({"x": np.full(300, 0.5), "y": np.full(300, 0.5),
                                   "h": np.full(300, 0.05), "mq": np.ones(300, np.int64)})
    with pytest.raises(P.SphError) as e:
        ctx.bg_update(B, big, 1)
    assert e.value.code == P.SPH_E_INVAL and "solids" in str(e.value)
    s = big.c()
    s.n, s.x = 10, None
    ns = C.c_int64(0)
    assert ctx.lib.sph_bg_update(ctx._h, C.byref(B.c()), C.byref(s), None, 0.0, 1,
                                 C.byref(ns)) == P.SPH_E_INVAL
    assert B.n == bg["x"].size


def test_internal_list_width_reported():
    """The adaptation's internal neighbour lists hold csr_k entries per
    particle of capacity: with room for 4, a shift's list does not fit and
    the call returns SPH_E_NOMEM naming the csr_k that does; the default
    width adapts the same state."""
    P = lib()
    s = W.tgv(20, seed=3)
    n = s["x"].size
    s["mref"] = np.full(n, float(s["mq"][0]) * s["mass_q"])
    print(f"[errors] csr_k n={n}", flush=True)
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=2 * n, csr_k=4)
    ps = particles(P, s, capacity=2 * n)
    with pytest.raises(P.SphError) as e:
        ctx.adapt(ps)
    assert e.value.code == P.SPH_E_NOMEM and "csr_k >=" in str(e.value)
    k = int(str(e.value).split("csr_k >= ")[1].split()[0])
    assert 5 <= k <= 200
    ctx = ctx_for(P, s, P.SPH_FP64, capacity=2 * n, csr_k=k)
    ps = particles(P, s, capacity=2 * n)
    ctx.adapt(ps)
    assert ps.n == n
