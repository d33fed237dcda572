"""Plain FP64 CPU oracle for the adaptive-resolution WCSPH hot path.

TEST INFRASTRUCTURE ONLY.  This package wraps ``sph_oracle.c`` (built into
``liboracle_sph.so`` by :func:`build`) with ctypes and numpy.  It is the
definition the HIP library is checked against and shares no code with it.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does.

Every function mirrors one passage of Muta & Ramachandran (arXiv 2107.01276);
the C source names the equation or section each one follows.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sph.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FMA contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Domain(C.Structure):
    _fields_ = [("lo", C.c_double * 2), ("hi", C.c_double * 2), ("periodic", C.c_int32 * 2)]


class Params(C.Structure):
    _fields_ = [("rho0", C.c_double), ("cs", C.c_double), ("nu", C.c_double),
                ("alpha_e", C.c_double), ("hdx", C.c_double), ("fx", C.c_double),
                ("fy", C.c_double), ("split_alpha", C.c_double), ("split_eps", C.c_double),
                ("mmax_f", C.c_double), ("mmin_f", C.c_double), ("mass_q", C.c_double),
                ("merge_iters", C.c_int32), ("shift_iters", C.c_int32), ("pref_mode", C.c_int32)]


class Bc(C.Structure):
    _fields_ = [("awx", C.c_double), ("awy", C.c_double), ("io_mode", C.c_int32),
                ("ur", C.c_double), ("vr", C.c_double), ("pr", C.c_double)]


def _bc(aw, io):
    """Wall acceleration and the inlet/outlet rule: io = None (zero-gradient)
    or (u_r, v_r, p_r), the reference state of the characteristic rule."""
    if io is None:
        return Bc(float(aw[0]), float(aw[1]), 0, 0.0, 0.0, 0.0)
    return Bc(float(aw[0]), float(aw[1]), 1, float(io[0]), float(io[1]), float(io[2]))


class Io(C.Structure):
    _fields_ = [("x_in", C.c_double), ("len_in", C.c_double), ("x_out", C.c_double),
                ("len_out", C.c_double)]


class BgParams(C.Structure):
    _fields_ = [("rho0", C.c_double), ("cr", C.c_double), ("ds_min", C.c_double),
                ("ds_max", C.c_double), ("n_r", C.c_double), ("split_alpha", C.c_double),
                ("split_eps", C.c_double), ("mmax_f", C.c_double), ("mass_q", C.c_double),
                ("smooth_iters", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        D, I64, I32, P = C.c_double, C.c_int64, C.c_int32, C.c_void_p
        sig = {
            "or_kf": (D, [D]), "or_kfp": (D, [D]), "or_w": (D, [D, D]), "or_dwdr": (D, [D, D]),
            "or_nbr_brute": (I64, [P, I64, P, P, P, P, P, I64]),
            "or_nbr_cells": (I64, [P, I64, P, P, P, P, P, I64]),
            "or_xnbr_brute": (I64, [P, I64, P, P, P, I64, P, P, P, P, P, I64]),
            "or_xnbr_cells_alloc": (I64, [P, I64, P, P, P, I64, P, P, P, P, P]),
            "or_free": (None, [P]),
            "or_pass_a": (None, [P, P, I64] + [P] * 13),
            "or_pass_b": (None, [P, P, I64] + [P] * 12 + [D] + [P] * 7),
            "or_boundary": (None, [P, P, P, I64] + [P] * 12),
            "or_rates_k": (C.c_int, [P, P, P, I64] + [P] * 9 + [D] + [P] * 9),
            "or_rates_k_scaled": (C.c_int, [P, P, P, I64] + [P] * 9 + [D] + [P] * 10),
            "or_rate_scales": (None, [P, P, I64] + [P] * 12 + [D] + [P] * 7),
            "or_body_force": (C.c_int, [P, P, P, I64] + [P] * 10),
            "or_move_solids": (None, [P, I64, P, D, D, D, D, P, P, P, P]),
            "or_step_k": (C.c_int, [P, P, P, I64] + [P] * 9 + [D, I64]),
            "or_inout": (I64, [P, I64, I64] + [P] * 12),
            "or_rates": (C.c_int, [P, P, I64] + [P] * 7 + [D] + [P] * 9),
            "or_step": (C.c_int, [P, P, I64] + [P] * 7 + [D, I64, P]),
            "or_adapt": (I64, [P, P, I64, I64] + [P] * 13),
            "or_split_only": (I64, [P, P, I64, I64] + [P] * 12),
            "or_merge_only": (I64, [P, P, I64] + [P] * 13),
            "or_shift_only": (C.c_int, [P, P, I64] + [P] * 10),
            "or_hupdate_only": (C.c_int, [P, P, I64] + [P] * 6),
            "or_mref_lookup": (C.c_int, [P, I64, P, P, P, I64, P, P, P, P, P]),
            "or_bg_update": (I64, [P, P, I64, I64] + [P] * 7 + [I64, P, P, P, P, D, I32, P]),
            "or_vorticity": (None, [P, I64] + [P] * 10),
            "or_shepard_to_bg": (C.c_int, [P, I64, P, P, P, I64, P, P, P, P, P, P]),
            "or_timestep": (D, [D, D, D, D]),
            "or_exact_sum": (D, [I64, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class Dom:
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    periodic: tuple = (True, True)

    def c(self):
        d = Domain()
        d.lo[0], d.lo[1] = self.lo
        d.hi[0], d.hi[1] = self.hi
        d.periodic[0], d.periodic[1] = int(self.periodic[0]), int(self.periodic[1])
        return d


@dataclass
class Prm:
    rho0: float = 1.0
    cs: float = 10.0
    nu: float = 0.01
    alpha_e: float = 1.5
    hdx: float = 1.0
    fx: float = 0.0
    fy: float = 0.0
    split_alpha: float = 0.9
    split_eps: float = 0.4
    mmax_f: float = 1.05
    mmin_f: float = 0.5
    mass_q: float = 2.0 ** -60
    merge_iters: int = 3
    shift_iters: int = 3
    pref_mode: int = 1

    def c(self):
        p = Params()
        for k in Params._fields_:
            setattr(p, k[0], getattr(self, k[0]))
        return p


@dataclass
class BgPrm:
    rho0: float = 1.0
    cr: float = 1.2
    ds_min: float = 0.1
    ds_max: float = 0.4
    n_r: float = 48.0
    split_alpha: float = 0.9
    split_eps: float = 0.4
    mmax_f: float = 1.05
    mass_q: float = 2.0 ** -60
    smooth_iters: int = 3

    def c(self):
        p = BgParams()
        for k in BgParams._fields_:
            setattr(p, k[0], getattr(self, k[0]))
        return p


# --------------------------------------------------------------------------
# kernel
# --------------------------------------------------------------------------

def kf(q):
    return lib().or_kf(float(q))


def kfp(q):
    return lib().or_kfp(float(q))


def w(r, h):
    return lib().or_w(float(r), float(h))


def dwdr(r, h):
    return lib().or_dwdr(float(r), float(h))


# --------------------------------------------------------------------------
# neighbours
# --------------------------------------------------------------------------

def neighbors(dom: Dom, x, y, h, method: str = "cells"):
    """CSR (row_ptr int64[n+1], col int32[nnz]); rows ascending, self included."""
    x, y, h = _f64(x), _f64(y), _f64(h)
    n = x.size
    rp = np.zeros(n + 1, np.int64)
    fn = lib().or_nbr_brute if method == "brute" else lib().or_nbr_cells
    d = dom.c()
    cap = max(64 * n, 1)
    while True:
        col = np.zeros(cap, np.int32)
        nnz = fn(C.byref(d), n, _p(x), _p(y), _p(h), _p(rp), _p(col), cap)
        if nnz < 0:
            raise RuntimeError(f"oracle neighbour build failed: {nnz}")
        if nnz <= cap:
            return rp, col[:nnz].copy()
        cap = int(nnz)


def cross_neighbors(dom: Dom, xa, ya, ha, xb, yb, hb, method: str = "cells"):
    xa, ya, ha, xb, yb, hb = map(_f64, (xa, ya, ha, xb, yb, hb))
    na, nb = xa.size, xb.size
    d = dom.c()
    if method == "brute":
        rp = np.zeros(na + 1, np.int64)
        cap = max(64 * na, 1)
        while True:
            col = np.zeros(cap, np.int32)
            nnz = lib().or_xnbr_brute(C.byref(d), na, _p(xa), _p(ya), _p(ha), nb, _p(xb),
                                      _p(yb), _p(hb), _p(rp), _p(col), cap)
            if nnz <= cap:
                return rp, col[:nnz].copy()
            cap = int(nnz)
    prp, pcol = C.c_void_p(), C.c_void_p()
    nnz = lib().or_xnbr_cells_alloc(C.byref(d), na, _p(xa), _p(ya), _p(ha), nb, _p(xb), _p(yb),
                                    _p(hb), C.byref(prp), C.byref(pcol))
    if nnz < 0:
        raise RuntimeError("oracle cross neighbour build failed")
    rp = np.ctypeslib.as_array(C.cast(prp, C.POINTER(C.c_int64)), shape=(na + 1,)).copy()
    col = np.ctypeslib.as_array(C.cast(pcol, C.POINTER(C.c_int32)), shape=(max(nnz, 1),))[:nnz].copy()
    lib().or_free(prp)
    lib().or_free(pcol)
    return rp, col


# --------------------------------------------------------------------------
# rates
# --------------------------------------------------------------------------

def pass_a(dom: Dom, prm: Prm, x, y, h, m, p, rp, col):
    x, y, h, m, p = map(_f64, (x, y, h, m, p))
    rp, col = _i64(rp), _i32(col)
    n = x.size
    out = {k: np.zeros(n) for k in ("rho", "beta", "nnb", "pavg", "dxs", "dys")}
    lib().or_pass_a(C.byref(dom.c()), C.byref(prm.c()), n, _p(x), _p(y), _p(h), _p(m), _p(p),
                    _p(rp), _p(col), *[_p(out[k]) for k in ("rho", "beta", "nnb", "pavg", "dxs", "dys")])
    return out


def pass_b(dom: Dom, prm: Prm, x, y, u, v, p, h, m, a, dt, rp, col, ug=None, vg=None):
    x, y, u, v, p, h, m = map(_f64, (x, y, u, v, p, h, m))
    ug = None if ug is None else _f64(ug)
    vg = None if vg is None else _f64(vg)
    rp, col = _i64(rp), _i32(col)
    n = x.size
    out = {k: np.zeros(n) for k in ("dpdt", "dudt", "dvdt")}
    lib().or_pass_b(C.byref(dom.c()), C.byref(prm.c()), n, _p(x), _p(y), _p(u), _p(v), _p(p),
                    _p(h), _p(m), _p(_f64(a["rho"])), _p(_f64(a["beta"])), _p(_f64(a["pavg"])),
                    _p(_f64(a["dxs"])), _p(_f64(a["dys"])), float(dt), _p(rp), _p(col),
                    _p(ug), _p(vg), _p(out["dpdt"]), _p(out["dudt"]), _p(out["dvdt"]))
    return out


RATE_FIELDS = ("rho", "beta", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")


def rate_scales(dom: Dom, prm: Prm, x, y, u, v, p, h, m, a, dt, rp, col, ug=None, vg=None):
    """Per-particle scales of the rates (or_rate_scales): for every field the
    sum of the magnitudes of its pair terms.  a: pass A outputs.  Returns
    {field: array}."""
    x, y, u, v, p, h, m = map(_f64, (x, y, u, v, p, h, m))
    ug = None if ug is None else _f64(ug)
    vg = None if vg is None else _f64(vg)
    rp, col = _i64(rp), _i32(col)
    n = x.size
    sc = np.zeros(8 * max(n, 1))
    lib().or_rate_scales(C.byref(dom.c()), C.byref(prm.c()), n, _p(x), _p(y), _p(u), _p(v),
                         _p(p), _p(h), _p(m), _p(_f64(a["rho"])), _p(_f64(a["beta"])),
                         _p(_f64(a["pavg"])), _p(_f64(a["dxs"])), _p(_f64(a["dys"])), float(dt),
                         _p(rp), _p(col), _p(ug), _p(vg), None, None, _p(sc))
    return {k: sc[f * n:(f + 1) * n].copy() for f, k in enumerate(RATE_FIELDS)}


def cond_error(a, b, scale):
    """max_i |a_i - b_i| / scale_i (0 where a_i == b_i): the error of a
    against the oracle's b relative to the size of the terms b_i sums."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.abs(a - b)
    if d.size == 0:
        return 0.0
    sc = np.asarray(scale, np.float64)
    r = np.where(d == 0, 0.0, d / np.where(sc > 0, sc, np.inf))
    r = np.where((d > 0) & ~(sc > 0), np.inf, r)
    return float(r.max())


FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3


def boundary(dom: Dom, prm: Prm, x, y, h, rho, kind, u, v, p, rp, col, aw=(0.0, 0.0), io=None):
    """Boundary pass of section 2.2 on copies of u, v, p.
    Returns (u, v, p, ug, vg)."""
    x, y, h, rho = map(_f64, (x, y, h, rho))
    u, v, p = (_f64(a).copy() for a in (u, v, p))
    kind, rp, col = _i32(kind), _i64(rp), _i32(col)
    n = x.size
    ug, vg = np.zeros(n), np.zeros(n)
    bc = _bc(aw, io)
    lib().or_boundary(C.byref(dom.c()), C.byref(prm.c()), C.byref(bc), n, _p(x), _p(y), _p(h),
                      _p(rho), _p(kind), _p(rp), _p(col), _p(u), _p(v), _p(p), _p(ug), _p(vg))
    return u, v, p, ug, vg


def rates_k(dom: Dom, prm: Prm, state: dict, dt: float, aw=(0.0, 0.0), io=None, scales=True):
    """One evaluation with boundary particles (state needs 'kind' and 'rho',
    the stored density).  Returns the fields plus the state's u, v, p after
    the boundary pass, and the per-particle scales (rate_scales) unless
    scales is False."""
    st = {k: _f64(state[k]).copy() for k in ("x", "y", "u", "v", "p", "h", "m", "rho")}
    kind = _i32(state["kind"])
    n = st["x"].size
    out = {k: np.zeros(n) for k in ("rho", "beta", "nnb", "pavg", "dxs", "dys", "dpdt", "dudt", "dvdt")}
    sc = np.zeros(8 * max(n, 1))
    bc = _bc(aw, io)
    rc = lib().or_rates_k_scaled(C.byref(dom.c()), C.byref(prm.c()), C.byref(bc), n,
                                 *[_p(st[k]) for k in ("x", "y", "u", "v", "p", "h", "m")],
                                 _p(kind), _p(st["rho"]), float(dt),
                                 *[_p(out[k]) for k in ("rho", "beta", "nnb", "pavg", "dxs",
                                                        "dys", "dpdt", "dudt", "dvdt")],
                                 _p(sc) if scales else None)
    if rc != 0:
        raise RuntimeError(f"oracle rates failed: {rc}")
    out["u_bc"], out["v_bc"], out["p_bc"] = st["u"], st["v"], st["p"]
    if scales:
        out["scale"] = {k: sc[f * n:(f + 1) * n].copy() for f, k in enumerate(RATE_FIELDS)}
    return out


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's row loops."""
    C.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def body_force(dom: Dom, prm: Prm, state: dict, aw=(0.0, 0.0), io=None):
    """Force on the solid particles, eq. (force-sph) of section 2.3, from one
    evaluation's state (boundary pass and pass A on copies).  Returns
    {"fp": (x, y), "fvisc": (x, y), "abs_p": (x, y), "abs_visc": (x, y)}: the
    pressure and viscous totals and the sums of their terms' magnitudes."""
    st = {k: _f64(state[k]).copy() for k in ("x", "y", "u", "v", "p", "h", "m", "rho")}
    kind = _i32(state["kind"])
    n = st["x"].size
    out = np.zeros(8)
    bc = _bc(aw, io)
    rc = lib().or_body_force(C.byref(dom.c()), C.byref(prm.c()), C.byref(bc), n,
                             *[_p(st[k]) for k in ("x", "y", "u", "v", "p", "h", "m")], _p(kind),
                             _p(st["rho"]), _p(out))
    if rc != 0:
        raise RuntimeError(f"oracle body force failed: {rc}")
    return {"fp": (out[0], out[1]), "fvisc": (out[2], out[3]), "abs_p": (out[4], out[5]),
            "abs_visc": (out[6], out[7])}


def force_coefficients(f: dict, rho0: float, U: float, L: float):
    """c_d (pressure), c_d (skin friction) and c_l (pressure), eq. (cdcl)."""
    q = 0.5 * rho0 * U * U * L
    return {"cd_p": f["fp"][0] / q, "cd_visc": f["fvisc"][0] / q, "cl": f["fp"][1] / q}


def step_k(dom: Dom, prm: Prm, state: dict, dt: float, nsteps: int, aw=(0.0, 0.0), io=None):
    """PEC steps with boundary particles on copies; state needs 'kind' and
    'rho' (stored density, updated to the latest summation)."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "u", "v", "p", "h", "m", "rho")}
    kind = _i32(state["kind"])
    n = s["x"].size
    bc = _bc(aw, io)
    rc = lib().or_step_k(C.byref(dom.c()), C.byref(prm.c()), C.byref(bc), n,
                         *[_p(s[k]) for k in ("x", "y", "u", "v", "p", "h", "m")], _p(kind),
                         _p(s["rho"]), float(dt), int(nsteps))
    if rc != 0:
        raise RuntimeError(f"oracle step failed: {rc}")
    s["kind"] = kind
    return s


def move_solids(dom: Dom, state: dict, disp, vel):
    """Rigid motion of the solid particles (kind 1) on a copy of the state:
    translated by disp (wrapped on periodic axes), velocity set to vel."""
    s = dict(state)
    for k in ("x", "y", "u", "v"):
        s[k] = _f64(state[k]).copy()
    kind = _i32(state["kind"])
    lib().or_move_solids(C.byref(dom.c()), kind.size, _p(kind), float(disp[0]), float(disp[1]),
                         float(vel[0]), float(vel[1]), _p(s["x"]), _p(s["y"]), _p(s["u"]),
                         _p(s["v"]))
    return s


_IO_F = ("x", "y", "u", "v", "p", "rho", "h", "mref")


def inout(io: dict, state: dict, cap: int):
    """Inlet/outlet update of section 2.2 on copies.  Returns (state, origin,
    counts) or raises on capacity."""
    n = state["x"].size
    st = {}
    for k in _IO_F:
        a = np.zeros(max(cap, 1))
        a[:n] = state[k]
        st[k] = a
    mq = np.zeros(max(cap, 1), np.int64); mq[:n] = state["mq"]
    kind = np.zeros(max(cap, 1), np.int32); kind[:n] = state["kind"]
    origin = np.zeros(max(cap, 1), np.int64)
    counts = np.zeros(4, np.int64)
    cio = Io(float(io["x_in"]), float(io["len_in"]), float(io["x_out"]), float(io["len_out"]))
    nn = lib().or_inout(C.byref(cio), n, cap, *[_p(st[k]) for k in _IO_F], _p(mq), _p(kind),
                        _p(origin), _p(counts))
    if nn < 0:
        raise RuntimeError(f"oracle inout failed: {nn}")
    out = {k: st[k][:nn].copy() for k in _IO_F}
    out["mq"], out["kind"] = mq[:nn].copy(), kind[:nn].copy()
    return out, origin[:nn].copy(), {"appended": int(counts[0]), "deleted": int(counts[1]),
                                     "to_fluid": int(counts[2]), "to_outlet": int(counts[3])}


def rates(dom: Dom, prm: Prm, x, y, u, v, p, h, m, dt, method: str = "cells"):
    """One evaluation: neighbours, pass A, pass B.  Returns a dict of fields."""
    rp, col = neighbors(dom, x, y, h, method)
    a = pass_a(dom, prm, x, y, h, m, p, rp, col)
    b = pass_b(dom, prm, x, y, u, v, p, h, m, a, dt, rp, col)
    a["scale"] = rate_scales(dom, prm, x, y, u, v, p, h, m, a, dt, rp, col)
    a.update(b)
    a["row_ptr"], a["col"] = rp, col
    return a


def step(dom: Dom, prm: Prm, state: dict, dt: float, nsteps: int):
    """PEC steps in place on copies; returns the new state dict (+ 'rho')."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "u", "v", "p", "h", "m")}
    n = s["x"].size
    rho = np.zeros(n)
    rc = lib().or_step(C.byref(dom.c()), C.byref(prm.c()), n, _p(s["x"]), _p(s["y"]), _p(s["u"]),
                       _p(s["v"]), _p(s["p"]), _p(s["h"]), _p(s["m"]), float(dt), int(nsteps), _p(rho))
    if rc != 0:
        raise RuntimeError(f"oracle step failed: {rc}")
    s["rho"] = rho
    return s


# --------------------------------------------------------------------------
# adaptation
# --------------------------------------------------------------------------

_ADAPT_F = ("x", "y", "u", "v", "p", "rho", "h", "mref")


def _adapt_arrays(state, cap):
    n = state["x"].size
    arrs = {}
    for k in _ADAPT_F:
        a = np.zeros(cap)
        a[:n] = state[k]
        arrs[k] = a
    mq = np.zeros(cap, np.int64)
    mq[:n] = state["mq"]
    kind = np.zeros(cap, np.int32)
    if "kind" in state:
        kind[:n] = state["kind"]
    arrs["mq"], arrs["kind"] = mq, kind
    arrs["origin"] = np.zeros(cap, np.int64)
    arrs["sat"] = np.zeros(cap, np.int32)
    return arrs


def adapt(dom: Dom, prm: Prm, state: dict, cap: int | None = None):
    """Split, merge x merge_iters, shift x shift_iters, h update (section 3.4).

    ``state`` holds x y u v p rho h mref (float64), mq (int64 mass quanta) and
    optionally kind (int32).  Returns (new_state, info) where info has
    origin, sat, n_split, n_required, merged (list per iteration).
    """
    n = state["x"].size
    if cap is None:
        cap = 7 * n + 8
    A = _adapt_arrays(state, cap)
    counts = np.zeros(2 + max(prm.merge_iters, 1), np.int64)
    nn = lib().or_adapt(C.byref(dom.c()), C.byref(prm.c()), n, cap,
                        *[_p(A[k]) for k in _ADAPT_F], _p(A["mq"]), _p(A["kind"]),
                        _p(A["origin"]), _p(A["sat"]), _p(counts))
    info = {"n_split": int(counts[0]), "n_required": int(counts[1]),
            "merged": [int(c) for c in counts[2:2 + prm.merge_iters]]}
    if nn < 0:
        info["error"] = int(nn)
        return None, info
    out = {k: A[k][:nn].copy() for k in list(_ADAPT_F) + ["mq", "kind"]}
    info["origin"] = A["origin"][:nn].copy()
    info["sat"] = A["sat"][:nn].copy()
    return out, info


def split_only(dom: Dom, prm: Prm, state: dict):
    n = state["x"].size
    cap = 7 * n + 8
    A = _adapt_arrays(state, cap)
    nn = lib().or_split_only(C.byref(dom.c()), C.byref(prm.c()), n, cap,
                             *[_p(A[k]) for k in _ADAPT_F], _p(A["mq"]), _p(A["kind"]),
                             _p(A["origin"]), _p(A["sat"]))
    out = {k: A[k][:nn].copy() for k in list(_ADAPT_F) + ["mq", "kind"]}
    return out, {"origin": A["origin"][:nn].copy(), "sat": A["sat"][:nn].copy()}


def merge_only(dom: Dom, prm: Prm, state: dict):
    n = state["x"].size
    A = _adapt_arrays(state, max(n, 1))
    npairs = C.c_int64(0)
    nn = lib().or_merge_only(C.byref(dom.c()), C.byref(prm.c()), n,
                             *[_p(A[k]) for k in _ADAPT_F], _p(A["mq"]), _p(A["kind"]),
                             _p(A["origin"]), _p(A["sat"]), C.byref(npairs))
    out = {k: A[k][:nn].copy() for k in list(_ADAPT_F) + ["mq", "kind"]}
    return out, {"origin": A["origin"][:nn].copy(), "pairs": int(npairs.value)}


def shift_only(dom: Dom, prm: Prm, state: dict):
    n = state["x"].size
    A = _adapt_arrays(state, max(n, 1))
    rc = lib().or_shift_only(C.byref(dom.c()), C.byref(prm.c()), n,
                             *[_p(A[k]) for k in _ADAPT_F], _p(A["mq"]), _p(A["kind"]))
    assert rc == 0
    return {k: A[k][:n].copy() for k in list(_ADAPT_F) + ["mq", "kind"]}


def hupdate_only(dom: Dom, prm: Prm, state: dict):
    n = state["x"].size
    A = _adapt_arrays(state, max(n, 1))
    rc = lib().or_hupdate_only(C.byref(dom.c()), C.byref(prm.c()), n, _p(A["x"]), _p(A["y"]),
                               _p(A["rho"]), _p(A["h"]), _p(A["mq"]), _p(A["kind"]))
    assert rc == 0
    return A["h"][:n].copy()


def mref_lookup(dom: Dom, x, y, h, bx, by, bh, bmref):
    x, y, h, bx, by, bh, bmref = map(_f64, (x, y, h, bx, by, bh, bmref))
    out = np.zeros(x.size)
    rc = lib().or_mref_lookup(C.byref(dom.c()), x.size, _p(x), _p(y), _p(h), bx.size, _p(bx),
                              _p(by), _p(bh), _p(bmref), _p(out))
    assert rc == 0
    return out


def bg_init_passes(ds_min: float, ds_max: float, cr: float) -> int:
    """Passes of the background initialisation of section 3.3: three per
    size level between ds_max and ds_min, 3 ceil(log_{C_r}(ds_max/ds_min))
    (the 1e-12 keeps an exact power of C_r from rounding up a level)."""
    return 3 * math.ceil(math.log(ds_max / ds_min) / math.log(cr) - 1e-12)


def bg_update(dom: Dom, bp: BgPrm, bg: dict, solids: dict, passes: int, cap: int | None = None,
              phi=None, phi_thresh: float = 0.0):
    """Background passes (section 3.3).  bg: x y h ds (f64), mask (i32), mq (i64), mref (f64)."""
    nb = bg["x"].size
    if cap is None:
        cap = max(8 * nb, 1024)
    A = {}
    for k in ("x", "y", "h", "ds", "mref"):
        a = np.zeros(cap)
        a[:nb] = bg[k]
        A[k] = a
    A["mask"] = np.zeros(cap, np.int32)
    A["mask"][:nb] = bg["mask"]
    A["mq"] = np.zeros(cap, np.int64)
    A["mq"][:nb] = bg["mq"]
    sx, sy, sh = (_f64(solids[k]) for k in ("x", "y", "h"))
    ph = None if phi is None else _f64(phi)
    nsplit = C.c_int64(0)
    nn = lib().or_bg_update(C.byref(dom.c()), C.byref(bp.c()), nb, cap, _p(A["x"]), _p(A["y"]),
                            _p(A["h"]), _p(A["ds"]), _p(A["mask"]), _p(A["mq"]), _p(A["mref"]),
                            sx.size, _p(sx), _p(sy), _p(sh), _p(ph), float(phi_thresh),
                            int(passes), C.byref(nsplit))
    if nn < 0:
        raise RuntimeError(f"oracle bg update failed: {nn}")
    out = {k: A[k][:nn].copy() for k in A}
    return out, int(nsplit.value)


def vorticity(dom: Dom, x, y, u, v, h, m, rho, rp, col):
    x, y, u, v, h, m, rho = map(_f64, (x, y, u, v, h, m, rho))
    out = np.zeros(x.size)
    lib().or_vorticity(C.byref(dom.c()), x.size, _p(x), _p(y), _p(u), _p(v), _p(h), _p(m), _p(rho),
                       _p(_i64(rp)), _p(_i32(col)), _p(out))
    return out


def shepard_to_bg(dom: Dom, bx, by, bh, x, y, h, f, kind=None):
    """Shepard average of the fluid field f at the background particles."""
    bx, by, bh, x, y, h, f = map(_f64, (bx, by, bh, x, y, h, f))
    kind = None if kind is None else _i32(kind)
    out = np.zeros(bx.size)
    rc = lib().or_shepard_to_bg(C.byref(dom.c()), bx.size, _p(bx), _p(by), _p(bh), x.size, _p(x),
                                _p(y), _p(h), _p(kind), _p(f), _p(out))
    assert rc == 0
    return out


# --------------------------------------------------------------------------
# diagnostics (section 4.1): kinetic energy, volume error, momentum
# --------------------------------------------------------------------------

def exact_sum(x) -> float:
    """The exact sum of the doubles x rounded once, ties to even (the long
    accumulator of the background update's sums)."""
    x = _f64(x)
    return float(lib().or_exact_sum(x.size, _p(x)))


def timestep(hmin, U, cs, nu):
    """eq. (timestep)."""
    return lib().or_timestep(float(hmin), float(U), float(cs), float(nu))


def dt_for(state: dict) -> float:
    """The time step of a workload: its explicit "dt" if it names one, else
    eq. (timestep) from its smallest smoothing length and reference speed."""
    if "dt" in state:
        return float(state["dt"])
    prm = state["params"]
    return timestep(state["h_min"], state["u_ref"], prm["cs"], prm["nu"])


def kinetic_energy(m, u, v):
    m, u, v = map(_f64, (m, u, v))
    return float(np.sum(0.5 * m * (u * u + v * v)))


def volume_error_pct(m, rho, area):
    """eps_V = |sum m/rho / L^2 - 1| * 100 (section 4.1)."""
    return float(abs(np.sum(_f64(m) / _f64(rho)) / area - 1.0) * 100.0)
