"""Python binding of the gfx950 adaptive-resolution WCSPH library.

Argument marshalling only: every step of the hot path runs in the HIP
library ``libsph.so`` (C ABI in ``include/sph.h``).  PyTorch provides device
memory (the particle arrays and the workspace) and the stream.  Importing
this package fails loudly if the library has not been built; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsph.so")

SPH_OK, SPH_E_INVAL, SPH_E_CAPACITY, SPH_E_NOMEM = 0, -1, -2, -3
SPH_E_DEVICE, SPH_E_NONFINITE, SPH_E_AGAIN = -4, -5, -6
SPH_FP64, SPH_FP32 = 0, 1
SPH_FLUID, SPH_SOLID, SPH_INLET, SPH_OUTLET = 0, 1, 2, 3
_ERRNAME = {0: "SPH_OK", -1: "SPH_E_INVAL", -2: "SPH_E_CAPACITY", -3: "SPH_E_NOMEM",
            -4: "SPH_E_DEVICE", -5: "SPH_E_NONFINITE", -6: "SPH_E_AGAIN"}


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAME.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# C structs (mirror include/sph.h)
# ---------------------------------------------------------------------------

class sph_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("periodic", C.c_int32 * 2),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2),
                ("h_lo", C.c_double), ("h_hi", C.c_double),
                ("rho0", C.c_double), ("cs", C.c_double), ("nu", C.c_double),
                ("alpha_e", C.c_double), ("hdx", C.c_double), ("u_ref", C.c_double),
                ("body_force", C.c_double * 2),
                ("split_alpha", C.c_double), ("split_eps", C.c_double),
                ("mmax_f", C.c_double), ("mmin_f", C.c_double), ("mass_q", C.c_double),
                ("merge_iters", C.c_int32), ("shift_iters", C.c_int32),
                ("cr", C.c_double), ("ds_min", C.c_double), ("ds_max", C.c_double),
                ("n_r", C.c_double), ("bg_smooth_iters", C.c_int32), ("bg_mass_q", C.c_double),
                ("wall_accel", C.c_double * 2), ("list_k", C.c_int32), ("lean", C.c_int32),
                ("list_skin", C.c_double), ("io_mode", C.c_int32), ("io_ref", C.c_double * 3),
                ("dt", C.c_double), ("sol_k", C.c_double), ("n_adapt", C.c_int32),
                ("n_bg", C.c_int32), ("bg_passes", C.c_int32), ("csr_k", C.c_int32)]


class sph_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p),
                ("p", C.c_void_p), ("rho", C.c_void_p), ("h", C.c_void_p), ("mref", C.c_void_p),
                ("mq", C.c_void_p), ("kind", C.c_void_p)]


class sph_csr(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("nnz_cap", C.c_int64),
                ("nnz", C.c_int64)]


class sph_rates_out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("rho", "beta", "pavg", "nnb", "dxs", "dys", "dpdt", "dudt", "dvdt")]


class sph_adapt_map(C.Structure):
    _fields_ = [("origin", C.c_void_p), ("sat", C.c_void_p), ("n_split", C.c_int64),
                ("n_required", C.c_int64), ("n_merged", C.c_int64 * 8)]


class sph_inout_params(C.Structure):
    _fields_ = [("x_in", C.c_double), ("len_in", C.c_double), ("x_out", C.c_double),
                ("len_out", C.c_double)]


class sph_inout_map(C.Structure):
    _fields_ = [("origin", C.c_void_p), ("n_appended", C.c_int64), ("n_deleted", C.c_int64),
                ("n_to_outlet", C.c_int64), ("n_required", C.c_int64)]


class sph_pool_stats(C.Structure):
    _fields_ = [("slots_total", C.c_int64), ("slots_used", C.c_int64),
                ("largest_free", C.c_int64), ("tables_total", C.c_int64),
                ("tables_used", C.c_int64), ("resident", C.c_int64), ("particles", C.c_int64),
                ("max_resident", C.c_int64), ("last_step_ms", C.c_double)]


class sph_background(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("h", C.c_void_p), ("ds", C.c_void_p),
                ("mref", C.c_void_p), ("mask", C.c_void_p), ("mq", C.c_void_p)]


SCHEDULE_FIELDS = ("a_lanes", "a_waves", "b_lanes", "b_unroll", "b_waves", "list_lanes")
# the launch-schedule variants compiled into the library (sph_set_schedule)
SCHEDULE_CHOICES = {"a_lanes": (2, 4, 8), "a_waves": (1, 4, 5), "b_lanes": (1, 2, 4),
                    "b_unroll": (2, 4), "b_waves": (1, 4), "list_lanes": (2, 4, 8)}
DEFAULT_SCHEDULE = {"a_lanes": 4, "a_waves": 5, "b_lanes": 2, "b_unroll": 2, "b_waves": 4,
                    "list_lanes": 4}


class sph_schedule(C.Structure):
    _fields_ = [(k, C.c_int32) for k in SCHEDULE_FIELDS]


class sph_diag(C.Structure):
    _fields_ = [("ke", C.c_double), ("vol", C.c_double), ("mom_x", C.c_double),
                ("mom_y", C.c_double), ("umax", C.c_double), ("mq_total", C.c_int64),
                ("n", C.c_int64)]


EXPORTS = ("sph_version", "sph_workspace_bytes", "sph_create", "sph_destroy", "sph_last_error",
           "sph_set_stream", "sph_build_neighbors", "sph_rates", "sph_pec", "sph_step",
           "sph_timestep", "sph_set_iteration", "sph_iteration", "sph_mref_lookup",
           "sph_adapt", "sph_bg_update", "sph_bg_init_passes", "sph_inout", "sph_diagnostics", "sph_body_force", "sph_move_solids",
           "sph_export_bytes", "sph_export", "sph_import",
           "sph_profile_enable",
           "sph_profile_read", "sph_profile_reset", "sph_vorticity", "sph_bg_update_solution", "sph_step_inout",
           "sph_pool_footprint", "sph_pool_create",
           "sph_pool_destroy", "sph_pool_last_error", "sph_pool_admit", "sph_pool_step",
           "sph_pool_sim_stats", "sph_pool_read", "sph_pool_retire", "sph_pool_info",
           "sph_rates_noalloc_bytes", "sph_rates_noalloc", "sph_set_schedule", "sph_get_schedule")

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libsph.so and declares the C signatures.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "sph_version": (C.c_int, []),
        "sph_workspace_bytes": (C.c_size_t, [P, I64]),
        "sph_create": (C.c_int, [P, I64, P, C.c_size_t, P, P]),
        "sph_destroy": (None, [P]),
        "sph_last_error": (C.c_char_p, [P]),
        "sph_set_stream": (C.c_int, [P, P]),
        "sph_build_neighbors": (C.c_int, [P, P, P]),
        "sph_rates": (C.c_int, [P, P, D, P]),
        "sph_pec": (C.c_int, [P, P, D, I32]),
        "sph_step": (C.c_int, [P, P, P, P, P, I32, P]),
        "sph_timestep": (D, [P, D]),
        "sph_set_iteration": (C.c_int, [P, I64]),
        "sph_iteration": (I64, [P]),
        "sph_mref_lookup": (C.c_int, [P, P, P]),
        "sph_adapt": (C.c_int, [P, P, P, P]),
        "sph_bg_update": (C.c_int, [P, P, P, P, D, I32, P]),
        "sph_bg_init_passes": (I32, [P]),
        "sph_set_schedule": (C.c_int, [P, P]),
        "sph_get_schedule": (C.c_int, [P, P]),
        "sph_inout": (C.c_int, [P, P, P, P]),
        "sph_vorticity": (C.c_int, [P, P, P]),
        "sph_step_inout": (C.c_int, [P, P, D, I32, P, P]),
        "sph_bg_update_solution": (C.c_int, [P, P, P, P, D, I32, P, P]),
        "sph_diagnostics": (C.c_int, [P, P, P]),
        "sph_body_force": (C.c_int, [P, P, P]),
        "sph_move_solids": (C.c_int, [P, P, P, P, P]),
        "sph_export_bytes": (C.c_size_t, [I64]),
        "sph_export": (C.c_int, [P, P, I64, D, P, C.c_size_t]),
        "sph_import": (C.c_int, [P, P, P, C.c_size_t, P, P]),
        "sph_profile_enable": (C.c_int, [P, I32]),
        "sph_profile_read": (C.c_int, [P, C.c_char_p, P, P]),
        "sph_profile_reset": (C.c_int, [P]),
        "sph_pool_footprint": (C.c_size_t, [P, I64]),
        "sph_pool_create": (C.c_int, [P, C.c_size_t, I32, P]),
        "sph_pool_destroy": (None, [P]),
        "sph_pool_last_error": (C.c_char_p, [P]),
        "sph_pool_admit": (C.c_int, [P, P, P, D, P, P]),
        "sph_pool_step": (C.c_int, [P, I32]),
        "sph_pool_sim_stats": (C.c_int, [P, I32, P, P, P]),
        "sph_pool_read": (C.c_int, [P, I32, P, P]),
        "sph_pool_retire": (C.c_int, [P, I32]),
        "sph_pool_info": (C.c_int, [P, P]),
        "sph_rates_noalloc_bytes": (C.c_size_t, [P, I64]),
        "sph_rates_noalloc": (C.c_int, [P, P, D, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------------------
# Python-side helpers
# ---------------------------------------------------------------------------

@dataclass
class Config:
    lo: tuple = (0.0, 0.0)
    hi: tuple = (1.0, 1.0)
    periodic: tuple = (True, True)
    h_lo: float = 0.02
    h_hi: float = 0.02
    precision: int = SPH_FP64
    rho0: float = 1.0
    cs: float = 10.0
    nu: float = 0.01
    alpha_e: float = 1.5
    hdx: float = 1.0
    u_ref: float = 1.0
    body_force: tuple = (0.0, 0.0)
    split_alpha: float = 0.9
    split_eps: float = 0.4
    mmax_f: float = 1.05
    mmin_f: float = 0.5
    mass_q: float = 2.0 ** -60
    merge_iters: int = 3
    shift_iters: int = 3
    cr: float = 1.05
    ds_min: float = 0.01
    ds_max: float = 0.64
    n_r: float = 48.0
    bg_smooth_iters: int = 3
    bg_mass_q: float = 2.0 ** -60
    wall_accel: tuple = (0.0, 0.0)
    list_k: int = 0
    lean: int = 0
    list_skin: float = 0.1
    io_mode: int = 0
    io_ref: tuple = (0.0, 0.0, 0.0)
    dt: float = 0.0
    sol_k: float = 0.0
    n_adapt: int = 0
    n_bg: int = 0
    bg_passes: int = 1
    csr_k: int = 0

    def c(self) -> sph_config:
        s = sph_config()
        s.precision = int(self.precision)
        s.periodic[0], s.periodic[1] = int(self.periodic[0]), int(self.periodic[1])
        s.lo[0], s.lo[1] = self.lo
        s.hi[0], s.hi[1] = self.hi
        s.body_force[0], s.body_force[1] = self.body_force
        s.wall_accel[0], s.wall_accel[1] = self.wall_accel
        s.io_ref[0], s.io_ref[1], s.io_ref[2] = self.io_ref
        for k in ("h_lo", "h_hi", "rho0", "cs", "nu", "alpha_e", "hdx", "u_ref", "split_alpha",
                  "split_eps", "mmax_f", "mmin_f", "mass_q", "merge_iters", "shift_iters", "cr",
                  "ds_min", "ds_max", "n_r", "bg_smooth_iters", "bg_mass_q", "list_k", "lean", "list_skin",
                  "io_mode", "dt", "sol_k", "n_adapt", "n_bg", "bg_passes", "csr_k"):
            setattr(s, k, getattr(self, k))
        return s


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


_F64 = ("x", "y", "u", "v", "p", "rho", "h", "mref")


class Particles:
    """Structure-of-arrays particle set in device memory (torch tensors)."""

    def __init__(self, capacity: int, device="cuda"):
        self.capacity = int(capacity)
        self.n = 0
        self.device = torch.device(device)
        for k in _F64:
            setattr(self, k, torch.zeros(self.capacity, dtype=torch.float64, device=self.device))
        self.mq = torch.zeros(self.capacity, dtype=torch.int64, device=self.device)
        self.kind = torch.zeros(self.capacity, dtype=torch.int32, device=self.device)

    @classmethod
    def from_arrays(cls, d: dict, capacity: int | None = None, device="cuda"):
        n = len(d["x"])
        P = cls(capacity or n, device)
        P.n = n
        for k in _F64:
            if k in d:
                getattr(P, k)[:n] = torch.as_tensor(d[k], dtype=torch.float64)
        if "rho" not in d:
            P.rho[:n] = 1.0
        P.mq[:n] = torch.as_tensor(d["mq"], dtype=torch.int64)
        if "kind" in d:
            P.kind[:n] = torch.as_tensor(d["kind"], dtype=torch.int32)
        return P

    def c(self) -> sph_particles:
        s = sph_particles()
        s.n, s.capacity = self.n, self.capacity
        for k in _F64:
            setattr(s, k, _ptr(getattr(self, k)))
        s.mq, s.kind = _ptr(self.mq), _ptr(self.kind)
        return s

    def numpy(self) -> dict:
        n = self.n
        out = {k: getattr(self, k)[:n].cpu().numpy() for k in _F64}
        out["mq"] = self.mq[:n].cpu().numpy()
        out["kind"] = self.kind[:n].cpu().numpy()
        return out


class Background:
    """Background particles of section 3.3 (device tensors)."""

    def __init__(self, capacity: int, device="cuda"):
        self.capacity = int(capacity)
        self.n = 0
        dev = torch.device(device)
        for k in ("x", "y", "h", "ds", "mref"):
            setattr(self, k, torch.zeros(self.capacity, dtype=torch.float64, device=dev))
        self.mask = torch.zeros(self.capacity, dtype=torch.int32, device=dev)
        self.mq = torch.zeros(self.capacity, dtype=torch.int64, device=dev)

    @classmethod
    def from_arrays(cls, d: dict, capacity: int | None = None, device="cuda"):
        n = len(d["x"])
        B = cls(capacity or n, device)
        B.n = n
        for k in ("x", "y", "h", "ds", "mref"):
            getattr(B, k)[:n] = torch.as_tensor(d[k], dtype=torch.float64)
        B.mask[:n] = torch.as_tensor(d["mask"], dtype=torch.int32)
        B.mq[:n] = torch.as_tensor(d["mq"], dtype=torch.int64)
        return B

    def c(self) -> sph_background:
        s = sph_background()
        s.n, s.capacity = self.n, self.capacity
        for k in ("x", "y", "h", "ds", "mref", "mask", "mq"):
            setattr(s, k, _ptr(getattr(self, k)))
        return s

    def numpy(self) -> dict:
        n = self.n
        out = {k: getattr(self, k)[:n].cpu().numpy() for k in ("x", "y", "h", "ds", "mref")}
        out["mask"] = self.mask[:n].cpu().numpy()
        out["mq"] = self.mq[:n].cpu().numpy()
        return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def rates_noalloc_bytes(cfg: "Config", n: int) -> int:
    """Scratch bytes sph_rates_noalloc needs for n particles."""
    return int(load_library().sph_rates_noalloc_bytes(C.byref(cfg.c()), int(n)))


def rates_noalloc(cfg: "Config", P: "Particles", dt: float, out: dict | None = None, stream=None):
    """One rate evaluation through sph_rates_noalloc (no context, no
    allocation inside the library; scratch is its static device array).
    `out` may hold preallocated float64 tensors of the fields."""
    lib = load_library()
    n = P.n
    if out is None:
        out = {k: torch.empty(max(n, 1), dtype=torch.float64, device=P.device)
               for k in ("rho", "beta", "pavg", "nnb", "dxs", "dys", "dpdt", "dudt", "dvdt")}
    ro = sph_rates_out(**{k: _ptr(v).value for k, v in out.items()})
    st = stream if stream is not None else torch.cuda.current_stream(P.device)
    ps = P.c()
    c = cfg.c()
    rc = lib.sph_rates_noalloc(C.byref(c), C.byref(ps), float(dt), C.byref(ro),
                               C.c_void_p(st.cuda_stream))
    if rc != SPH_OK:
        msg = lib.sph_last_error(None)
        raise SphError(rc, msg.decode() if msg else "")
    return {k: v[:n] for k, v in out.items()}


class Context:
    """A library context bound to one device, stream and workspace."""

    def __init__(self, cfg: Config, capacity: int, device="cuda", stream=None):
        self.lib = load_library()
        self.cfg = cfg
        self.device = torch.device(device)
        self.capacity = int(capacity)
        self._c = cfg.c()
        nbytes = self.lib.sph_workspace_bytes(C.byref(self._c), self.capacity)
        if nbytes == 0:
            raise SphError(SPH_E_INVAL, "invalid configuration")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.sph_create(C.byref(self._c), self.capacity, _ptr(self.workspace), nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != SPH_OK:
            raise SphError(rc, "sph_create failed")
        self._h = h

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self.lib.sph_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _check(self, rc):
        if rc != SPH_OK:
            msg = self.lib.sph_last_error(self._h)
            raise SphError(rc, msg.decode() if msg else "")

    # -- hot path ----------------------------------------------------------

    def build_neighbors(self, P: Particles, csr: bool = True, nnz_cap: int | None = None):
        ps = P.c()
        if not csr:
            self._check(self.lib.sph_build_neighbors(self._h, C.byref(ps), None))
            return None
        cap = nnz_cap if nnz_cap is not None else max(96 * P.n, 1)
        rp = torch.empty(P.n + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        out = sph_csr(row_ptr=_ptr(rp).value, col=_ptr(col).value, nnz_cap=cap, nnz=0)
        rc = self.lib.sph_build_neighbors(self._h, C.byref(ps), C.byref(out))
        if rc == SPH_E_CAPACITY and nnz_cap is None:
            return self.build_neighbors(P, True, int(out.nnz))
        self._check(rc)
        return rp, col[:out.nnz]

    def rates(self, P: Particles, dt: float):
        n = P.n
        out = {k: torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
               for k in ("rho", "beta", "pavg", "nnb", "dxs", "dys", "dpdt", "dudt", "dvdt")}
        ro = sph_rates_out(**{k: _ptr(v).value for k, v in out.items()})
        ps = P.c()
        self._check(self.lib.sph_rates(self._h, C.byref(ps), float(dt), C.byref(ro)))
        return {k: v[:n] for k, v in out.items()}

    def step(self, P: Particles, dt: float, nsteps: int = 1):
        """nsteps plain PEC steps (sph_pec)."""
        ps = P.c()
        self._check(self.lib.sph_pec(self._h, C.byref(ps), float(dt), int(nsteps)))

    def run(self, P: Particles, nsteps: int, bg: "Background | None" = None,
            solids: "Particles | None" = None, io: dict | None = None, diag: bool = False):
        """nsteps iterations of the schedule of section 3.4 (sph_step): the
        background update every cfg.n_bg and the adaptation every
        cfg.n_adapt iterations, then the step (dt = cfg.dt, or eq. timestep)
        and the inlet/outlet update when io is given.  Returns the
        diagnostics of the final state when diag is set."""
        ps = P.c()
        bs = bg.c() if bg is not None else None
        ss = solids.c() if solids is not None else None
        prm = (sph_inout_params(float(io["x_in"]), float(io["len_in"]), float(io["x_out"]),
                                float(io["len_out"])) if io is not None else None)
        d = sph_diag()
        rc = self.lib.sph_step(self._h, C.byref(ps), C.byref(bs) if bs is not None else None,
                               C.byref(ss) if ss is not None else None,
                               C.byref(prm) if prm is not None else None, int(nsteps),
                               C.byref(d) if diag else None)
        P.n = int(ps.n)
        if bg is not None:
            bg.n = int(bs.n)
        self._check(rc)
        if diag:
            return {k: getattr(d, k) for k, _ in sph_diag._fields_}
        return None

    @property
    def iteration(self) -> int:
        return int(self.lib.sph_iteration(self._h))

    @iteration.setter
    def iteration(self, it: int):
        self._check(self.lib.sph_set_iteration(self._h, int(it)))

    def mref_lookup(self, P: Particles, bg: Background):
        ps, bs = P.c(), bg.c()
        self._check(self.lib.sph_mref_lookup(self._h, C.byref(ps), C.byref(bs)))

    def adapt(self, P: Particles, bg: Background | None = None):
        origin = torch.empty(P.capacity, dtype=torch.int64, device=self.device)
        sat = torch.empty(P.capacity, dtype=torch.int32, device=self.device)
        m = sph_adapt_map(origin=_ptr(origin).value, sat=_ptr(sat).value)
        ps = P.c()
        bs = bg.c() if bg is not None else None
        rc = self.lib.sph_adapt(self._h, C.byref(ps), C.byref(bs) if bs is not None else None,
                                C.byref(m))
        info = {"n_split": int(m.n_split), "n_required": int(m.n_required),
                "merged": [int(m.n_merged[k]) for k in range(self.cfg.merge_iters)]}
        if rc == SPH_E_CAPACITY:
            info["error"] = rc
            return info
        self._check(rc)
        P.n = int(ps.n)
        info["origin"] = origin[:P.n]
        info["sat"] = sat[:P.n]
        return info

    def step_inout(self, P: Particles, dt: float, nsteps: int, io: dict):
        """nsteps of (step, inlet/outlet update) in one call (sph_step_inout)."""
        origin = torch.empty(P.capacity, dtype=torch.int64, device=self.device)
        m = sph_inout_map(origin=_ptr(origin).value)
        prm = sph_inout_params(float(io["x_in"]), float(io["len_in"]), float(io["x_out"]),
                               float(io["len_out"]))
        ps = P.c()
        rc = self.lib.sph_step_inout(self._h, C.byref(ps), float(dt), int(nsteps), C.byref(prm),
                                     C.byref(m))
        P.n = int(ps.n)
        self._check(rc)
        info = {"appended": int(m.n_appended), "deleted": int(m.n_deleted),
                "to_outlet": int(m.n_to_outlet)}
        if info["appended"] or info["deleted"]:
            info["origin"] = origin[:P.n]
        else:
            info["origin"] = torch.arange(P.n, dtype=torch.int64, device=self.device)
        return info

    def vorticity(self, P: Particles):
        out = torch.empty(max(P.n, 1), dtype=torch.float64, device=self.device)
        ps = P.c()
        self._check(self.lib.sph_vorticity(self._h, C.byref(ps), _ptr(out)))
        return out[:P.n]

    def bg_update_solution(self, bg: "Background", solids: Particles, fluid: Particles,
                           k_frac: float, passes: int):
        bs, ss, fs = bg.c(), solids.c(), fluid.c()
        ns, om = C.c_int64(0), C.c_double(0)
        self._check(self.lib.sph_bg_update_solution(self._h, C.byref(bs), C.byref(ss), C.byref(fs),
                                                    float(k_frac), int(passes), C.byref(ns),
                                                    C.byref(om)))
        bg.n = int(bs.n)
        return {"nsplit": int(ns.value), "omega_max": om.value}

    def inout(self, P: Particles, io: dict):
        """Inlet/outlet update (sph_inout); io has x_in, len_in, x_out, len_out."""
        origin = torch.empty(P.capacity, dtype=torch.int64, device=self.device)
        m = sph_inout_map(origin=_ptr(origin).value)
        prm = sph_inout_params(float(io["x_in"]), float(io["len_in"]), float(io["x_out"]),
                               float(io["len_out"]))
        ps = P.c()
        rc = self.lib.sph_inout(self._h, C.byref(ps), C.byref(prm), C.byref(m))
        info = {"appended": int(m.n_appended), "deleted": int(m.n_deleted),
                "to_outlet": int(m.n_to_outlet), "n_required": int(m.n_required)}
        if rc == SPH_E_CAPACITY:
            info["error"] = rc
            return info
        self._check(rc)
        P.n = int(ps.n)
        if info["appended"] or info["deleted"]:
            info["origin"] = origin[:P.n]
        else:  # no slot moved: the map is the identity (the library leaves it unwritten)
            info["origin"] = torch.arange(P.n, dtype=torch.int64, device=self.device)
        return info

    def bg_update(self, bg: Background, solids: Particles, passes: int, phi=None,
                  phi_thresh: float = 0.0):
        bs, ss = bg.c(), solids.c()
        ns = C.c_int64(0)
        self._check(self.lib.sph_bg_update(self._h, C.byref(bs), C.byref(ss), _ptr(phi),
                                           float(phi_thresh), int(passes), C.byref(ns)))
        bg.n = int(bs.n)
        return int(ns.value)

    def body_force(self, P: Particles) -> dict:
        """Force on the solid particles (sph_body_force): pressure and
        viscous totals and the magnitude sums of their terms."""
        f = (C.c_double * 8)()
        ps = P.c()
        self._check(self.lib.sph_body_force(self._h, C.byref(ps), f))
        return {"fp": (f[0], f[1]), "fvisc": (f[2], f[3]), "abs_p": (f[4], f[5]),
                "abs_visc": (f[6], f[7])}

    def move_solids(self, P: Particles, disp, vel, acc=(0.0, 0.0)):
        """Prescribed rigid motion of the solids (sph_move_solids): translate
        by disp, set their velocity to vel and the wall acceleration to acc."""
        D2 = C.c_double * 2
        ps = P.c()
        self._check(self.lib.sph_move_solids(self._h, C.byref(ps), D2(*disp), D2(*vel), D2(*acc)))

    def export(self, P: Particles, step: int = 0, time: float = 0.0):
        """Checkpoint of P (sph_export) as a numpy uint8 array; write it with
        `arr.tofile(path)` and read it back with `numpy.fromfile(path, numpy.uint8)`."""
        import numpy as np
        buf = np.empty(self.lib.sph_export_bytes(int(P.n)), dtype=np.uint8)
        ps = P.c()
        self._check(self.lib.sph_export(self._h, C.byref(ps), int(step), float(time),
                                        buf.ctypes.data_as(C.c_void_p), buf.size))
        return buf

    def import_(self, P: Particles, buf):
        """Restores a checkpoint into P (sph_import); returns (step, time)."""
        import numpy as np
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        ps = P.c()
        st, tm = C.c_int64(0), C.c_double(0.0)
        self._check(self.lib.sph_import(self._h, C.byref(ps), buf.ctypes.data_as(C.c_void_p),
                                        buf.size, C.byref(st), C.byref(tm)))
        P.n = int(ps.n)
        return int(st.value), float(tm.value)

    def diagnostics(self, P: Particles) -> dict:
        d = sph_diag()
        ps = P.c()
        self._check(self.lib.sph_diagnostics(self._h, C.byref(ps), C.byref(d)))
        return {k: getattr(d, k) for k, _ in sph_diag._fields_}

    # -- profiling ---------------------------------------------------------

    PROFILE_BITS = {"pass_a": 1, "pass_b": 2, "build": 4, "list": 8}

    @property
    def schedule(self) -> dict:
        """The context's launch schedule (sph_get_schedule)."""
        sc = sph_schedule()
        self._check(self.lib.sph_get_schedule(self._h, C.byref(sc)))
        return {k: int(getattr(sc, k)) for k in SCHEDULE_FIELDS}

    def set_schedule(self, **kw) -> dict:
        """Changes the named fields of the launch schedule (sph_set_schedule);
        SphError for a combination not compiled in."""
        cur = self.schedule
        unknown = set(kw) - set(SCHEDULE_FIELDS)
        if unknown:
            raise ValueError(f"unknown schedule fields {sorted(unknown)}")
        cur.update({k: int(v) for k, v in kw.items()})
        sc = sph_schedule(**cur)
        self._check(self.lib.sph_set_schedule(self._h, C.byref(sc)))
        return cur

    def profile(self, on: bool = True, kernels=("pass_a", "pass_b", "build", "list"), every: int = 1):
        """Brackets every `every`-th launch of the named kernels with events."""
        if not 1 <= every <= 255:
            raise ValueError("every must be in [1, 255]")
        mask = (sum(self.PROFILE_BITS[k] for k in kernels) | (every << 8)) if on else 0
        self._check(self.lib.sph_profile_enable(self._h, int(mask)))

    def profile_reset(self):
        self._check(self.lib.sph_profile_reset(self._h))

    def profile_read(self, kernel: str):
        ms, cnt = C.c_double(0), C.c_int64(0)
        self._check(self.lib.sph_profile_read(self._h, kernel.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value


def footprint(cfg: Config, n: int) -> int:
    """Arena bytes one simulation of n particles takes in a serving pool."""
    return int(load_library().sph_pool_footprint(C.byref(cfg.c()), int(n)))


class Pool:
    """Serving pool (sph_pool_*): independent fluid-only simulations resident
    in one device arena, advanced together by one batched step."""

    def __init__(self, arena_bytes: int, max_sims: int = 256, device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        rc = self.lib.sph_pool_create(_ptr(self.arena), int(arena_bytes), int(max_sims), C.byref(h))
        if rc != SPH_OK:
            raise SphError(rc, "pool creation failed")
        self._h = h
        self._inputs = []   # initial states read by copies not yet known to be done

    def _check(self, rc):
        if rc != SPH_OK:
            raise SphError(rc, self.lib.sph_pool_last_error(self._h).decode())

    def footprint(self, cfg: Config, n: int) -> int:
        return footprint(cfg, n)

    def admit(self, cfg: Config, P: Particles, dt: float):
        """Returns the simulation id, or None when the arena has no room."""
        c = cfg.c()
        ps = P.c()
        ps.kind = None
        sid = C.c_int32(-1)
        st = torch.cuda.current_stream(self.device)
        rc = self.lib.sph_pool_admit(self._h, C.byref(c), C.byref(ps), float(dt),
                                     C.c_void_p(st.cuda_stream), C.byref(sid))
        if rc == SPH_E_AGAIN:
            return None
        self._check(rc)
        self._inputs.append(P)   # kept alive until the next step has copied it
        return int(sid.value)

    def step(self, nsteps: int = 1):
        self._check(self.lib.sph_pool_step(self._h, int(nsteps)))
        self._inputs.clear()

    def stats(self, sim_id: int, pairs: bool = False) -> dict:
        ms, st, pe = C.c_double(0), C.c_int64(0), C.c_int64(0)
        self._check(self.lib.sph_pool_sim_stats(self._h, int(sim_id), C.byref(ms), C.byref(st),
                                                C.byref(pe) if pairs else None))
        out = {"last_ms": ms.value, "steps": st.value}
        if pairs:
            out["pair_evals"] = pe.value
        return out

    def read(self, sim_id: int, P: Particles):
        ps = P.c()
        ps.mref, ps.kind = None, None
        st = torch.cuda.current_stream(self.device)
        self._check(self.lib.sph_pool_read(self._h, int(sim_id), C.byref(ps), C.c_void_p(st.cuda_stream)))
        P.n = int(ps.n)
        return P

    def retire(self, sim_id: int):
        self._check(self.lib.sph_pool_retire(self._h, int(sim_id)))

    def info(self) -> dict:
        st = sph_pool_stats()
        self._check(self.lib.sph_pool_info(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in sph_pool_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self.lib.sph_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timestep(cfg: Config, h_min: float = 0.0) -> float:
    """eq. (timestep) for the configuration (sph_timestep); h_min <= 0 takes
    cfg.h_lo."""
    return float(load_library().sph_timestep(C.byref(cfg.c()), float(h_min)))


def bg_init_passes(cfg: Config) -> int:
    """Passes of the background initialisation from ds_max (section 3.3,
    sph_bg_init_passes): 3 ceil(ln(ds_max/ds_min) / ln C_r)."""
    return int(load_library().sph_bg_init_passes(C.byref(cfg.c())))


def config_for(domain, params: dict, h_lo: float, h_hi: float, precision=SPH_FP64,
               mass_q: float = 2.0 ** -60, **kw) -> Config:
    """Config from a workload's domain/params (see the workloads module);
    params may also name the inlet/outlet rule (io_mode, io_ref)."""
    for k in ("io_mode", "io_ref"):
        if k in params and k not in kw:
            kw[k] = params[k]
    return Config(lo=tuple(domain.lo), hi=tuple(domain.hi), periodic=tuple(domain.periodic),
                  h_lo=h_lo, h_hi=h_hi, precision=precision, rho0=params["rho0"],
                  cs=params["cs"], nu=params["nu"], hdx=params["hdx"], mass_q=mass_q, **kw)
