"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This module holds problem set-ups only (particle placement, initial fields,
masses in integer quanta); none of the SPH method's arithmetic lives here, so
the oracle and the HIP library can both be fed from it without sharing any of
the computation they are compared on.  Every generator takes an explicit seed
and uses numpy's PCG64 generator.

Workloads follow the set-ups of Muta & Ramachandran (arXiv 2107.01276):
the periodic Taylor-Green vortex (section 4.1), the Gresho-Chan vortex
(section 4.2), and the channel with a
circular cylinder (section 4.4), built here from a stated grading recipe
because the paper's layout figure is not available.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def mass_quantum(m_cap: float) -> float:
    """Power-of-two mass quantum: every mass up to m_cap is an integer number
    of quanta below 2**41, so mq * q is exact in double and the int64 ledger
    total of up to 2**22 particles at the cap cannot overflow; the resolution,
    2**-40 of the cap, is far below any mass difference the method makes."""
    e = math.floor(math.log2(m_cap))
    return math.ldexp(1.0, e - 40)


def quantize_mass(m: np.ndarray, q: float) -> np.ndarray:
    return np.rint(np.asarray(m, dtype=np.float64) / q).astype(np.int64)


@dataclass
class Domain:
    lo: tuple
    hi: tuple
    periodic: tuple

    @property
    def area(self):
        return (self.hi[0] - self.lo[0]) * (self.hi[1] - self.lo[1])


# ---------------------------------------------------------------------------
# Taylor-Green vortex on the periodic unit square (section 4.1)
# ---------------------------------------------------------------------------

def tgv_fields(x, y, t=0.0, re=100.0):
    """Exact Taylor-Green solution (U = L = rho0 = 1), decay rate b = -8 pi^2/Re."""
    b = -8.0 * math.pi ** 2 / re
    e = math.exp(b * t)
    u = -e * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
    v = e * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    p = -(e * e) * (np.cos(4 * np.pi * x) + np.cos(4 * np.pi * y)) / 4.0
    return u, v, p


def tgv(nx: int = 50, seed: int = 1, jitter: float = 0.05, hdx: float = 1.0,
        re: float = 100.0, rho0: float = 1.0, cs: float = 10.0, perturb: bool = True):
    """nx*nx particles on a lattice jittered by U(-jitter, jitter)*dx per axis."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / nx
    i, j = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    x = ((i.ravel() + 0.5) * dx).astype(np.float64)
    y = ((j.ravel() + 0.5) * dx).astype(np.float64)
    if perturb and jitter > 0:
        x = x + rng.uniform(-jitter, jitter, x.size) * dx
        y = y + rng.uniform(-jitter, jitter, y.size) * dx
    x = np.mod(x, 1.0)
    y = np.mod(y, 1.0)
    u, v, p = tgv_fields(x, y, 0.0, re)
    m = np.full(x.size, rho0 * dx * dx)
    q = mass_quantum(1.05 * m.max())
    mq = quantize_mass(m, q)
    h = np.full(x.size, hdx * dx)
    nu = 1.0 / re
    return {
        "x": x, "y": y, "u": u, "v": v, "p": p, "h": h,
        "mq": mq, "mass_q": q, "m": mq.astype(np.float64) * q,
        "rho": np.full(x.size, rho0), "mref": np.full(x.size, rho0 * dx * dx),
        "kind": np.zeros(x.size, np.int32),
        "domain": Domain((0.0, 0.0), (1.0, 1.0), (True, True)),
        "params": {"rho0": rho0, "cs": cs, "nu": nu, "hdx": hdx, "re": re},
        "h_min": hdx * dx, "u_ref": 1.0, "dx": dx,
    }


# ---------------------------------------------------------------------------
# Gresho-Chan vortex on the periodic unit square (section 4.2)
# ---------------------------------------------------------------------------

GC_R = 0.2   # radius of the solid-body core, in units of the box length
GC_P0 = 5.0  # reference pressure


def gresho_chan_fields(x, y, rho0: float = 1.0):
    """Exact steady state of the vortex centred at the origin (positions in
    [-0.5, 0.5)): the azimuthal velocity of eq. (gc-az) and the pressure that
    balances its centrifugal force, eq. (gc-p).  Reading: the outer pressure
    constant is 4 ln 2 - 2 (the printed 4 ln 2 - 4 breaks continuity at
    r = 2R; the middle branch gives 4 ln 2 - 2 there)."""
    r = np.hypot(x, y)
    R = GC_R
    uphi = np.where(r < R, r / R, np.where(r < 2 * R, 2.0 - r / R, 0.0))
    rs = np.maximum(r, 1e-300)
    p_mid = 4.0 - 4.0 * math.log(0.2) + 12.5 * r * r - 20.0 * r + 4.0 * np.log(rs)
    p = GC_P0 + rho0 * np.where(r < R, 12.5 * r * r,
                                np.where(r < 2 * R, p_mid, 4.0 * math.log(2.0) - 2.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.where(r > 0, -uphi * y / rs, 0.0)
        v = np.where(r > 0, uphi * x / rs, 0.0)
    return u, v, p, uphi


def gresho_chan(nx: int = 50, hdx: float = 1.0, rho0: float = 1.0, cs: float = 10.0):
    """nx*nx particles on a uniform Cartesian lattice of the periodic box
    [-0.5, 0.5)^2 (section 4.2: uniform grid start, c_s = 10, h/dx = 1,
    inviscid), with the exact fields of `gresho_chan_fields`."""
    dx = 1.0 / nx
    i, j = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    x = (-0.5 + (i.ravel() + 0.5) * dx).astype(np.float64)
    y = (-0.5 + (j.ravel() + 0.5) * dx).astype(np.float64)
    u, v, p, _ = gresho_chan_fields(x, y, rho0)
    m = np.full(x.size, rho0 * dx * dx)
    q = mass_quantum(1.05 * m.max())
    mq = quantize_mass(m, q)
    h = np.full(x.size, hdx * dx)
    return {
        "x": x, "y": y, "u": u, "v": v, "p": p, "h": h,
        "mq": mq, "mass_q": q, "m": mq.astype(np.float64) * q,
        "rho": np.full(x.size, rho0), "mref": m.copy(), "kind": np.zeros(x.size, np.int32),
        "domain": Domain((-0.5, -0.5), (0.5, 0.5), (True, True)),
        "params": {"rho0": rho0, "cs": cs, "nu": 0.0, "hdx": hdx},
        "h_min": hdx * dx, "u_ref": 1.0, "dx": dx,
    }


def gresho_chan_background(nx: int = 50, radius: float = 0.45, frac: float = 0.5,
                           sparsity: float = 2.0, rho0: float = 1.0):
    """Prescribed background for the adaptive run: a lattice of spacing
    sparsity * dx whose particles inside `radius` of the origin ask for
    m_ref = frac * rho0 dx^2 (the refined region of section 4.2) and
    rho0 dx^2 elsewhere; h = 1.3 * sparsity * dx."""
    dx = 1.0 / nx
    nb = int(round(nx / sparsity))
    db = 1.0 / nb
    i, j = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    x = (-0.5 + (i.ravel() + 0.5) * db).astype(np.float64)
    y = (-0.5 + (j.ravel() + 0.5) * db).astype(np.float64)
    m0 = rho0 * dx * dx
    inner = np.hypot(x, y) < radius
    mref = np.where(inner, frac * m0, m0)
    ds = np.where(inner, math.sqrt(frac) * dx, dx)
    q = mass_quantum(1.05 * m0)
    return {"x": x, "y": y, "h": np.full(x.size, 1.3 * db), "ds": ds,
            "mask": inner.astype(np.int32), "mq": quantize_mass(mref, q), "mass_q": q,
            "mref": mref}


# ---------------------------------------------------------------------------
# Random variable-h sets for neighbour-search parity
# ---------------------------------------------------------------------------

def random_varh(n: int, seed: int, h_lo: float = 0.01, ratio: float = 8.0,
                periodic=(True, True), lo=(0.0, 0.0), hi=(1.0, 1.0)):
    """Uniform positions, smoothing lengths log-uniform in [h_lo, ratio*h_lo]."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo[0], hi[0], n)
    y = rng.uniform(lo[1], hi[1], n)
    h = h_lo * np.exp(rng.uniform(0.0, math.log(ratio), n))
    return {"x": x, "y": y, "h": h, "domain": Domain(tuple(lo), tuple(hi), tuple(periodic))}


def clustered_varh(n: int, seed: int, h_lo: float = 0.004, ratio: float = 16.0,
                   periodic=(False, True), lo=(0.0, -1.0), hi=(3.0, 1.0)):
    """Positions concentrated around a point, h growing with distance from it
    (the structure of a graded refinement around a body)."""
    rng = np.random.default_rng(seed)
    cx, cy = lo[0] + 0.35 * (hi[0] - lo[0]), 0.5 * (lo[1] + hi[1])
    r = np.abs(rng.normal(0.0, 0.35, n)) + 0.02
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.clip(cx + r * np.cos(th), lo[0], np.nextafter(hi[0], lo[0]))
    y = cy + r * np.sin(th)
    span = hi[1] - lo[1]
    y = lo[1] + np.mod(y - lo[1], span)
    y = np.where(y >= hi[1], lo[1], y)
    t = np.clip(r / r.max(), 0, 1)
    h = h_lo * ratio ** t * np.exp(rng.uniform(-0.1, 0.1, n))
    return {"x": x, "y": y, "h": h, "domain": Domain(tuple(lo), tuple(hi), tuple(periodic))}


# ---------------------------------------------------------------------------
# Channel with a circular cylinder (section 4.4 set-up, graded by distance)
# ---------------------------------------------------------------------------

@dataclass
class ChannelSpec:
    length: float = 30.0          # in D
    height: float = 20.0          # in D
    cyl_x: float = 10.0
    cyl_y: float = 0.0
    diameter: float = 1.0
    ds_min: float = 0.01          # D/100
    ratio: int = 64               # ds_max / ds_min
    cr: float = 1.05              # size growth per layer
    rows_per_layer: float = 5.0   # particle rows per C_r layer
    hdx: float = 1.2
    rho0: float = 1.0
    u_inf: float = 1.0
    re: float = 100.0
    cs: float = 10.0
    wall_layers: int = 5
    io_layers: int = 4            # inlet/outlet buffer columns (0: closed ends)
    jitter: float = 0.05


def _ring_points(rng, r, ds, cx, cy):
    n = max(int(round(2 * math.pi * r / ds)), 3)
    th = rng.uniform(0, 2 * math.pi) + 2 * math.pi * np.arange(n) / n
    return cx + r * np.cos(th), cy + r * np.sin(th)


def channel_cylinder(spec: ChannelSpec | None = None, seed: int = 2):
    """Fluid graded by distance d from the cylinder surface, plus solid
    dummy-particle layers inside the cylinder.

    Recipe: the target size grows by the factor C_r every `rows_per_layer`
    rows, i.e. s(d) = ds_min + d ln(C_r)/rows_per_layer, capped at ds_max.
    Fluid spacings are restricted to ds_min * 2**(k/2) (each refinement level
    halves the mass), so a particle at distance d takes the largest such
    spacing not above s(d).  Rings of constant spacing are laid around the
    cylinder until the spacing reaches ds_max; outside, a lattice of spacing
    ~ds_max fills the channel (periodic in y).  Every particle is jittered by
    U(-jitter, jitter) of its spacing.  Velocity is the potential flow past
    the cylinder, pressure from Bernoulli.
    """
    s = spec or ChannelSpec()
    rng = np.random.default_rng(seed)
    R = 0.5 * s.diameter
    ds_max = s.ds_min * s.ratio
    nlev = int(round(2 * math.log2(s.ratio)))
    lev_ds = s.ds_min * np.sqrt(2.0) ** np.arange(nlev + 1)
    lo = (0.0, s.cyl_y - 0.5 * s.height)
    hi = (s.length, s.cyl_y + 0.5 * s.height)
    slope = math.log(s.cr) / s.rows_per_layer

    xs, ys, dss = [], [], []
    r = R + 0.5 * s.ds_min
    while True:
        d = r - R
        target = min(s.ds_min + d * slope, ds_max)
        k = int(np.searchsorted(lev_ds, target * (1 + 1e-12), side="right") - 1)
        k = max(0, min(k, nlev))
        ds = lev_ds[k]
        if k == nlev or target >= ds_max:
            break
        px, py = _ring_points(rng, r, ds, s.cyl_x, s.cyl_y)
        xs.append(px); ys.append(py); dss.append(np.full(px.size, ds))
        r += ds
    r_outer = r
    # outer lattice at ~ds_max, aligned to the periodic height
    ny = max(int(round(s.height / ds_max)), 1)
    dyl = s.height / ny
    nx = max(int(round(s.length / dyl)), 1)
    dxl = s.length / nx
    gi, gj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    gx = lo[0] + (gi.ravel() + 0.5) * dxl
    gy = lo[1] + (gj.ravel() + 0.5) * dyl
    keep = np.hypot(gx - s.cyl_x, gy - s.cyl_y) >= r_outer + 0.25 * dyl
    xs.append(gx[keep]); ys.append(gy[keep]); dss.append(np.full(int(keep.sum()), math.sqrt(dxl * dyl)))
    x = np.concatenate(xs); y = np.concatenate(ys); ds = np.concatenate(dss)
    x = x + rng.uniform(-s.jitter, s.jitter, x.size) * ds
    y = y + rng.uniform(-s.jitter, s.jitter, y.size) * ds
    inside = (x >= lo[0]) & (x < hi[0]) & (y >= lo[1]) & (y < hi[1])
    x, y, ds = x[inside], y[inside], ds[inside]

    u, v, p = _potential_flow(s, x, y)
    return _assemble_channel(s, rng, x, y, ds, u, v, p, lev_ds, nlev, slope, lo, hi)


def _potential_flow(s, x, y):
    """Potential flow past the cylinder, pressure from Bernoulli."""
    X, Y = x - s.cyl_x, y - s.cyl_y
    r2 = X * X + Y * Y
    R2 = (0.5 * s.diameter) ** 2
    u = s.u_inf * (1.0 - R2 * (X * X - Y * Y) / (r2 * r2))
    v = -s.u_inf * 2.0 * R2 * X * Y / (r2 * r2)
    p = 0.5 * s.rho0 * (s.u_inf ** 2 - (u * u + v * v))
    return u, v, p


def _assemble_channel(s, rng, x, y, ds, u, v, p, lev_ds, nlev, slope, lo, hi):
    """Adds the inlet and outlet columns and the solid layers of the
    cylinder to graded fluid particles (x, y, spacing ds, fields u, v, p)
    and returns the state dict of a channel workload."""
    R = 0.5 * s.diameter
    ds_max = s.ds_min * s.ratio

    # inlet buffer columns left of x = 0 (prescribed u_inf) and outlet
    # columns right of x = length, each a lattice at the graded spacing the
    # fluid has where the zone meets it (the spacing level of s(d) at the
    # point of the boundary closest to the cylinder)
    def zone_ds(d):
        target = min(s.ds_min + d * slope, ds_max)
        k = int(np.searchsorted(lev_ds, target * (1 + 1e-12), side="right") - 1)
        return float(lev_ds[max(0, min(k, nlev))])
    zx, zy, zk, zd = [], [], [], []
    for side, kd in ((-1, INLET), (1, OUTLET)):
        if s.io_layers <= 0:
            continue
        edge = lo[0] if side < 0 else hi[0]
        dsz = zone_ds(abs(edge - s.cyl_x) - R)
        nyz = max(int(round(s.height / dsz)), 1)
        dyz = s.height / nyz
        cols = np.arange(s.io_layers)
        ci, cj = np.meshgrid(cols, np.arange(nyz), indexing="ij")
        cx = edge + side * (ci.ravel() + 0.5) * dyz
        cy = lo[1] + (cj.ravel() + 0.5) * dyz
        cx = cx + rng.uniform(-s.jitter, s.jitter, cx.size) * dyz
        cy = cy + rng.uniform(-s.jitter, s.jitter, cy.size) * dyz
        zx.append(cx); zy.append(cy); zk.append(np.full(cx.size, kd, np.int32))
        zd.append(np.full(cx.size, dyz))
        if side < 0:
            len_in = s.io_layers * dyz
        else:
            len_out = s.io_layers * dyz
    if zx:
        zx = np.concatenate(zx); zy = np.concatenate(zy); zk = np.concatenate(zk); zd = np.concatenate(zd)
    else:
        zx = zy = zd = np.zeros(0); zk = np.zeros(0, np.int32)
        len_in = len_out = 0.0
    nz = zx.size
    x = np.concatenate([x, zx]); y = np.concatenate([y, zy]); ds = np.concatenate([ds, zd])
    u = np.concatenate([u, np.full(nz, s.u_inf)]); v = np.concatenate([v, np.zeros(nz)])
    p = np.concatenate([p, np.zeros(nz)])
    kind_f = np.concatenate([np.zeros(x.size - nz, np.int32), zk])

    # solid dummy layers inside the cylinder at ds_min
    sx, sy = [], []
    for L in range(s.wall_layers):
        rr = R - (L + 0.5) * s.ds_min
        if rr <= 0:
            break
        px, py = _ring_points(rng, rr, s.ds_min, s.cyl_x, s.cyl_y)
        sx.append(px); sy.append(py)
    sx = np.concatenate(sx); sy = np.concatenate(sy)
    nf, ns = x.size, sx.size

    m_f = s.rho0 * ds * ds
    m_s = np.full(ns, s.rho0 * s.ds_min ** 2)
    q = mass_quantum(1.05 * s.rho0 * ds_max ** 2 * 1.5)
    allm = np.concatenate([m_f, m_s])
    mq = quantize_mass(allm, q)
    X = np.concatenate([x, sx]); Yv = np.concatenate([y, sy])
    H = np.concatenate([s.hdx * ds, np.full(ns, s.hdx * s.ds_min)])
    U = np.concatenate([u, np.zeros(ns)]); V = np.concatenate([v, np.zeros(ns)])
    P = np.concatenate([p, np.zeros(ns)])
    kind = np.concatenate([kind_f, np.full(ns, SOLID, np.int32)])
    nu = s.u_inf * s.diameter / s.re
    return {
        "x": X, "y": Yv, "u": U, "v": V, "p": P, "h": H, "mq": mq, "mass_q": q,
        "m": mq.astype(np.float64) * q, "rho": np.full(X.size, s.rho0),
        "mref": np.concatenate([m_f, m_s]), "kind": kind, "n_fluid": int((kind == FLUID).sum()), "n_solid": ns,
        "domain": Domain((lo[0] - len_in - 2 * s.ds_min * s.ratio, lo[1]),
                         (hi[0] + len_out + 2 * s.ds_min * s.ratio, hi[1]), (False, True)),
        "io": {"x_in": lo[0], "len_in": len_in, "x_out": hi[0], "len_out": len_out},
        "params": {"rho0": s.rho0, "cs": s.cs, "nu": nu, "hdx": s.hdx, "re": s.re,
                   "u_inf": s.u_inf, "io_mode": 1, "io_ref": (s.u_inf, 0.0, 0.0)},
        "h_min": s.hdx * s.ds_min, "u_ref": s.u_inf, "spec": s,
    }


def channel_wake(spec: ChannelSpec | None = None, seed: int = 2, wake=(10.5, 18.5, 0.6),
                 vortices: int = 8, gamma: float = 2.0, core: float = 0.2):
    """The channel after its wake has been refined by the vorticity criterion
    (the 1:250, Re = 1000 channel): the target size is graded by the
    distance d to the nearer of the cylinder and the wake band
    [x0, x1] x [-w, w], s(d) = ds_min + d ln(C_r)/rows_per_layer (capped at
    ds_max), snapped to the levels ds_min 2^(k/2).  Each level fills the
    points where it is the snapped size with a lattice of its spacing
    (jittered by U(-jitter, jitter) of it), which leaves seams of at most one
    spacing between levels.  The velocity is the potential flow plus a
    street of `vortices` Lamb-Oseen vortices of alternating sign along the
    band (circulation gamma, core radius `core`, at y = +-0.3, one D apart),
    so that |vorticity| peaks in the wake.  Inlet, outlet and solids as in
    `channel_cylinder`."""
    s = spec or ChannelSpec(ds_min=1.0 / 250.0, ratio=250, re=1000.0)
    rng = np.random.default_rng(seed)
    R = 0.5 * s.diameter
    ds_max = s.ds_min * s.ratio
    nlev = int(math.floor(2 * math.log2(s.ratio) + 1e-9))
    lev_ds = s.ds_min * np.sqrt(2.0) ** np.arange(nlev + 1)
    lo = (0.0, s.cyl_y - 0.5 * s.height)
    hi = (s.length, s.cyl_y + 0.5 * s.height)
    slope = math.log(s.cr) / s.rows_per_layer
    x0, x1, w = wake

    def dist(px, py):
        dc = np.maximum(np.hypot(px - s.cyl_x, py - s.cyl_y) - R, 0.0)
        dwx = np.maximum(np.maximum(x0 - px, px - x1), 0.0)
        dwy = np.maximum(np.abs(py - s.cyl_y) - w, 0.0)
        return np.minimum(dc, np.hypot(dwx, dwy))

    def level(px, py):
        target = np.minimum(s.ds_min + dist(px, py) * slope, ds_max)
        k = np.floor(np.log(target * (1 + 1e-12) / s.ds_min) / math.log(math.sqrt(2.0)))
        return np.clip(k, 0, nlev).astype(np.int64)

    xs, ys, dss = [], [], []
    for k in range(nlev + 1):
        a = float(lev_ds[k])
        reach = (float(lev_ds[k + 1]) - s.ds_min) / slope if k < nlev else math.inf
        bx0 = max(lo[0], min(s.cyl_x - R, x0) - reach)
        bx1 = min(hi[0], max(s.cyl_x + R, x1) + reach)
        by0 = max(lo[1], s.cyl_y - max(R, w) - reach)
        by1 = min(hi[1], s.cyl_y + max(R, w) + reach)
        i0, i1 = int(math.floor((bx0 - lo[0]) / a)), int(math.ceil((bx1 - lo[0]) / a))
        j0, j1 = int(math.floor((by0 - lo[1]) / a)), int(math.ceil((by1 - lo[1]) / a))
        gi, gj = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1), indexing="ij")
        px = lo[0] + (gi.ravel() + 0.5) * a
        py = lo[1] + (gj.ravel() + 0.5) * a
        keep = (level(px, py) == k) & (np.hypot(px - s.cyl_x, py - s.cyl_y) >= R + 0.5 * s.ds_min)
        keep &= (px >= lo[0]) & (px < hi[0]) & (py >= lo[1]) & (py < hi[1])
        xs.append(px[keep]); ys.append(py[keep]); dss.append(np.full(int(keep.sum()), a))
    x = np.concatenate(xs); y = np.concatenate(ys); ds = np.concatenate(dss)
    x = x + rng.uniform(-s.jitter, s.jitter, x.size) * ds
    y = y + rng.uniform(-s.jitter, s.jitter, y.size) * ds
    inside = (x >= lo[0]) & (x < hi[0]) & (y >= lo[1]) & (y < hi[1])
    x, y, ds = x[inside], y[inside], ds[inside]
    u, v, p = _potential_flow(s, x, y)
    for n in range(vortices):
        vx = x0 + 0.5 + n * 1.0
        vy = s.cyl_y + (0.3 if n % 2 == 0 else -0.3)
        g = gamma if n % 2 == 0 else -gamma
        X, Y = x - vx, y - vy
        r2 = np.maximum(X * X + Y * Y, 1e-300)
        ut = g / (2 * math.pi * r2) * (1.0 - np.exp(-r2 / (core * core)))
        u += -ut * Y
        v += ut * X
    return _assemble_channel(s, rng, x, y, ds, u, v, p, lev_ds, nlev, slope, lo, hi)


def oscillating_cylinder(spec: ChannelSpec | None = None, seed: int = 2, amp: float = 0.5,
                         period: float = 5.0):
    """The channel with a cylinder oscillating across the stream,
    y_c(t) = amp D sin(2 pi t / period), at t = 0: 1:100, Re = 200, D/400,
    refined to ds_min over the band the body sweeps
    ([x_c - 0.6 D, x_c + 0.6 D] x [-(amp + 0.6) D, (amp + 0.6) D]) and graded
    around it as `channel_wake` grades (no vortex street).  `motion` holds
    the amplitude and period for `body_motion`."""
    s = spec or ChannelSpec(ds_min=1.0 / 400.0, ratio=100, re=200.0)
    D = s.diameter
    st = channel_wake(s, seed, wake=(s.cyl_x - 0.6 * D, s.cyl_x + 0.6 * D, (amp + 0.6) * D),
                      vortices=0)
    st["motion"] = {"amp": amp * D, "period": period}
    return st


def body_motion(t: float, amp: float, period: float):
    """Transverse position, velocity and acceleration of the oscillating
    body at time t."""
    w = 2.0 * math.pi / period
    return amp * math.sin(w * t), amp * w * math.cos(w * t), -amp * w * w * math.sin(w * t)


def channel_background(spec: ChannelSpec | None = None, seed: int = 3, sparsity: float = 2.0):
    """Background particles for the channel, prescribed from the grading
    recipe of `channel_cylinder` (section 3.3 allows the reference mass to be
    assigned directly; for a stationary body the background is never
    updated).  Rings around the cylinder at spacing `sparsity` * s(d), with
    size ds = s(d) (the continuous target size), m_ref = rho0 ds^2 and
    h = 1.3 * sparsity * s(d) (about N_r = 48 neighbours)."""
    s = spec or ChannelSpec()
    rng = np.random.default_rng(seed)
    R = 0.5 * s.diameter
    ds_max = s.ds_min * s.ratio
    slope = math.log(s.cr) / s.rows_per_layer
    lo = (0.0, s.cyl_y - 0.5 * s.height)
    hi = (s.length, s.cyl_y + 0.5 * s.height)
    rmax = math.hypot(max(s.cyl_x - lo[0], hi[0] - s.cyl_x), 0.5 * s.height) + ds_max
    xs, ys, dss = [], [], []
    r = R
    while r < rmax:
        size = min(s.ds_min + (r - R) * slope, ds_max)
        step = sparsity * size
        px, py = _ring_points(rng, r, step, s.cyl_x, s.cyl_y)
        xs.append(px); ys.append(py); dss.append(np.full(px.size, size))
        r += step
    x = np.concatenate(xs); y = np.concatenate(ys); ds = np.concatenate(dss)
    keep = (x >= lo[0]) & (x < hi[0]) & (y >= lo[1]) & (y < hi[1])
    x, y, ds = x[keep], y[keep], ds[keep]
    m = s.rho0 * ds * ds
    q = mass_quantum(1.05 * s.rho0 * ds_max ** 2 * 1.5)
    return {"x": x, "y": y, "h": 1.3 * sparsity * ds, "ds": ds,
            "mask": (ds <= s.ds_min * (1 + 1e-12)).astype(np.int32),
            "mq": quantize_mass(m, q), "mass_q": q, "mref": m}


FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3


def wall_box(nx: int = 20, ny: int = 20, layers: int = 3, jitter: float = 0.0, seed: int = 5,
             hdx: float = 1.2, rho0: float = 1.0, top: bool = True):
    """Fluid on [0, 1) x [0, ny/nx) (periodic in x, open in y) between
    `layers` rows of wall particles below (and above when `top`), all on one
    lattice of spacing 1/nx; fluid positions jittered by U(-j, j) dx."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / nx
    H = ny * dx
    j_lo = -layers
    j_hi = ny + (layers if top else 0)
    i, j = np.meshgrid(np.arange(nx), np.arange(j_lo, j_hi), indexing="ij")
    i, j = i.ravel(), j.ravel()
    x = (i + 0.5) * dx
    y = (j + 0.5) * dx
    kind = np.where((j < 0) | (j >= ny), SOLID, FLUID).astype(np.int32)
    fl = kind == FLUID
    if jitter > 0:
        x[fl] = np.mod(x[fl] + rng.uniform(-jitter, jitter, fl.sum()) * dx, 1.0)
        y[fl] = y[fl] + rng.uniform(-jitter, jitter, fl.sum()) * dx
    n = x.size
    m = np.full(n, rho0 * dx * dx)
    q = mass_quantum(1.05 * m.max() * 1.5)
    dom = Domain((0.0, -(layers + 1) * dx), (1.0, H + (layers + 1) * dx), (True, False))
    return {"x": x, "y": y, "u": np.zeros(n), "v": np.zeros(n), "p": np.zeros(n),
            "rho": np.full(n, rho0), "h": np.full(n, hdx * dx), "m": m,
            "mq": quantize_mass(m, q), "mass_q": q, "mref": m.copy(), "kind": kind,
            "domain": dom, "dx": dx, "H": H}


def inout_strip(nx: int = 30, ny: int = 10, n_in: int = 4, n_out: int = 4, U: float = 1.0,
                seed: int = 6, jitter: float = 0.0, hdx: float = 1.2, rho0: float = 1.0):
    """A channel strip periodic in y: inlet particles on x in [-n_in dx, 0),
    fluid on [0, L), outlet particles on [L, L + n_out dx), L = nx dx,
    dx = 1/ny; uniform velocity (U, 0)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / ny
    i, j = np.meshgrid(np.arange(-n_in, nx + n_out), np.arange(ny), indexing="ij")
    i, j = i.ravel(), j.ravel()
    x = (i + 0.5) * dx
    y = (j + 0.5) * dx
    if jitter > 0:
        x = x + rng.uniform(-jitter, jitter, x.size) * dx
        y = np.mod(y + rng.uniform(-jitter, jitter, y.size) * dx, 1.0)
    L = nx * dx
    kind = np.where(x < 0.0, INLET, np.where(x >= L, OUTLET, FLUID)).astype(np.int32)
    n = x.size
    m = np.full(n, rho0 * dx * dx)
    q = mass_quantum(1.05 * m.max() * 1.5)
    dom = Domain((-(n_in + 2) * dx, 0.0), (L + (n_out + 2) * dx, 1.0), (False, True))
    io = {"x_in": 0.0, "len_in": n_in * dx, "x_out": L, "len_out": n_out * dx}
    return {"x": x, "y": y, "u": np.full(n, U), "v": np.zeros(n), "p": np.zeros(n),
            "rho": np.full(n, rho0), "h": np.full(n, hdx * dx), "m": m,
            "mq": quantize_mass(m, q), "mass_q": q, "mref": m.copy(), "kind": kind,
            "domain": dom, "dx": dx, "io": io}


def background_lattice(domain: Domain, ds_max: float, hdx: float, rho0: float,
                       seed: int = 0, jitter: float = 0.0):
    """Background particles at the coarsest size ds_max (section 3.3)."""
    rng = np.random.default_rng(seed)
    Lx = domain.hi[0] - domain.lo[0]
    Ly = domain.hi[1] - domain.lo[1]
    nx = max(int(round(Lx / ds_max)), 1)
    ny = max(int(round(Ly / ds_max)), 1)
    gi, gj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = domain.lo[0] + (gi.ravel() + 0.5) * (Lx / nx)
    y = domain.lo[1] + (gj.ravel() + 0.5) * (Ly / ny)
    if jitter > 0:
        x = x + rng.uniform(-jitter, jitter, x.size) * ds_max
        y = y + rng.uniform(-jitter, jitter, y.size) * ds_max
    n = x.size
    m = rho0 * ds_max * ds_max
    q = mass_quantum(1.05 * m * 1.5)
    return {"x": x, "y": y, "h": np.full(n, hdx * ds_max), "ds": np.full(n, ds_max),
            "mask": np.zeros(n, np.int32), "mq": np.full(n, int(round(m / q)), np.int64),
            "mass_q": q, "mref": np.full(n, m)}


def square_solid(cx: float, cy: float, side: float, ds: float, hdx: float, layers: int = 3):
    """A square solid body discretised at spacing ds (section 3.3 example)."""
    xs, ys = [], []
    n = max(int(round(side / ds)), 1)
    for L in range(layers):
        a = side / 2 - (L + 0.5) * ds
        if a <= 0:
            break
        m = max(int(round(2 * a / ds)), 1)
        t = np.linspace(-a, a, m + 1)
        xs += [cx + t, cx + t, np.full(m + 1, cx - a), np.full(m + 1, cx + a)]
        ys += [np.full(m + 1, cy - a), np.full(m + 1, cy + a), cy + t, cy + t]
    x = np.concatenate(xs); y = np.concatenate(ys)
    pts = np.unique(np.round(np.stack([x, y], 1), 12), axis=0)
    del n
    return {"x": pts[:, 0].copy(), "y": pts[:, 1].copy(), "h": np.full(len(pts), hdx * ds)}


def region_markers(lo, hi, ds: float, hdx: float = 1.0):
    """A user-defined refinement region (section 3.3): marker particles on a
    lattice of spacing ds filling the rectangle [lo, hi], handed to the
    background update as a solid body.  They only mark the background
    particles near them and take no part in the flow."""
    nx = max(int(round((hi[0] - lo[0]) / ds)), 1)
    ny = max(int(round((hi[1] - lo[1]) / ds)), 1)
    gi, gj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = lo[0] + (gi.ravel() + 0.5) * (hi[0] - lo[0]) / nx
    y = lo[1] + (gj.ravel() + 0.5) * (hi[1] - lo[1]) / ny
    return {"x": x.astype(np.float64), "y": y.astype(np.float64), "h": np.full(x.size, hdx * ds)}


def tgv_zone(nx: int = 50, re: float = 200.0, zone=((0.1, 0.1), (0.5, 0.5)), ratio: float = 2.0,
             cr: float = 1.2, cs: float = 10.0, rho0: float = 1.0):
    """Taylor-Green vortex with an inner refinement zone (section 4.1): the
    fluid starts on the plain nx*nx lattice (dx_max = 1/nx, h = dx) with the
    exact fields; the background starts as a lattice at dx_max over the
    periodic square, and marker particles filling the zone at dx_max/ratio
    ask for ds_min = dx_max/ratio there.  `bg_params` holds C_r, ds_min and
    ds_max."""
    s = tgv(nx, jitter=0.0, perturb=False, re=re, cs=cs, rho0=rho0)
    dx = 1.0 / nx
    s["background"] = background_lattice(s["domain"], dx, 1.2, rho0)
    s["markers"] = region_markers(zone[0], zone[1], dx / ratio)
    s["zone"] = zone
    s["bg_params"] = {"cr": cr, "ds_min": dx / ratio, "ds_max": dx}
    return s


def two_squares(t: float, gap: float = 3.0, side: float = 1.0, ds: float = 0.1, speed: float = 1.0,
                hdx: float = 1.2):
    """The two square bodies of the moving-geometry example of section 3.3 at
    time t: unit squares centred at (-(gap/2 + speed t), 0) and
    (gap/2 + speed t, 0), each moving away from the other."""
    off = 0.5 * gap + speed * t
    a = square_solid(-off, 0.0, side, ds, hdx)
    b = square_solid(off, 0.0, side, ds, hdx)
    return {k: np.concatenate([a[k], b[k]]) for k in ("x", "y", "h")}


# ---------------------------------------------------------------------------
# Serving mix: independent periodic vortex instances
# ---------------------------------------------------------------------------

def serving_requests(n_req: int = 256, seed: int = 4, n_lo: int = 2000, n_hi: int = 200000,
                     re_lo: float = 100.0, re_hi: float = 1000.0, rate: float = 1.0):
    """Request specs: particle count log-uniform in [n_lo, n_hi] (lattice side
    ceil(sqrt N)), Re uniform in [re_lo, re_hi], Poisson arrival times at
    `rate` requests per unit time."""
    rng = np.random.default_rng(seed)
    N = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_req))).astype(np.int64)
    side = np.ceil(np.sqrt(N)).astype(np.int64)
    re = rng.uniform(re_lo, re_hi, n_req)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    seeds = rng.integers(1, 2 ** 31 - 1, n_req)
    return [{"side": int(side[k]), "re": float(re[k]), "arrival": float(arrivals[k]),
             "seed": int(seeds[k])} for k in range(n_req)]
