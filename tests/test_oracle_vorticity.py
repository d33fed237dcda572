"""Pins of the oracle's vorticity (section 3.3, solution adaptivity): the
first-order difference SPH curl returns 2 Omega for a rigid rotation (a
linear field, exact up to the lattice sum of the kernel gradient) and the
Taylor-Green vorticity 4 pi cos(2 pi x) cos(2 pi y) to second order in h."""
import numpy as np

import workloads as W


def test_vorticity_rigid_rotation(orc):
    n = 40
    dx = 1.0 / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = (i.ravel() + 0.5) * dx
    y = (j.ravel() + 0.5) * dx
    h = np.full(x.size, 1.2 * dx)
    m = np.full(x.size, dx * dx)
    rho = np.ones(x.size)
    Om = 0.8
    u, v = -Om * (y - 0.5), Om * (x - 0.5)
    dom = orc.Dom((0.0, 0.0), (1.0, 1.0), (False, False))
    rp, col = orc.neighbors(dom, x, y, h)
    w = orc.vorticity(dom, x, y, u, v, h, m, rho, rp, col)
    inner = (np.abs(x - 0.5) < 0.3) & (np.abs(y - 0.5) < 0.3)
    np.testing.assert_allclose(w[inner], 2 * Om, rtol=2e-3)
    # a uniform translation has none
    w0 = orc.vorticity(dom, x, y, np.full(x.size, 0.3), np.full(x.size, -0.1), h, m, rho, rp, col)
    assert np.max(np.abs(w0)) < 1e-12


def test_vorticity_taylor_green(orc):
    s = W.tgv(nx=50, seed=1, jitter=0.0, hdx=1.0)
    dom = orc.Dom()
    rho = np.ones(s["x"].size)
    rp, col = orc.neighbors(dom, s["x"], s["y"], s["h"])
    w = orc.vorticity(dom, s["x"], s["y"], s["u"], s["v"], s["h"], s["m"], rho, rp, col)
    ref = 4 * np.pi * np.cos(2 * np.pi * s["x"]) * np.cos(2 * np.pi * s["y"])
    assert np.max(np.abs(w - ref)) < 0.02 * 4 * np.pi
    # the sign convention: omega = dv/dx - du/dy
    assert np.corrcoef(w, ref)[0, 1] > 0.999


def _lattice(n, L=1.0):
    dx = L / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return (i.ravel() + 0.5) * dx, (j.ravel() + 0.5) * dx, dx


def test_shepard_to_bg_constant_and_linear(orc):
    # Shepard weights sum to one: a constant is carried exactly; a linear
    # field is exact wherever the weights are symmetric about the point
    # (lattice sites and cell centres far from the edges)
    x, y, dx = _lattice(40)
    h = np.full(x.size, 1.2 * dx)
    dom = orc.Dom((0.0, 0.0), (1.0, 1.0), (False, False))
    bx = np.array([0.5, 0.5 + 0.5 * dx, 20.5 * dx, 0.3 - 0.5 * dx + dx * 0.0])
    by = np.array([0.5, 0.5 + 0.5 * dx, 14.5 * dx, 0.3])
    bx[3], by[3] = 12.5 * dx, 12.0 * dx          # cell-edge midpoint: symmetric too
    bh = np.array([2.5 * dx, 3.1 * dx, 1.2 * dx, 2.0 * dx])
    c = orc.shepard_to_bg(dom, bx, by, bh, x, y, h, np.full(x.size, 2.75))
    np.testing.assert_allclose(c, 2.75, rtol=1e-14)
    f = 3.0 * x - 1.5 * y + 0.25
    phi = orc.shepard_to_bg(dom, bx, by, bh, x, y, h, f)
    np.testing.assert_allclose(phi, 3.0 * bx - 1.5 * by + 0.25, rtol=0, atol=1e-13)
    # near an open edge the weights are one-sided and the average is biased
    e = orc.shepard_to_bg(dom, np.array([0.25 * dx]), np.array([0.5]), np.array([2 * dx]), x, y, h, f)
    assert abs(e[0] - (3.0 * 0.25 * dx - 1.5 * 0.5 + 0.25)) > 0.1 * dx
    # kind filter: non-fluid particles do not contribute; none in range gives 0
    kind = np.where(x > 0.5, 1, 0).astype(np.int32)
    g = orc.shepard_to_bg(dom, np.array([0.9]), np.array([0.5]), np.array([1.5 * dx]), x, y, h,
                          np.ones(x.size), kind)
    assert g[0] == 0.0


def test_solution_mark_lasts_the_update(orc):
    # one background particle marked by phi: it and its split children end at
    # ds_min with mask 3 after several passes; the sizes around are graded by
    # C_r; the same update without phi marks nothing and stays coarse
    dom = W.Domain((0.0, 0.0), (1.0, 1.0), (True, True))
    bg = W.background_lattice(dom, 0.1, 1.2, 1.0)
    phi = np.zeros(bg["x"].size)
    k = int(np.argmin(np.hypot(bg["x"] - 0.55, bg["y"] - 0.55)))
    phi[k] = 1.0
    bp = orc.BgPrm(cr=1.2, ds_min=0.025, ds_max=0.1, mass_q=bg["mass_q"])
    empty = {"x": np.zeros(0), "y": np.zeros(0), "h": np.zeros(0)}
    ob, ns = orc.bg_update(orc.Dom((0, 0), (1, 1), (True, True)), bp, bg, empty, 8, cap=40000,
                           phi=phi, phi_thresh=0.5)
    marked = ob["mask"] == 3
    assert marked.sum() >= 7 and ns > 0
    assert np.all(ob["ds"][marked] == 0.025)
    assert set(np.unique(ob["mask"])) <= {0, 3}
    # graded away from the marked spot: the size grows with distance
    d = np.hypot(ob["x"] - bg["x"][k], ob["y"] - bg["y"][k])
    far = d > 0.35
    assert ob["ds"][far].min() > ob["ds"][marked].max()
    ob2, ns2 = orc.bg_update(orc.Dom((0, 0), (1, 1), (True, True)), bp, bg, empty, 8, cap=40000)
    assert ns2 == 0 and np.all(ob2["mask"] == 0) and np.all(ob2["ds"] == 0.1)
