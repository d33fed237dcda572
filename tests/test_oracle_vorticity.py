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
