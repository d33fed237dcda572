"""Pins of the oracle's force on solid particles (eq. force-sph, section 2.3)
against closed forms.

- Pressure: a circular body of dummy particles in fluid at rest with a
  linear pressure field p = G (x - x_c) feels -G times its area along x
  (the integral of -p n over its surface), and no lift.  The one-sided SPH
  sums converge to it at first order in the particle spacing.
- Viscous: fluid over a flat wall with the linear profile u = G y exerts the
  shear stress rho0 nu G on the wall, i.e. rho0 nu G L over a periodic length
  L.  On a lattice the discrete sum is a fixed fraction of it at every
  resolution (a moment of the kernel), within 1%.
"""
import math

import numpy as np

import oracle
import workloads as W
from gpu_util import odom


def _cylinder_in_gradient(ds, G):
    spec = W.ChannelSpec(length=4.0, height=4.0, cyl_x=2.0, ds_min=ds, ratio=8, io_layers=0,
                         jitter=0.0)
    s = dict(W.channel_cylinder(spec, seed=2))
    s["u"] = np.zeros_like(s["x"])
    s["v"] = np.zeros_like(s["x"])
    s["p"] = G * (s["x"] - spec.cyl_x)
    prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"], hdx=s["params"]["hdx"],
                     mass_q=s["mass_q"])
    return oracle.body_force(odom(s["domain"]), prm, s), math.pi * 0.25 * spec.diameter ** 2


def test_pressure_force_is_archimedes():
    G = 0.7
    errs = []
    for ds in (0.02, 0.01):
        f, area = _cylinder_in_gradient(ds, G)
        ratio = f["fp"][0] / (-G * area)
        errs.append(abs(ratio - 1.0))
        assert abs(ratio - 1.0) < 0.03, (ds, ratio)
        # no lift in a field that varies along x only (mirror symmetry, up
        # to the jitter-free lattice's rounding)
        assert abs(f["fp"][1]) < 1e-6 * f["abs_p"][1], (ds, f["fp"][1])
        assert f["fvisc"] == (0.0, 0.0)
    # first-order convergence: halving the spacing about halves the error
    assert errs[1] < 0.6 * errs[0], errs


def test_viscous_force_is_wall_shear():
    G, nu = 0.8, 0.05
    ratios = []
    for nx in (20, 40):
        s = dict(W.wall_box(nx=nx, ny=nx // 2, layers=3, top=False, hdx=1.2))
        fl = s["kind"] == W.FLUID
        s["u"] = np.where(fl, G * s["y"], 0.0)
        prm = oracle.Prm(rho0=1.0, cs=10.0, nu=nu, hdx=1.2, mass_q=s["mass_q"])
        f = oracle.body_force(odom(s["domain"]), prm, s)
        ratios.append(f["fvisc"][0] / (1.0 * nu * G * 1.0))
        assert abs(f["fvisc"][1]) < 1e-12 * f["abs_visc"][0]
        assert f["fp"] == (0.0, 0.0)          # p = 0 everywhere
    assert abs(ratios[0] - 1.0) < 0.01, ratios
    assert abs(ratios[0] - ratios[1]) < 1e-9, ratios


def test_force_coefficients():
    f = {"fp": (0.3, -0.1), "fvisc": (0.05, 0.0)}
    c = oracle.force_coefficients(f, rho0=1.0, U=2.0, L=0.5)
    q = 0.5 * 1.0 * 4.0 * 0.5
    assert c == {"cd_p": 0.3 / q, "cd_visc": 0.05 / q, "cl": -0.1 / q}
