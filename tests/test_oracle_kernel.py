"""Pins of the oracle's quintic spline kernel (eq. kernel, section 2) and the
time step (eq. timestep) against closed forms and printed values."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize


def test_normalisation(orc):
    # A smoothing kernel integrates to one over its support in 2D.
    for h in (0.3, 1.0, 1.7):
        tot = 0.0
        for a, b in ((0, h), (h, 2 * h), (2 * h, 3 * h)):
            val, _ = integrate.quad(lambda r: 2 * math.pi * r * orc.w(r, h), a, b,
                                    epsabs=1e-14, epsrel=1e-13, limit=200)
            tot += val
        assert abs(tot - 1.0) < 1e-12


def test_value_at_origin(orc):
    # f(0) = 3^5 - 6*2^5 + 15 = 66, so W(0,1) = 66 * 7 / (478 pi).
    assert orc.kf(0.0) == 66.0
    assert orc.w(0.0, 1.0) == pytest.approx(66 * 7 / (478 * math.pi), rel=1e-15)
    assert orc.w(0.0, 1.0) == pytest.approx(0.3076551619600655, rel=1e-15)


def test_compact_support_and_continuity(orc):
    for q in (3.0, 3.5, 10.0):
        assert orc.kf(q) == 0.0 and orc.kfp(q) == 0.0
    eps = 1e-9
    for q in (1.0, 2.0, 3.0):
        assert abs(orc.kf(q - eps) - orc.kf(q + eps)) < 1e-6
        assert abs(orc.kfp(q - eps) - orc.kfp(q + eps)) < 1e-6
    # each piece drops exactly the term that vanishes at its breakpoint
    assert orc.kf(1.0) == 2 ** 5 - 6 * 1 ** 5
    assert orc.kf(2.0) == 1.0


def test_derivative_matches_function(orc):
    d = 1e-6
    for q in np.linspace(0.05, 2.95, 59):
        num = (orc.kf(q + d) - orc.kf(q - d)) / (2 * d)
        assert orc.kfp(q) == pytest.approx(num, rel=1e-7, abs=1e-7)
    for h in (0.01, 0.5):
        for r in np.linspace(0.02, 2.9, 12) * h:
            dd = 1e-7 * h
            num = (orc.w(r + dd, h) - orc.w(r - dd, h)) / (2 * dd)
            assert orc.dwdr(r, h) == pytest.approx(num, rel=1e-6)


def test_scaling_in_h(orc):
    for h in (0.01, 0.37, 2.0):
        for q in (0.0, 0.4, 1.3, 2.6):
            assert orc.w(q * h, h) == pytest.approx(orc.w(q, 1.0) / h ** 2, rel=1e-14)
            assert orc.dwdr(q * h, h) == pytest.approx(orc.dwdr(q, 1.0) / h ** 3, rel=1e-14)


def test_inflection_point_printed(orc):
    # Section 2.1 prints the inflection point of the quintic spline,
    # xi = 0.759298480738450; it is the zero of f'' on (0, 1).
    d = 1e-5
    fpp = lambda q: (orc.kfp(q + d) - orc.kfp(q - d)) / (2 * d)
    root = optimize.brentq(fpp, 0.5, 0.95, xtol=1e-14)
    assert abs(root - 0.759298480738450) < 1e-8


def test_timestep_printed_table(orc):
    # Table fpc-perf prints dt = 0.0011, 0.00055, 0.00027 for D/dx_min =
    # 50, 100, 200 with D = 2, h/dx = 1.2, U = 1, c_s = 10, Re = 3000.
    D, U, cs, re = 2.0, 1.0, 10.0, 3000.0
    nu = U * D / re
    for ratio, printed in ((50, 0.0011), (100, 0.00055), (200, 0.00027)):
        dt = orc.timestep(1.2 * D / ratio, U, cs, nu)
        assert float(f"{dt:.2g}") == printed
    # config of the periodic vortex: h = dx = 1/50, c_s = 10, Re = 100
    assert orc.timestep(0.02, 1.0, 10.0, 0.01) == pytest.approx(0.25 * 0.02 / 11.0, rel=1e-15)
