"""Pin of the oracle's pass B on the Gresho-Chan vortex (section 4.2): at
the exact steady state the inviscid momentum rate is the centripetal
acceleration -u_phi^2 / r (the pressure gradient that balances the
centrifugal force).  On the uniform start lattice the relative L1 error of
the SPH rate converges at second order in the spacing (3.2% at 40^2
particles, 0.85% at 80^2)."""
import numpy as np

import oracle
import workloads as W
from gpu_util import odom


def _rel_err(nx):
    s = W.gresho_chan(nx)
    prm = oracle.Prm(rho0=1.0, cs=10.0, nu=0.0, hdx=1.0, mass_q=s["mass_q"])
    o = oracle.rates(odom(s["domain"]), prm, s["x"], s["y"], s["u"], s["v"], s["p"], s["h"], s["m"],
                     oracle.dt_for(s))
    x, y = s["x"], s["y"]
    r2 = np.maximum(x * x + y * y, 1e-300)
    _, _, _, uphi = W.gresho_chan_fields(x, y)
    ax, ay = -uphi ** 2 * x / r2, -uphi ** 2 * y / r2
    err = np.abs(o["dudt"] - ax) + np.abs(o["dvdt"] - ay)
    return err.sum() / (np.abs(ax) + np.abs(ay)).sum()


def test_fields_are_the_closed_form():
    x = np.array([0.05, 0.0, 0.3, 0.45])
    y = np.array([0.0, 0.2 - 1e-12, 0.0, 0.1])
    u, v, p, uphi = W.gresho_chan_fields(x, y)
    assert np.allclose(uphi, [0.25, 1.0, 0.5, 0.0], atol=1e-10)
    # pressure continuous at r = R and r = 2R, constant outside
    R = W.GC_R
    for r0 in (R, 2 * R):
        _, _, pl, _ = W.gresho_chan_fields(np.array([r0 - 1e-9]), np.array([0.0]))
        _, _, pr, _ = W.gresho_chan_fields(np.array([r0 + 1e-9]), np.array([0.0]))
        assert abs(pl[0] - pr[0]) < 1e-7
    # dp/dr = u_phi^2 / r (rho0 = 1) by a central difference
    r = np.array([0.1, 0.3])
    dp = (W.gresho_chan_fields(r + 1e-6, 0 * r)[2] - W.gresho_chan_fields(r - 1e-6, 0 * r)[2]) / 2e-6
    up = W.gresho_chan_fields(r, 0 * r)[3]
    assert np.allclose(dp, up ** 2 / r, rtol=1e-6)


def test_rate_is_centripetal_second_order():
    e40, e80 = _rel_err(40), _rel_err(80)
    assert e40 < 0.04, e40
    assert e80 < 0.35 * e40, (e40, e80)
