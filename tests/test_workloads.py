"""Host-side checks of the seeded input generators (no method arithmetic)."""
import numpy as np

import workloads as W


def test_channel_background_grading():
    spec = W.ChannelSpec()
    bg = W.channel_background(spec, seed=3)
    x, y, ds = bg["x"], bg["y"], bg["ds"]
    assert x.size > 1000
    # inside the channel
    assert x.min() >= 0 and x.max() < spec.length
    assert y.min() >= spec.cyl_y - spec.height / 2 and y.max() < spec.cyl_y + spec.height / 2
    # sizes graded between the finest spacing and the 1:ratio cap
    assert ds.min() >= spec.ds_min * (1 - 1e-12)
    assert ds.max() <= spec.ds_min * spec.ratio * (1 + 1e-12)
    # the size grows with distance from the cylinder (monotone by construction)
    d = np.hypot(x - spec.cyl_x, y - spec.cyl_y) - spec.diameter / 2
    order = np.argsort(d)
    assert np.all(np.diff(ds[order]) >= -1e-15)
    # reference mass on the integer ledger: |mq q - rho0 ds^2| within half a quantum
    q = bg["mass_q"]
    assert np.all(np.abs(bg["mq"] * q - spec.rho0 * ds * ds) <= 0.5 * q + 1e-18)
    # only the finest layer is masked
    assert np.array_equal(bg["mask"] == 1, ds <= spec.ds_min * (1 + 1e-12))
    assert bg["mask"].sum() > 0


def test_channel_background_seeded():
    a = W.channel_background(seed=3)
    b = W.channel_background(seed=3)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])


def test_channel_wake_levels_and_band():
    """The wake-refined channel (small spec): spacings on the sqrt(2)
    levels, the finest level fills the wake band, sizes grow away from it,
    no fluid inside the cylinder, and a ratio that is not a power of two
    is generated (its ring grading stops at the cap)."""
    import math
    spec = W.ChannelSpec(length=6.0, height=4.0, cyl_x=2.0, ds_min=0.02, ratio=25, re=1000.0,
                         io_layers=2)
    s = W.channel_wake(spec, wake=(2.5, 4.5, 0.4), vortices=3)
    fl = s["kind"] == W.FLUID
    ds = s["h"][fl] / spec.hdx
    lev = np.log(ds / spec.ds_min) / math.log(math.sqrt(2.0))
    assert np.allclose(lev, np.round(lev), atol=1e-9) and lev.max() <= 2 * math.log2(25)
    x, y = s["x"][fl], s["y"][fl]
    band = (x > 2.6) & (x < 4.4) & (np.abs(y) < 0.3)
    assert band.sum() > 0 and np.all(ds[band] == spec.ds_min)
    assert np.corrcoef(np.abs(y[x > 5.0]), ds[x > 5.0])[0, 1] > 0.5
    assert np.all(np.hypot(x - spec.cyl_x, y - spec.cyl_y) > 0.5)
    assert s["n_solid"] > 0 and (s["kind"] == W.INLET).sum() > 0
    c = W.channel_cylinder(W.ChannelSpec(length=6.0, height=4.0, cyl_x=2.0, ds_min=0.02,
                                         ratio=25), seed=2)
    assert c["x"].size > 0


def test_body_motion():
    """y = A sin(wt): velocity and acceleration are its derivatives."""
    import math
    A, T = 0.5, 5.0
    for t in (0.0, 0.7, 1.25, 3.1):
        y, v, a = W.body_motion(t, A, T)
        e = 1e-6
        yp, vp, _ = W.body_motion(t + e, A, T)
        ym, vm, _ = W.body_motion(t - e, A, T)
        assert abs((yp - ym) / (2 * e) - v) < 1e-8 and abs((vp - vm) / (2 * e) - a) < 1e-7
        assert abs(y - A * math.sin(2 * math.pi * t / T)) < 1e-15


def test_mass_ledgers_fit_int64():
    """Every workload's ledger total, summed exactly with Python integers,
    stays below 2^63 (the diagnostics sum it in checked int64) and equals
    numpy's int64 sum (which would wrap silently otherwise)."""
    cases = [W.tgv(50, seed=1), W.channel_cylinder(seed=2), W.channel_wake(),
             W.oscillating_cylinder(), W.gresho_chan(80)]
    for s in cases:
        mq = s["mq"]
        exact = sum(int(v) for v in mq.tolist())
        assert 0 < exact < 2 ** 63
        assert exact == int(mq.sum(dtype=np.int64))
        assert int(mq.max()) < 2 ** 53
