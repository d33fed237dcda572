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
