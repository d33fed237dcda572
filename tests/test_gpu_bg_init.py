"""The background initialisation of section 3.3 on the channel with a
cylinder: from a lattice at ds_max, 3 ceil(ln(ds_max/ds_min)/ln C_r) passes
of the background update around the body's solid particles.

At the benchmark's size (D/100, 1:64, C_r = 1.05: 258 passes, about 4.3e5
background particles at the end) the oracle takes about 16 s per pass, so it
checks the first four passes there (1.6e3 to 1.2e5 particles, the growth of
the refined region), and the whole procedure on the same channel at D/12.5,
1:8 (129 passes).  Counts, splits, marks and the mass ledger are exact;
sizes, m_ref, positions and h agree within 1e-12.  The full 258 passes run
on the GPU with properties that hold at any size: the ledger, the size range,
the marks at ds_min, no split left pending, and the same result from two
contexts."""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import lib, odom

pytestmark = pytest.mark.gpu


def _setup(spec):
    s = W.channel_cylinder(spec)
    ds_max = spec.ds_min * spec.ratio
    bg = W.background_lattice(s["domain"], ds_max, 1.2, spec.rho0)
    sol = s["kind"] == W.SOLID
    sd = {"x": s["x"][sol], "y": s["y"][sol], "h": s["h"][sol]}
    return s, bg, sd, ds_max


def _ctx(P, s, spec, bg, cap):
    d = s["domain"]
    ds_max = spec.ds_min * spec.ratio
    cfg = P.Config(lo=d.lo, hi=d.hi, periodic=d.periodic, h_lo=0.25 * spec.ds_min,
                   h_hi=2.5 * ds_max, cr=spec.cr, ds_min=spec.ds_min, ds_max=ds_max,
                   bg_mass_q=bg["mass_q"], mass_q=s["mass_q"])
    return cfg, P.Context(cfg, cap)


def _solids(P, sd):
    return P.Particles.from_arrays(dict(sd, mq=np.ones(sd["x"].size, np.int64)))


def _compare(gb, ob, tag):
    assert gb["x"].size == ob["x"].size, tag
    assert np.array_equal(gb["mask"], ob["mask"]) and np.array_equal(gb["mq"], ob["mq"]), tag
    for k in ("ds", "mref"):
        assert np.allclose(gb[k], ob[k], rtol=1e-12, atol=0), (tag, k)
    for k in ("x", "y", "h"):
        e = float(np.max(np.abs(gb[k] - ob[k])))
        print(f"[bg-init] {tag} max|d{k}| = {e:.2e}", flush=True)
        assert e < 1e-12, (tag, k, e)


def _oracle(s, spec, bg, sd, passes, cap):
    ds_max = spec.ds_min * spec.ratio
    bp = oracle.BgPrm(cr=spec.cr, ds_min=spec.ds_min, ds_max=ds_max, mass_q=bg["mass_q"])
    return oracle.bg_update(odom(s["domain"]), bp, bg, sd, passes, cap=cap)


def test_channel_first_passes_vs_oracle():
    P = lib()
    spec = W.ChannelSpec()
    s, bg, sd, _ = _setup(spec)
    cap = 600_000
    cfg, ctx = _ctx(P, s, spec, bg, cap)
    assert P.bg_init_passes(cfg) == 258
    B = P.Background.from_arrays(bg, cap)
    print(f"[bg-init] D/100 1:64 bg0={bg['x'].size} solids={sd['x'].size}: 4 passes", flush=True)
    nsplit = ctx.bg_update(B, _solids(P, sd), 4)
    t = time.perf_counter()
    ob, onsplit = _oracle(s, spec, bg, sd, 4, cap)
    print(f"[bg-init] gpu n={B.n} splits={nsplit}; oracle n={ob['x'].size} splits={onsplit} "
          f"({time.perf_counter() - t:.1f} s)", flush=True)
    assert nsplit == onsplit > 0
    _compare(B.numpy(), ob, "4 passes")


def test_channel_whole_procedure_vs_oracle():
    P = lib()
    spec = W.ChannelSpec(ds_min=0.08, ratio=8)
    s, bg, sd, _ = _setup(spec)
    cap = 200_000
    cfg, ctx = _ctx(P, s, spec, bg, cap)
    passes = P.bg_init_passes(cfg)
    assert passes == oracle.bg_init_passes(spec.ds_min, spec.ds_min * spec.ratio, spec.cr) == 129
    B = P.Background.from_arrays(bg, cap)
    print(f"[bg-init] D/12.5 1:8 bg0={bg['x'].size}: {passes} passes", flush=True)
    nsplit = ctx.bg_update(B, _solids(P, sd), passes)
    t = time.perf_counter()
    ob, onsplit = _oracle(s, spec, bg, sd, passes, cap)
    print(f"[bg-init] gpu n={B.n} splits={nsplit}; oracle n={ob['x'].size} splits={onsplit} "
          f"({time.perf_counter() - t:.1f} s)", flush=True)
    assert nsplit == onsplit > 0
    _compare(B.numpy(), ob, "whole procedure")


def test_channel_config_size_procedure():
    P = lib()
    spec = W.ChannelSpec()
    s, bg, sd, ds_max = _setup(spec)
    cap = 1_000_000
    results = []
    for rep in range(2):
        cfg, ctx = _ctx(P, s, spec, bg, cap)
        B = P.Background.from_arrays(bg, cap)
        passes = P.bg_init_passes(cfg)
        t = time.perf_counter()
        nsplit = ctx.bg_update(B, _solids(P, sd), passes)
        ms = (time.perf_counter() - t) * 1e3
        print(f"[bg-init] D/100 1:64 run {rep}: {passes} passes, n={B.n}, splits={nsplit}, "
              f"{ms:.0f} ms", flush=True)
        results.append((B.numpy(), nsplit))
        del ctx, B
    (b, ns), (b2, ns2) = results
    assert ns == ns2 and b["x"].size == b2["x"].size
    for k in b:
        assert np.array_equal(b[k], b2[k]), k
    # the ledger: splits move mass between slots, never create or lose any
    assert int(b["mq"].sum()) == int(bg["mq"].sum())
    assert b["x"].size == bg["x"].size + 6 * ns
    # the sizes: graded within [ds_min, ds_max], ds_min at every mark
    assert b["ds"].min() == spec.ds_min and b["ds"].max() == ds_max
    assert np.all(b["ds"][b["mask"] > 0] == spec.ds_min)
    assert np.array_equal(b["mref"], 1.0 * b["ds"] * b["ds"])
    # the procedure has reached its end: no particle above the split bound
    cfg, _ = _ctx(P, s, spec, bg, 16)
    m = b["mq"] * bg["mass_q"]
    assert np.all(m <= cfg.mmax_f * b["mref"])
    # the refined region reaches the body: every solid particle has a
    # background particle at ds_min within 3 h of it
    fine = b["mask"] > 0
    fx, fy = b["x"][fine], b["y"][fine]
    for k in range(0, sd["x"].size, 7):
        r2 = (fx - sd["x"][k]) ** 2 + (fy - sd["y"][k]) ** 2
        assert r2.min() < (3.0 * sd["h"][k]) ** 2
