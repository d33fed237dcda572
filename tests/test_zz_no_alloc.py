"""The rate evaluation that allocates nothing (sph_rates_noalloc, scratch in
a static device array) against the context-based sph_rates with the same
configuration (a lean workspace, the list built afresh): the same kernels on
the same input give the same bits.  Two calls in a row on one GPU share the
static scratch; the second has fewer particles, so stale contents of the
first would show.  Both are also checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import check_rates, ctx_for, lib, odom, particles

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "beta", "pavg", "nnb", "dxs", "dys", "dpdt", "dudt", "dvdt")


def _wall_case():
    s = W.wall_box(nx=40, ny=36, layers=3, jitter=0.1, seed=31)
    rng = np.random.default_rng(32)
    fl = s["kind"] == W.FLUID
    n = s["x"].size
    s["u"] = np.where(fl, 0.3 * np.sin(2 * np.pi * s["x"]) + 0.05 * rng.standard_normal(n), 0.0)
    s["v"] = np.where(fl, 0.1 * rng.standard_normal(n), 0.0)
    s["p"] = np.where(fl, 1.0 - 2.0 * s["y"], 0.0)
    s["rho"] = 1.0 + 0.01 * rng.standard_normal(n)
    s["params"] = {"rho0": 1.0, "cs": 10.0, "nu": 0.01, "hdx": 1.0}
    s["m"] = s["mq"] * s["mass_q"]
    return s


def _cases():
    big = _wall_case()
    small = W.tgv(24, seed=5)
    return (("wall box", big, (0.0, -2.0)), ("tgv 24x24", small, (0.0, 0.0)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_context_rates(prec):
    P = lib()
    pr = P.SPH_FP64 if prec == "fp64" else P.SPH_FP32
    ns = []
    for label, s, body in _cases():
        n = s["x"].size
        ns.append(n)
        print(f"[noalloc] {label} n={n} prec={prec}", flush=True)
        ctx = ctx_for(P, s, pr, body_force=body, lean=1, list_skin=0.0)
        assert P.rates_noalloc_bytes(ctx.cfg, n) <= P.NOALLOC_SCRATCH_BYTES
        ps = particles(P, s)
        ref = ctx.rates(ps, 1e-4)
        ps2 = particles(P, s)
        got = P.rates_noalloc(ctx.cfg, ps2, 1e-4)
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(got[k], ref[k]), (label, k)
        # the boundary values written into the state, as sph_rates writes them
        for k in ("p", "u", "v"):
            assert torch.equal(getattr(ps2, k)[:n], getattr(ps, k)[:n]), (label, k)
        prm = oracle.Prm(rho0=1.0, cs=s["params"]["cs"], nu=s["params"]["nu"],
                         hdx=s["params"]["hdx"], fx=body[0], fy=body[1], mass_q=s["mass_q"])
        if "kind" in s:
            o = oracle.rates_k(odom(s["domain"]), prm, s, 1e-4)
        else:
            o = oracle.rates(odom(s["domain"]), prm, s["x"], s["y"], s["u"], s["v"], s["p"],
                             s["h"], s["mq"] * s["mass_q"], 1e-4)
        check_rates(got, o, prec, f"noalloc {label}")
    assert ns[1] < ns[0]


def test_noalloc_rejects_oversize():
    """More particles than the static scratch holds: SPH_E_NOMEM with a
    message, decided on the host before any device work."""
    P = lib()
    s = W.tgv(24, seed=5)
    cfg = P.config_for(s["domain"], s["params"], float(s["h"].min()), float(s["h"].max()),
                       mass_q=s["mass_q"])
    n_big = 400_000
    assert P.rates_noalloc_bytes(cfg, n_big) > P.NOALLOC_SCRATCH_BYTES
    ps = particles(P, s)
    ps.n = n_big
    ps.capacity = n_big   # the arrays are never touched: the size check comes first
    with pytest.raises(P.SphError) as e:
        P.rates_noalloc(cfg, ps, 1e-4, out={k: torch.empty(1, dtype=torch.float64, device="cuda")
                                             for k in FIELDS})
    assert e.value.code == P.SPH_E_NOMEM and "scratch" in str(e.value)
