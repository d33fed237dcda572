"""Density errors of splitting and merging (section 3.2), from the oracle's
own split and merge and its kernel, by quadrature on a fine grid where the
particles have full support:

- eq. (global-error): E_s = || m_p W_p - sum_k m_k W_k ||^2 for one particle
  split into seven.  At the paper's alpha = 0.9, eps = 0.4 it is 0.17% of
  || m_p W_p ||^2; the plausible mistakes in the split geometry (the
  hexagon radius taken from the child's h, alpha applied twice, the
  children keeping the parent's h, twice the radius) give 0.39% to 5.5%.
- eq. (merge-error), read as the same L2 norm (as printed the integrand
  integrates to zero): the error of merging two particles is small when
  they are close and of equal mass, and grows with the separation and the
  mass ratio, as the paper reports."""
import numpy as np
import pytest

import workloads as W

HP = 0.1


@pytest.fixture(scope="module")
def grid(orc):
    L = 3.0 * HP * 1.6
    g = np.linspace(-L, L, 161)
    X, Y = np.meshgrid(g, g, indexing="ij")
    kw = np.vectorize(orc.w)
    return X, Y, (g[1] - g[0]) ** 2, kw


def _state(x, y, h, m, q, mref):
    n = len(x)
    return {"x": np.array(x, float), "y": np.array(y, float), "u": np.zeros(n), "v": np.zeros(n),
            "p": np.zeros(n), "rho": np.ones(n), "h": np.array(h, float),
            "mref": np.array(mref, float), "mq": np.array([int(round(mi / q)) for mi in m], np.int64),
            "kind": np.zeros(n, np.int32)}


def _split_error(orc, grid, alpha, eps):
    X, Y, dA, kw = grid
    dom = orc.Dom((-1.0, -1.0), (1.0, 1.0), (False, False))
    q = W.mass_quantum(1.05)
    out, _ = orc.split_only(dom, orc.Prm(mass_q=q, split_alpha=alpha, split_eps=eps),
                            _state([0.0], [0.0], [HP], [1.0], q, [0.1]))
    assert out["x"].size == 7
    mk = out["mq"] * q
    rho_c = sum(mk[k] * kw(np.hypot(X - out["x"][k], Y - out["y"][k]), out["h"][k])
                for k in range(7))
    wp = kw(np.hypot(X, Y), HP)
    return float(np.sum((wp - rho_c) ** 2) * dA) / float(np.sum(wp ** 2) * dA)


def test_split_density_error(orc, grid):
    e = _split_error(orc, grid, 0.9, 0.4)
    assert e < 2.5e-3, e
    for alpha, eps in ((0.9, 0.36), (0.81, 0.4), (1.0, 0.4), (0.9, 0.8)):
        assert _split_error(orc, grid, alpha, eps) > 1.5 * e, (alpha, eps)


def _merge_error(orc, grid, d, ratio):
    X, Y, dA, kw = grid
    dom = orc.Dom((-1.0, -1.0), (1.0, 1.0), (False, False))
    q = W.mass_quantum(1.05 * 10.0)
    ma, mb = ratio / (1.0 + ratio), 1.0 / (1.0 + ratio)
    ha, hb = HP * np.sqrt(ma), HP * np.sqrt(mb)
    xa, xb = -d * HP * mb, d * HP * ma  # centre of mass at the origin
    st = _state([xa, xb], [0.0, 0.0], [ha, hb], [ma, mb], q, [10.0, 10.0])
    out, info = orc.merge_only(dom, orc.Prm(mass_q=q), st)
    assert info["pairs"] == 1 and out["x"].size == 1
    mm = out["mq"][0] * q
    rho_m = mm * kw(np.hypot(X - out["x"][0], Y - out["y"][0]), out["h"][0])
    rho_ab = (st["mq"][0] * q) * kw(np.hypot(X - xa, Y), ha) + (st["mq"][1] * q) * kw(
        np.hypot(X - xb, Y), hb)
    return float(np.sum((rho_m - rho_ab) ** 2) * dA) / float(np.sum(rho_ab ** 2) * dA)


def test_merge_density_error_trends(orc, grid):
    e_close = _merge_error(orc, grid, 0.2, 1.0)
    e_far = _merge_error(orc, grid, 0.6, 1.0)
    e_ratio = _merge_error(orc, grid, 0.6, 4.0)
    print(f"merge errors: close {e_close:.3e} far {e_far:.3e} ratio-4 {e_ratio:.3e}")
    assert e_close < 1e-2
    assert e_far > 2.0 * e_close
    assert e_ratio > e_far
