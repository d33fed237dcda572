"""Pins of the oracle's neighbour relation: j in N(i) iff r_ij < 3 max(h_i, h_j)
(quintic support, section 2; symmetric because the rates use W(h_i) and
W(h_j)).  The cell-list build is checked against brute force, brute force
against an exact lattice count and against an independent numpy test."""
import numpy as np
import pytest

import workloads as W


def _dom(orc, d):
    return orc.Dom(d.lo, d.hi, d.periodic)


def _csr_equal(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _numpy_pairs(x, y, h, dom):
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    for a, d in ((0, dx), (1, dy)):
        if dom.periodic[a]:
            L = dom.hi[a] - dom.lo[a]
            d[d > L / 2] -= L
            d[d < -L / 2] += L
    r2 = dx * dx + dy * dy
    R = 3 * np.maximum(h[:, None], h[None, :])
    return r2 < R * R


@pytest.mark.parametrize("case", ["periodic", "open", "clustered", "mixed"])
def test_cells_equal_brute(orc, case):
    if case == "periodic":
        s = W.random_varh(1500, seed=11, h_lo=0.006, ratio=8)
    elif case == "open":
        s = W.random_varh(1500, seed=12, h_lo=0.006, ratio=8, periodic=(False, False))
    elif case == "clustered":
        s = W.clustered_varh(1800, seed=13)
    else:
        s = W.random_varh(1200, seed=14, h_lo=0.01, ratio=3, periodic=(True, False),
                          lo=(-1.0, 0.5), hi=(2.0, 1.25))
    dom = _dom(orc, s["domain"])
    b = orc.neighbors(dom, s["x"], s["y"], s["h"], "brute")
    c = orc.neighbors(dom, s["x"], s["y"], s["h"], "cells")
    assert _csr_equal(b, c)
    # independent vectorised predicate
    M = _numpy_pairs(s["x"], s["y"], s["h"], s["domain"])
    assert b[1].size == M.sum()
    rows = np.repeat(np.arange(s["x"].size), np.diff(b[0]))
    assert M[rows, b[1]].all()
    # symmetric, self included, rows ascending
    assert np.array_equal(M, M.T)
    assert all(np.all(np.diff(b[1][b[0][i]:b[0][i + 1]]) > 0) for i in range(0, s["x"].size, 97))
    assert M.diagonal().all()


def test_lattice_counts_exact(orc):
    # power-of-two lattice: all distances exact, the tie r = 3h is excluded
    n = 64
    dx = 1.0 / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = (i.ravel() + 0.5) * dx
    y = (j.ravel() + 0.5) * dx
    dom = orc.Dom()
    rp, _ = orc.neighbors(dom, x, y, np.full(x.size, dx))
    # lattice points with a^2 + b^2 < 9: the 5x5 block
    assert np.all(np.diff(rp) == 25)
    rp, _ = orc.neighbors(dom, x, y, np.full(x.size, 1.2 * dx))
    cnt = sum(1 for a in range(-4, 5) for b in range(-4, 5) if a * a + b * b < 3.6 ** 2)
    assert cnt == 37 and np.all(np.diff(rp) == 37)


def test_cross_cells_equal_brute(orc):
    a = W.random_varh(700, seed=21, h_lo=0.01, ratio=4)
    b = W.random_varh(500, seed=22, h_lo=0.02, ratio=6)
    dom = _dom(orc, a["domain"])
    r1 = orc.cross_neighbors(dom, a["x"], a["y"], a["h"], b["x"], b["y"], b["h"], "brute")
    r2 = orc.cross_neighbors(dom, a["x"], a["y"], a["h"], b["x"], b["y"], b["h"], "cells")
    assert _csr_equal(r1, r2)


def test_empty_and_single(orc):
    dom = orc.Dom()
    rp, col = orc.neighbors(dom, np.zeros(0), np.zeros(0), np.zeros(0))
    assert rp.tolist() == [0] and col.size == 0
    rp, col = orc.neighbors(dom, np.array([0.5]), np.array([0.5]), np.array([0.1]))
    assert rp.tolist() == [0, 1] and col.tolist() == [0]
