"""Pins of the oracle's exact sum (the long accumulator of the background
update's sums over neighbours): it equals Python's math.fsum, which rounds
the exact sum once to nearest with ties to even, bit for bit, on sums built
to be hard: near-total cancellation, terms across the whole exponent range,
subnormal results, exact ties, and every ordering of the same terms."""
import math
import struct

import numpy as np
import pytest


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def _same(a, b):
    return struct.pack("<d", a) == struct.pack("<d", b)


def _check(orc, x):
    x = np.asarray(x, dtype=np.float64)
    ref = math.fsum(x.tolist())
    got = orc.exact_sum(x)
    assert _same(got, ref), (got, ref, x[:8])


def test_exact_sum_special_cases(orc):
    tiny = 5e-324
    cases = [
        [], [0.0], [1.0], [-1.0], [1e308, -1e308], [1e308, 5e307, -1e308],
        [tiny], [tiny, tiny, tiny], [-tiny, 2 * tiny], [2.2250738585072014e-308, -tiny],
        [1.0, 2.0 ** -53],                     # a tie: stays at 1 (even)
        [1.0 + 2.0 ** -52, 2.0 ** -53],        # a tie: rounds up to even
        [1.0, 2.0 ** -53, 2.0 ** -105],        # just above the tie
        [1.0, -(2.0 ** -54), -(2.0 ** -160)],  # just below the half-way point
        [2.0 ** 1000, -(2.0 ** 1000), 3e-320],
        [0.1, 0.2, 0.3, -0.6], [1e16, 1.0, -1e16],
        [-0.1, -0.2, -0.3, 0.6], [1.5, -1.5, 1e-300, -1e-300 + 1e-310],
    ]
    for c in cases:
        _check(orc, c)


def test_exact_sum_random(orc):
    rng = np.random.default_rng(17)
    for t in range(400):
        n = int(rng.integers(1, 300))
        kind = t % 4
        if kind == 0:      # one scale
            x = rng.normal(size=n)
        elif kind == 1:    # wide exponent range
            x = rng.normal(size=n) * np.exp2(rng.integers(-1070, 1000, size=n).astype(float))
        elif kind == 2:    # mirror pairs with small leftovers: near-total cancellation
            a = rng.normal(size=n) * np.exp2(rng.integers(-40, 40, size=n).astype(float))
            x = np.concatenate([a, -a, rng.normal(size=3) * 1e-30])
        else:              # shift-like terms of a near-symmetric neighbourhood
            a = rng.uniform(-1, 1, size=n)
            x = np.concatenate([a * 1e-3, -a * 1e-3 * (1 + rng.normal(size=n) * 1e-15)])
        _check(orc, x)
        _check(orc, x[rng.permutation(x.size)])


def test_exact_sum_is_order_free(orc):
    rng = np.random.default_rng(5)
    a = rng.normal(size=200) * np.exp2(rng.integers(-60, 60, size=200).astype(float))
    x = np.concatenate([a, -a[::-1] * (1 + 1e-16), [1e-200]])
    ref = orc.exact_sum(x)
    for _ in range(20):
        assert _same(orc.exact_sum(x[rng.permutation(x.size)]), ref)
