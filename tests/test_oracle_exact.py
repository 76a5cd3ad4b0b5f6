"""Pins for the oracle's correctly rounded dot product.

The oracle defines every inner product as the exact sum of the exact products,
rounded once to nearest-even.  These tests check it against Python's exact
rational arithmetic (``fractions.Fraction``; ``float(Fraction)`` is correctly
rounded), on random data and on cases built to trip a wrong rounding, a lost
carry, a dropped sign, subnormals and overflow.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def exact_ref(x, y):
    s = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    try:
        return float(s)
    except OverflowError:
        return math.copysign(math.inf, s)


@pytest.mark.parametrize("seed", range(6))
def test_random_vs_fraction(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    scale = 10.0 ** rng.uniform(-30, 30, size=n)
    x = rng.standard_normal(n) * scale
    y = rng.standard_normal(n) / scale * 10.0 ** rng.uniform(-5, 5, size=n)
    assert oracle.exact_dot(x, y) == exact_ref(x, y)


def test_cancellation():
    x = np.array([1e300, 1.0, -1e300, 1e-300])
    y = np.array([1e5, 3.0, 1e5, 1e-20])
    assert oracle.exact_dot(x, y) == 3.0
    # naive summation loses the small term entirely
    v = np.array([1.0, 1e-30, -1.0])
    assert oracle.exact_sum(v) == 1e-30


def test_ties_to_even():
    u = 2.0 ** -53
    # exact 1 + 2^-53 is the midpoint between 1 and 1+2^-52: rounds to even (1)
    assert oracle.exact_sum([1.0, u]) == 1.0
    # 1 + 3*2^-53 is the midpoint between 1+2^-52 and 1+2^-51: rounds to 1+2^-51
    assert oracle.exact_sum([1.0, u, u, u]) == 1.0 + 2.0 ** -51
    # just above the midpoint rounds up
    assert oracle.exact_sum([1.0, u, 2.0 ** -200]) == 1.0 + 2.0 ** -52
    # just below rounds down, also for negative sums
    assert oracle.exact_sum([-1.0, -u, 2.0 ** -200]) == -1.0


def test_subnormal_and_underflow():
    tiny = 5e-324
    assert oracle.exact_sum([tiny, tiny, tiny]) == 3 * tiny
    x = np.array([1e-200, 3e-170])
    y = np.array([1e-200, 1e-160])
    assert oracle.exact_dot(x, y) == exact_ref(x, y)
    # products far below the subnormal range round to zero
    assert oracle.exact_dot([1e-300], [1e-300]) == 0.0
    # ... unless they accumulate: 2^-1075 is a tie (to 0), 3*2^-1076 rounds up
    a = 2.0 ** -537
    b = 2.0 ** -538
    assert oracle.exact_dot([a], [b]) == 0.0
    assert oracle.exact_dot([a, a, a], [b, b, b]) == exact_ref([a] * 3, [b] * 3)


def test_overflow_and_nonfinite():
    assert oracle.exact_dot([1e200], [1e200]) == math.inf
    assert oracle.exact_dot([1e200, -1e200], [1e200, 1e200]) == 0.0
    assert oracle.exact_dot([-1e200], [1e200]) == -math.inf
    assert math.isnan(oracle.exact_dot([1.0, math.nan], [1.0, 1.0]))
    assert oracle.exact_dot([], []) == 0.0


def test_order_independent():
    rng = np.random.default_rng(7)
    x = rng.standard_normal(5000) * 10.0 ** rng.uniform(-8, 8, 5000)
    y = rng.standard_normal(5000)
    a = oracle.exact_dot(x, y)
    perm = rng.permutation(5000)
    assert oracle.exact_dot(x[perm], y[perm]) == a
    assert oracle.exact_dot(x[::-1].copy(), y[::-1].copy()) == a


def test_exp_rounded_to_nearest():
    """The oracle's exp (the Gaussian source) is exp(x) rounded once to the
    nearest double: against a 40-digit decimal exponential converted to the
    nearest double, on random and special arguments of the source's range."""
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    rng = np.random.default_rng(3)
    xs = list(-150.0 * rng.random(20000)) + list(-rng.random(2000) * 1e-3) + [0.0, -0.0, -1e-300, -700.0,
                                                                              -0.34657359027997264, -84.375]
    for x in xs:
        want = float(Decimal(x).exp())
        got = oracle.core.exp_rn(x)
        assert got == want, (x.hex(), got.hex(), want.hex())
