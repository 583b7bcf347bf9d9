"""Pins of the oracle's arithmetic against exact rational arithmetic (CPU only).

* TwoSum / QuickTwoSum / TwoProd (Sec. 2) are error-free: s == fl(a+b) (resp. fl(ab))
  and s + e == a + b (resp. ab) exactly, checked with Fractions on random and
  adversarial operands.
* Double-double add and multiply (Algs 1-2), the DD-times-binary64 product (Alg 3,
  with the trailing product restored) and the QD/TD sloppy add and multiply (Sec. 2,
  after Hida, Li and Bailey) meet error bounds relative to the exact result.  A
  dropped or mis-signed term in any of them shows up as an error of order 2^-53 or
  2^-106 relative, far outside the bounds.
* Commutativity where it holds bitwise (DD add and mul, QD add), exactness on
  small-integer inputs, non-overlapping outputs.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import ref
from workloads import random_mp, is_nonoverlapping

F = Fraction


def _adversarial_pairs(rng, n):
    a = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-60, 60, n)
    b = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-60, 60, n)
    extra_a = [1.0, 1.0, -1.0, 2.0 ** 52, 1.0 + 2 ** -52, 0.0, -0.0, 3.0, 1e300, 1e-300, 0.1, 2.0 ** -1022]
    extra_b = [2.0 ** -53, -2.0 ** -53, 1.0, 0.5, -(1.0 + 2 ** -52), 5.0, 0.0, -3.0, -1e300, 1e-300, 0.2,
               2.0 ** -1022]
    return np.concatenate([a, extra_a]), np.concatenate([b, extra_b])


def test_two_sum_exact():
    rng = np.random.default_rng(11)
    a, b = _adversarial_pairs(rng, 20000)
    s, e = ref.eft("two_sum", a, b)
    for ai, bi, si, ei in zip(a, b, s, e):
        assert si == ai + bi
        assert F(si) + F(ei) == F(ai) + F(bi)


def test_quick_two_sum_exact_when_ordered():
    rng = np.random.default_rng(12)
    a, b = _adversarial_pairs(rng, 20000)
    big = np.where(np.abs(a) >= np.abs(b), a, b)
    small = np.where(np.abs(a) >= np.abs(b), b, a)
    s, e = ref.eft("quick_two_sum", big, small)
    for ai, bi, si, ei in zip(big, small, s, e):
        assert si == ai + bi
        assert F(si) + F(ei) == F(ai) + F(bi)


def test_two_prod_exact():
    rng = np.random.default_rng(13)
    a = rng.uniform(-1, 1, 20000) * 2.0 ** rng.integers(-300, 300, 20000)
    b = rng.uniform(-1, 1, 20000) * 2.0 ** rng.integers(-300, 300, 20000)
    a = np.concatenate([a, [1.0 + 2 ** -52, 3.0, 2.0 ** 26 + 1, 0.0, -7.0, 0.1]])
    b = np.concatenate([b, [1.0 - 2 ** -53, 1.0 / 3, 2.0 ** 26 - 1, 5.0, -0.0, 0.1]])
    p, e = ref.eft("two_prod", a, b)
    for ai, bi, pi, ei in zip(a, b, p, e):
        assert pi == ai * bi
        assert F(pi) + F(ei) == F(ai) * F(bi)


def _exact(x, i):
    return sum((F(float(c)) for c in x[:, i]), F(0))


# (K, op) -> bits b with |computed - exact| <= 2^-b * scale  (scale = |x|+|y| for add, |x||y| for mul)
BOUNDS = {(2, "add"): 103, (2, "mul"): 103, (3, "add"): 154, (3, "mul"): 154, (4, "add"): 204, (4, "mul"): 204}


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_mp_ops_error_bound(K, op):
    rng = np.random.default_rng(100 + K)
    n = 3000
    x = random_mp(n, K, rng)
    y = random_mp(n, K, rng)
    # include heavy cancellation (y ~ -x) and wide exponent gaps
    y[:, :300] = -x[:, :300]
    y[1:, :300] = random_mp(300, K, rng)[1:] * 1e-3
    x[:, 300:600] *= 2.0 ** 70
    r = ref.elementwise(K, op, x, y)
    assert is_nonoverlapping(r)
    bits = BOUNDS[(K, op)]
    worst = 0.0
    for i in range(n):
        ex_x, ex_y, got = _exact(x, i), _exact(y, i), _exact(r, i)
        ex = ex_x + ex_y if op == "add" else ex_x * ex_y
        scale = abs(ex_x) + abs(ex_y) if op == "add" else abs(ex_x * ex_y)
        err = abs(got - ex)
        assert err * 2 ** bits <= scale, (K, op, i, float(err / scale))
        if scale:
            worst = max(worst, float(err / scale))
    # the bound is not vacuous: the op is far more accurate than the next precision down
    assert worst < 2.0 ** -(53 * K - 10)


def test_dd_mul_d_bound():
    rng = np.random.default_rng(7)
    n = 3000
    x = random_mp(n, 2, rng)
    y = rng.uniform(-4, 4, n)
    r = ref.elementwise(2, "mul_d", x, y)
    for i in range(n):
        ex = _exact(x, i) * F(float(y[i]))
        assert abs(_exact(r, i) - ex) * 2 ** 104 <= abs(ex)


@pytest.mark.parametrize("K,op", [(2, "add"), (2, "mul"), (3, "add"), (4, "add")])
def test_commutative_bitwise(K, op):
    rng = np.random.default_rng(21)
    x = random_mp(2000, K, rng)
    y = random_mp(2000, K, rng)
    assert np.array_equal(ref.elementwise(K, op, x, y), ref.elementwise(K, op, y, x))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_small_integers_exact(K):
    rng = np.random.default_rng(5)
    n = 2000
    x = np.zeros((K, n))
    y = np.zeros((K, n))
    x[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    y[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    for op in ("add", "mul"):
        r = ref.elementwise(K, op, x, y)
        ex = x[0] + y[0] if op == "add" else x[0] * y[0]
        assert np.array_equal(r[0], ex)
        assert np.all(r[1:] == 0)


def test_renorm_preserves_value_and_separates():
    rng = np.random.default_rng(3)
    n = 3000
    c = np.zeros((5, n))
    c[0] = rng.uniform(-1, 1, n)
    for k in range(1, 5):
        c[k] = c[k - 1] * 2.0 ** -50 * rng.uniform(-1, 1, n)
    c[:, :100] = 0.0                 # all-zero input
    c[2, 100:200] = 0.0              # zero in the middle
    r = ref.renorm5(c)
    assert is_nonoverlapping(r)
    for i in range(n):
        tot = sum((F(float(v)) for v in c[:, i]), F(0))
        got = _exact(r, i)
        assert abs(got - tot) <= abs(tot) * F(1, 2 ** 206)
    assert np.all(r[:, :100] == 0)
