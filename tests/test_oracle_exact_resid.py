"""Pins of the exact-residual oracle (oracle_exact_residual, used to certify solves).

Its exact residual, rounded to binary64, must equal an independent exact computation
with Python integers (oracle/exact.py) rounded by Python's correctly rounded integer
division, bit for bit, for DD/TD/QD and binary64 matrices with wide exponent ranges
and heavy cancellation; its norm bounds must bracket the exact rational norms within
a relative 1e-9; integer systems solved exactly give a zero residual."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, ref
from workloads import random_csr, random_mp

SCALE = 1 << (-exact.E_SCALE)


def python_exact(row_ptr, col_idx, a, b, x):
    """(r_i exact Fractions, b_i exact Fractions) by exact.py's integer products."""
    ys, _ = exact.exact_row_products(row_ptr, col_idx, a, x)
    n = b.shape[1]
    r = [Fraction(exact.fixed_mp(b[:, i]) - ys[i], SCALE) for i in range(n)]
    bb = [Fraction(exact.fixed_mp(b[:, i]), SCALE) for i in range(n)]
    return r, bb


def check(row_ptr, col_idx, a, b, x):
    got = ref.exact_residual(row_ptr, col_idx, a, b, x, want_vector=True)
    a2 = a.reshape(1, -1) if a.ndim == 1 else a
    r, bv = python_exact(row_ptr, col_idx, a2, b, x)
    want = np.array([float(v) for v in r])
    assert np.array_equal(got["r"], want), np.nonzero(got["r"] != want)[0][:5]
    rr = sum(v * v for v in r)
    bb = sum(v * v for v in bv)
    assert Fraction(got["rr_upper"]) >= rr
    assert Fraction(got["bb_lower"]) <= bb
    if rr > 0:
        assert Fraction(got["rr_upper"]) <= rr * Fraction(1 + 10 ** -9)
    assert Fraction(got["bb_lower"]) >= bb * Fraction(1 - 10 ** -9)
    return got, r


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_matches_python_integers(K):
    rng = np.random.default_rng(40 + K)
    n = 300
    lengths = rng.integers(0, 12, n)
    row_ptr, col_idx, a, _ = random_csr(n, n, lengths, max(K, 2), rng)
    a = a[0] if K == 1 else a[:K]
    Kx = max(K, 2)
    x = random_mp(n, Kx, rng)
    # scale rows and columns over a wide exponent range
    x *= np.ldexp(1.0, rng.integers(-300, 300, n))[None, :]
    b = random_mp(n, Kx, rng) * np.ldexp(1.0, rng.integers(-300, 300, n))[None, :]
    check(row_ptr, col_idx, a, b, x)


def test_cancellation_to_the_last_bit():
    """b equal to A x up to a planted tail: the residual is exactly that tail (far
    below every stored leading component)."""
    rng = np.random.default_rng(50)
    n = 200
    lengths = rng.integers(1, 8, n)
    row_ptr, col_idx, a, _ = random_csr(n, n, lengths, 2, rng)
    x = random_mp(n, 2, rng)
    b = ref.spmv(2, row_ptr, col_idx, a, x)      # DD product: exact up to ~2^-100 relative
    got, r = check(row_ptr, col_idx, a, b, x)
    assert all(abs(v) <= 2.0 ** -90 * 50 for v in r)
    assert got["relres_upper"] < 1e-25


def test_integer_system_solved_exactly_is_zero():
    rng = np.random.default_rng(51)
    n = 500
    lengths = rng.integers(1, 9, n)
    row_ptr, col_idx, _, _ = random_csr(n, n, lengths, 2, rng)
    a = np.zeros((2, col_idx.size))
    a[0] = rng.integers(-1000, 1000, col_idx.size)
    x = np.zeros((2, n))
    x[0] = rng.integers(-1000, 1000, n)
    b = np.zeros((2, n))
    for i in range(n):
        s = sum(int(a[0, k]) * int(x[0, col_idx[k]]) for k in range(row_ptr[i], row_ptr[i + 1]))
        b[0, i] = float(s)
    got = ref.exact_residual(row_ptr, col_idx, a, b, x, want_vector=True)
    assert got["rr_upper"] == 0.0 and np.all(got["r"] == 0)
    # one unit changed in one b entry: the residual is exactly that unit
    b[0, 7] += 1.0
    got = ref.exact_residual(row_ptr, col_idx, a, b, x, want_vector=True)
    assert got["r"][7] == 1.0 and np.count_nonzero(got["r"]) == 1
    assert 1.0 <= got["rr_upper"] <= 1.0 + 1e-9


def test_sign_and_scaling_invariants():
    """r(-b, -x... ) : negating b and x negates r exactly; scaling b and x by 2^k scales
    r by 2^k exactly."""
    rng = np.random.default_rng(52)
    n = 150
    lengths = rng.integers(0, 10, n)
    row_ptr, col_idx, a, _ = random_csr(n, n, lengths, 3, rng)
    x = random_mp(n, 3, rng)
    b = random_mp(n, 3, rng)
    r0 = ref.exact_residual(row_ptr, col_idx, a, b, x, want_vector=True)["r"]
    r1 = ref.exact_residual(row_ptr, col_idx, a, -b, -x, want_vector=True)["r"]
    r2 = ref.exact_residual(row_ptr, col_idx, a, b * 2.0 ** 37, x * 2.0 ** 37, want_vector=True)["r"]
    assert np.array_equal(r1, -r0)
    assert np.array_equal(r2, r0 * 2.0 ** 37)


def test_rounding_ties_to_even():
    """Residuals exactly halfway between two binary64 values round to the even one
    (rows without entries, so r = b exactly)."""
    row_ptr = np.zeros(6, dtype=np.int32)
    col_idx = np.zeros(0, dtype=np.int32)
    a = np.zeros((2, 0))
    t = 2.0 ** 53
    b = np.array([[t, t, t + 2, -t, 1.0], [1.0, 3.0, 1.0, -1.0, 2.0 ** -60]])
    got, _ = check(row_ptr, col_idx, a, b, np.zeros((2, 5)))
    assert list(got["r"]) == [t, t + 4, t + 4, -t, 1.0]
