"""Pins of the oracle's binary64-matrix products (CPU only): the K-component times
binary64 multiplications (Algs 3-5) and the SpMV of a binary64 matrix with a
K-component vector built on them.

* mul_d meets |r - x y| <= 2^-b |x y| (b = 104 / 155 / 205 for DD / TD / QD) against
  exact rational products, on random, widely scaled and cancellation-free operands
  with full tails; a misread of any garbled step of Alg 4 (x[3] added instead of
  multiplied, the error pair multiplied instead of summed, a dropped order-eps^3
  term) costs far more than 2^-160 relative and fails it.
* Small integers give exact products with zero tails.
* DD: the binary64-matrix SpMV equals the DD SpMV of the same matrix stored with zero
  trailing components, value for value (Alg 3 is Alg 2 with a zero trailing part).
* The 5x5 example of Sec. 3 times sqrt(2)[1..5] is sqrt(2)[7,-14,15,-22,40] to the
  K-component precision; integer data give exact rows; the exact-rational row bound
  max(len,1) 2^-b sum|a||x| (b = 100/150/200) holds on ragged random matrices.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref, exact
from workloads import random_csr, random_mp, sqrt2_vector, is_nonoverlapping

F = Fraction
MULD_BITS = {2: 104, 3: 155, 4: 205}
ROW_BITS = {2: 100, 3: 150, 4: 200}


def _exact(x, i):
    return sum((F(float(c)) for c in x[:, i]), F(0))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_mul_d_bound(K):
    rng = np.random.default_rng(300 + K)
    n = 3000
    x = random_mp(n, K, rng)
    x[:, 1000:1500] *= 2.0 ** 80
    y = rng.uniform(-4, 4, n) * 2.0 ** rng.integers(-40, 40, n)
    r = ref.elementwise(K, "mul_d", x, y)
    assert is_nonoverlapping(r)
    worst = 0.0
    for i in range(n):
        ex = _exact(x, i) * F(float(y[i]))
        err = abs(_exact(r, i) - ex)
        assert err * 2 ** MULD_BITS[K] <= abs(ex), (K, i, float(err / abs(ex)))
        worst = max(worst, float(err / abs(ex)))
    assert worst < 2.0 ** -(53 * K - 10)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_mul_d_small_integers_exact(K):
    rng = np.random.default_rng(310 + K)
    n = 2000
    x = np.zeros((K, n))
    x[0] = rng.integers(-2 ** 25, 2 ** 25, n)
    y = rng.integers(-2 ** 25, 2 ** 25, n).astype(np.float64)
    r = ref.elementwise(K, "mul_d", x, y)
    assert np.array_equal(r[0], x[0] * y)
    assert np.all(r[1:] == 0)


def test_dd_dmat_equals_zero_tail_dd_spmv():
    rng = np.random.default_rng(320)
    lengths = np.concatenate([[0, 1, 2, 3, 64, 65, 300], rng.integers(0, 120, 60)])
    row_ptr, col_idx, a2, _ = random_csr(lengths.size, 500, lengths, 2, rng)
    a = a2[0].copy()
    x = random_mp(500, 2, rng)
    padded = np.zeros((2, a.size))
    padded[0] = a
    for lw in (None, np.zeros(lengths.size, dtype=np.uint8)):
        got = ref.spmv_dmat(2, row_ptr, col_idx, a, x, log2w=lw)
        want = ref.spmv(2, row_ptr, col_idx, padded, x, log2w=lw)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_5x5_times_sqrt2(golden_dir, K):
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        g = json.load(f)
    row_ptr = np.array(g["csr_indptr"], dtype=np.int32)
    col_idx = np.array(g["csr_indices"], dtype=np.int32)
    a = np.array(g["csr_data"], dtype=np.float64)
    y = ref.spmv_dmat(K, row_ptr, col_idx, a, sqrt2_vector(5, K))
    m = g["Av_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    for i in range(5):
        got = exact.mp_value(y[:, i])
        tol = Fraction(abs(m[i]) * 16, 2 ** (53 * K - 6))
        lo, hi = abs(got) - tol, abs(got) + tol
        assert got * m[i] > 0 and lo * lo <= 2 * m[i] * m[i] <= hi * hi, (K, i)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_integer_rows_exact_and_bound(K):
    rng = np.random.default_rng(330 + K)
    lengths = rng.integers(0, 250, 50)
    row_ptr, col_idx, _, _ = random_csr(50, 300, lengths, K, rng)
    a = rng.integers(-2 ** 20, 2 ** 20, col_idx.size).astype(np.float64)
    x = np.zeros((K, 300))
    x[0] = rng.integers(-2 ** 20, 2 ** 20, 300)
    rows = np.repeat(np.arange(50), np.diff(row_ptr))
    want = np.zeros(50, dtype=object)
    for k in range(col_idx.size):
        want[rows[k]] += int(a[k]) * int(x[0, col_idx[k]])
    y = ref.spmv_dmat(K, row_ptr, col_idx, a, x)
    assert [int(v) for v in y[0]] == list(want) and np.all(y[1:] == 0)
    # ragged random values: exact-rational row bound
    lengths = np.concatenate([[0, 1, 2, 5, 64, 65, 400], rng.integers(0, 150, 30)])
    row_ptr, col_idx, _, _ = random_csr(lengths.size, 600, lengths, K, rng)
    a = rng.uniform(-1, 1, col_idx.size)
    x = random_mp(600, K, rng)
    padded = np.zeros((K, a.size))
    padded[0] = a
    lw_max = np.array([min(10, int(math.log2(max(1, L)))) for L in lengths], dtype=np.uint8)
    for lw in (None, np.zeros(lengths.size, dtype=np.uint8), lw_max):
        y = ref.spmv_dmat(K, row_ptr, col_idx, a, x, log2w=lw)
        ys, ss = exact.exact_row_products(row_ptr, col_idx, padded, x)
        for i in range(lengths.size):
            got = exact.fixed_mp(y[:, i])
            ratio = exact.error_ratio(got, ys[i], ss[i], int(lengths[i]), ROW_BITS[K])
            assert ratio <= 1.0, (K, i, ratio)
