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
* Complex (Eq. 3 with these products): a_im = x_im = 0 gives the real product and a
  zero imaginary part; x -> i x gives y -> i y exactly; integer data are exact; the row
  bound holds for both parts; the 5x5 example times sqrt(2+3i)[1..5] has the modulus
  and phase of sqrt(2+3i) m.  (Swapping the matrix parts of one cross term, or the sign
  of the imaginary combination, fails these.)
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


# ---------------------------------------------------------------------------
# complex matrix of binary64 values times a K-component complex vector (Eq. 3 with
# the products of Algs 3-5)
# ---------------------------------------------------------------------------

def _complex_case(K, seed, n_rows=40, n_cols=300, maxlen=120):
    rng = np.random.default_rng(seed)
    lengths = np.concatenate([[0, 1, 2, 3, 64, 65], rng.integers(0, maxlen, n_rows - 6)])
    row_ptr, col_idx, _, _ = random_csr(lengths.size, n_cols, lengths, K, rng)
    a_re = rng.uniform(-1, 1, col_idx.size)
    a_im = rng.uniform(-1, 1, col_idx.size)
    x_re = random_mp(n_cols, K, rng)
    x_im = random_mp(n_cols, K, rng)
    return lengths, row_ptr, col_idx, a_re, a_im, x_re, x_im


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_complex_reduces_to_real(K):
    """With a_im = 0 and x_im = 0 the real part is the real binary64-matrix product and
    the imaginary part is zero, for every summation order."""
    lengths, row_ptr, col_idx, a_re, _, x_re, _ = _complex_case(K, 340 + K)
    zi_a = np.zeros_like(a_re)
    zi_x = np.zeros_like(x_re)
    for lw in (None, np.zeros(lengths.size, dtype=np.uint8)):
        yr, yi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, zi_a, x_re, zi_x, log2w=lw)
        assert np.array_equal(yr, ref.spmv_dmat(K, row_ptr, col_idx, a_re, x_re, log2w=lw))
        assert np.all(yi == 0)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_complex_times_i(K):
    """x -> i x gives y -> i y exactly (negation commutes with every rounded step); a
    swapped matrix part or sign in the cross terms breaks it."""
    lengths, row_ptr, col_idx, a_re, a_im, x_re, x_im = _complex_case(K, 350 + K)
    yr, yi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im)
    yr2, yi2 = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, -x_im, x_re)
    assert np.array_equal(yr2, -yi) and np.array_equal(yi2, yr)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_complex_integers_exact_and_bound(K):
    rng = np.random.default_rng(360 + K)
    lengths = rng.integers(0, 200, 40)
    row_ptr, col_idx, _, _ = random_csr(40, 300, lengths, K, rng)
    a_re = rng.integers(-2 ** 20, 2 ** 20, col_idx.size).astype(np.float64)
    a_im = rng.integers(-2 ** 20, 2 ** 20, col_idx.size).astype(np.float64)
    x_re = np.zeros((K, 300))
    x_im = np.zeros((K, 300))
    x_re[0] = rng.integers(-2 ** 20, 2 ** 20, 300)
    x_im[0] = rng.integers(-2 ** 20, 2 ** 20, 300)
    rows = np.repeat(np.arange(40), np.diff(row_ptr))
    wr = [0] * 40
    wi = [0] * 40
    for k in range(col_idx.size):
        j = col_idx[k]
        ar, ai, xr, xi = int(a_re[k]), int(a_im[k]), int(x_re[0, j]), int(x_im[0, j])
        wr[rows[k]] += ar * xr - ai * xi
        wi[rows[k]] += ar * xi + ai * xr
    yr, yi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im)
    assert [int(v) for v in yr[0]] == wr and [int(v) for v in yi[0]] == wi
    assert np.all(yr[1:] == 0) and np.all(yi[1:] == 0)
    # random values, ragged rows: |y - exact| <= max(len,1) 2^-b sum of the absolute products
    lengths, row_ptr, col_idx, a_re, a_im, x_re, x_im = _complex_case(K, 370 + K)
    for lw in (None, np.zeros(lengths.size, dtype=np.uint8)):
        yr, yi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im, log2w=lw)
        for i in range(lengths.size):
            er = ei = sr = si = F(0)
            for k in range(row_ptr[i], row_ptr[i + 1]):
                j = col_idx[k]
                ar, ai = F(float(a_re[k])), F(float(a_im[k]))
                xr, xi = _exact(x_re, j), _exact(x_im, j)
                er += ar * xr - ai * xi
                ei += ar * xi + ai * xr
                sr += abs(ar * xr) + abs(ai * xi)
                si += abs(ar * xi) + abs(ai * xr)
            L = max(1, int(lengths[i]))
            assert abs(_exact(yr, i) - er) * 2 ** ROW_BITS[K] <= L * sr, (K, i)
            assert abs(_exact(yi, i) - ei) * 2 ** ROW_BITS[K] <= L * si, (K, i)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dmat_complex_5x5_times_sqrt_2p3i(golden_dir, K):
    """The 5x5 example of Sec. 3 as a complex matrix with zero imaginary part times
    sqrt(2+3i)[1..5] (Eq. 4): y = sqrt(2+3i) m with m = A [1..5], so |y_j|^2 = sqrt(13) m_j^2
    and y_im / y_re = tan(atan2(3, 2) / 2) to the K-component precision."""
    from workloads import sqrt_2p3i_vector
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        g = json.load(f)
    row_ptr = np.array(g["csr_indptr"], dtype=np.int32)
    col_idx = np.array(g["csr_indices"], dtype=np.int32)
    a = np.array(g["csr_data"], dtype=np.float64)
    m = g["Av_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    vre, vim = sqrt_2p3i_vector(5, K)
    yr, yi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a, np.zeros_like(a), vre, vim)
    for i in range(5):
        re, im = exact.mp_value(yr[:, i]), exact.mp_value(yi[:, i])
        # (re^2 + im^2)^2 = 13 m^4 (|sqrt(2+3i)|^4 = 13)
        lhs = (re * re + im * im) ** 2
        rhs = 13 * F(m[i]) ** 4
        assert abs(lhs - rhs) <= rhs * F(64, 2 ** (53 * K - 8)), (K, i)
        # the phase: 2 re im / (re^2 - im^2) = tan(atan2(3, 2)) = 3/2
        assert abs(2 * re * im * 2 - 3 * (re * re - im * im)) <= abs(re * re) * F(64, 2 ** (53 * K - 8)), (K, i)
