"""Pins of the oracle's CSR SpMV (CPU only).

* The 5x5 example of Sec. 3 (Eq. 1): the printed COO and CSR arrays are reproduced
  from the dense matrix, and A v with the paper's v = sqrt(2)[1..5] (Sec. 4, Eq. 4)
  equals sqrt(2)[7,-14,15,-22,40] to the K-component precision, real and complex
  (v = sqrt(2+3i)[1..5]).
* Hand-derived rows (tests/golden/order_rows.json) whose DD result depends on the
  summation order, pinning the lane/fold reading of Fig. 1.
* Integer inputs small enough that every partial sum is exact give the exact product
  with zero tails, in every order.
* Exact-rational error bound |y - Ax| <= max(len,1) 2^-b sum|a||x| with b = 100/150/200
  (DD/TD/QD) on the 2D 5-point workload (49,600 nnz) and on ragged random matrices.
* Invariants that hold bitwise: power-of-two scaling, y(-A) = -y(A), row permutation;
  complex: A_im = x_im = 0 reproduces the real product, x -> i x maps y -> i y.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref, exact
from workloads import (csr_from_dense, paper_example_5x5, sqrt2_vector, sqrt_2p3i_vector, laplace2d_5pt,
                       random_csr, random_mp)

BITS = {2: 100, 3: 150, 4: 200}


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _val(s):
    if isinstance(s, str):
        assert s.startswith("2^")
        return 2.0 ** int(s[2:])
    return float(s)


def test_5x5_csr_arrays_match_paper(golden_dir):
    g = _load(golden_dir, "csr_5x5.json")
    row_ptr, col_idx, vals = csr_from_dense(np.array(g["dense"], dtype=float))
    assert list(row_ptr) == g["csr_indptr"]
    assert list(col_idx) == g["csr_indices"]
    assert list(vals) == g["csr_data"]
    # COO row-wise order is the same sequence with explicit rows
    rows = np.repeat(np.arange(5), np.diff(row_ptr))
    assert list(rows) == g["coo_row"] and list(col_idx) == g["coo_col"]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_5x5_times_sqrt2(golden_dir, K):
    g = _load(golden_dir, "csr_5x5.json")
    row_ptr = np.array(g["csr_indptr"], dtype=np.int32)
    col_idx = np.array(g["csr_indices"], dtype=np.int32)
    a = np.zeros((K, 8))
    a[0] = g["csr_data"]
    v = sqrt2_vector(5, K)
    y = ref.spmv(K, row_ptr, col_idx, a, v)
    m = g["Av_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    for i in range(5):
        got = exact.mp_value(y[:, i])
        # |got - sqrt2 m|: compare squares with exact integers, tolerance from the K-component rounding
        tol = Fraction(abs(m[i]) * 16, 2 ** (53 * K - 6))
        assert got * m[i] > 0
        lo, hi = abs(got) - tol, abs(got) + tol
        assert lo * lo <= 2 * m[i] * m[i] <= hi * hi, (K, i)
    # A^T v from the same arrays, read column-wise (transpose by re-indexing)
    dense = np.array(g["dense"], dtype=float)
    rpt, cit, vt = csr_from_dense(dense.T)
    at = np.zeros((K, vt.size))
    at[0] = vt
    yt = ref.spmv(K, rpt, cit, at, v)
    mt = g["ATv_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    for i in range(5):
        got = exact.mp_value(yt[:, i])
        tol = Fraction(abs(mt[i]) * 16, 2 ** (53 * K - 6))
        lo, hi = abs(got) - tol, abs(got) + tol
        assert got * mt[i] > 0 and lo * lo <= 2 * mt[i] * mt[i] <= hi * hi


@pytest.mark.parametrize("K", [2, 3, 4])
def test_5x5_complex_times_sqrt_2p3i(golden_dir, K):
    g = _load(golden_dir, "csr_5x5.json")
    row_ptr = np.array(g["csr_indptr"], dtype=np.int32)
    col_idx = np.array(g["csr_indices"], dtype=np.int32)
    a_re = np.zeros((K, 8))
    a_re[0] = g["csr_data"]
    a_im = np.zeros((K, 8))
    vre, vim = sqrt_2p3i_vector(5, K)
    yre, yim = ref.spmv(K, row_ptr, col_idx, a_re, vre, a_im=a_im, x_im=vim)
    m = g["Av_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    # (yre + i yim) / m must equal sqrt(2+3i) = p + iq, with p^2 - q^2 = 2 and 2pq = 3
    for i in range(5):
        p = exact.mp_value(yre[:, i]) / m[i]
        q = exact.mp_value(yim[:, i]) / m[i]
        tol = Fraction(64, 2 ** (53 * K - 8))
        assert abs(p * p - q * q - 2) <= tol and abs(2 * p * q - 3) <= tol
        assert p > 0 and q > 0


def test_order_rows(golden_dir):
    g = _load(golden_dir, "order_rows.json")
    for row in g["rows"]:
        a_hi = [_val(v) for v in row["a_hi"]]
        n = len(a_hi)
        row_ptr = np.array([0, n], dtype=np.int32)
        col_idx = np.arange(n, dtype=np.int32)
        a = np.zeros((2, n))
        a[0] = a_hi
        x = np.zeros((2, n))
        x[0] = 1.0
        for wkey, exp in row["expected"].items():
            lw = int(math.log2(int(wkey[1:])))
            y = ref.spmv(2, row_ptr, col_idx, a, x, log2w=np.array([lw], dtype=np.uint8))
            assert list(y[:, 0]) == [_val(e) for e in exp], (row["name"], wkey)
        # the canonical order is the largest power of two <= min(len, 64)
        y = ref.spmv(2, row_ptr, col_idx, a, x)
        lw = int(math.log2(n))
        assert list(y[:, 0]) == [_val(e) for e in row["expected"]["W%d" % (1 << lw)]]


def test_canonical_width_rule():
    L = np.array([0, 1, 2, 3, 4, 7, 8, 63, 64, 65, 4096])
    assert list(ref.canonical_log2w(L)) == [0, 0, 1, 1, 2, 2, 3, 5, 6, 6, 6]
    assert [ref.lib().oracle_canonical_log2w(int(v)) for v in L] == [0, 0, 1, 1, 2, 2, 3, 5, 6, 6, 6]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_small_integer_products_exact(K):
    rng = np.random.default_rng(40 + K)
    lengths = rng.integers(0, 300, 60)
    row_ptr, col_idx, _, _ = random_csr(60, 400, lengths, K, rng)
    a = np.zeros((K, col_idx.size))
    a[0] = rng.integers(-2 ** 20, 2 ** 20, col_idx.size)
    x = np.zeros((K, 400))
    x[0] = rng.integers(-2 ** 20, 2 ** 20, 400)
    dense_a = np.zeros((60, 400))
    rows = np.repeat(np.arange(60), np.diff(row_ptr))
    dense_a[rows, col_idx] = a[0]
    want = [int(sum(int(dense_a[i, j]) * int(x[0, j]) for j in range(400))) for i in range(60)]
    for lw in (None, np.zeros(60, dtype=np.uint8)):
        y = ref.spmv(K, row_ptr, col_idx, a, x, log2w=lw)
        assert [int(v) for v in y[0]] == want
        assert np.all(y[1:] == 0)


def _check_bound(K, row_ptr, col_idx, a, x, y, rows=None):
    ys, ss = exact.exact_row_products(row_ptr, col_idx, a, x, rows=rows)
    rows = range(len(row_ptr) - 1) if rows is None else rows
    worst = 0.0
    for r, i in enumerate(rows):
        got = exact.fixed_mp(y[:, i])
        L = int(row_ptr[i + 1] - row_ptr[i])
        ratio = exact.error_ratio(got, ys[r], ss[r], L, BITS[K])
        assert ratio <= 1.0, (K, i, ratio)
        worst = max(worst, ratio)
    return worst


def test_dd_bound_laplace2d_c0():
    row_ptr, col_idx, a = laplace2d_5pt(100, K=2, seed=0)
    assert row_ptr[-1] == 49600
    rng = np.random.default_rng(0)
    x = random_mp(10000, 2, rng)
    y = ref.spmv(2, row_ptr, col_idx, a, x)
    worst = _check_bound(2, row_ptr, col_idx, a, x, y)
    assert worst < 2.0 ** -3  # far inside the bound


@pytest.mark.parametrize("K", [2, 3, 4])
def test_bound_ragged_random(K):
    rng = np.random.default_rng(60 + K)
    lengths = np.concatenate([[0, 1, 2, 3, 64, 65, 127, 600], rng.integers(0, 200, 40)])
    row_ptr, col_idx, a, _ = random_csr(lengths.size, 700, lengths, K, rng)
    x = random_mp(700, K, rng)
    lw_max = np.array([min(10, int(math.log2(max(1, L)))) for L in lengths], dtype=np.uint8)
    for lw in (None, np.zeros(lengths.size, dtype=np.uint8), lw_max):
        y = ref.spmv(K, row_ptr, col_idx, a, x, log2w=lw)
        _check_bound(K, row_ptr, col_idx, a, x, y)
        assert np.all(y[:, 0] == 0)


def test_bad_lane_width_rejected():
    row_ptr = np.array([0, 3], dtype=np.int32)
    col_idx = np.arange(3, dtype=np.int32)
    a = np.ones((2, 3))
    x = np.ones((2, 3))
    with pytest.raises(ValueError):
        ref.spmv(2, row_ptr, col_idx, a, x, log2w=np.array([2], dtype=np.uint8))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_invariants_bitwise(K):
    rng = np.random.default_rng(80 + K)
    lengths = rng.integers(0, 150, 80)
    row_ptr, col_idx, a, _ = random_csr(80, 300, lengths, K, rng)
    x = random_mp(300, K, rng)
    y = ref.spmv(K, row_ptr, col_idx, a, x)
    # power-of-two scaling
    assert np.array_equal(ref.spmv(K, row_ptr, col_idx, a * 2.0 ** 37, x * 2.0 ** -11), y * 2.0 ** 26)
    # negation
    assert np.array_equal(ref.spmv(K, row_ptr, col_idx, -a, x), -y)
    # row permutation (rows keep their own order and lane width)
    perm = rng.permutation(80)
    L = np.diff(row_ptr)
    rp2 = np.concatenate([[0], np.cumsum(L[perm])]).astype(np.int32)
    seg = [np.arange(row_ptr[i], row_ptr[i + 1]) for i in perm]
    idx = np.concatenate(seg)
    y2 = ref.spmv(K, rp2, col_idx[idx], a[:, idx], x)
    assert np.array_equal(y2, y[:, perm])


@pytest.mark.parametrize("K", [2, 3, 4])
def test_complex_pins(K):
    rng = np.random.default_rng(90 + K)
    lengths = rng.integers(0, 100, 50)
    row_ptr, col_idx, a_re, a_im = random_csr(50, 200, lengths, K, rng, cplx=True)
    x_re = random_mp(200, K, rng)
    x_im = random_mp(200, K, rng)
    zero_a = np.zeros_like(a_re)
    zero_x = np.zeros_like(x_re)
    yr = ref.spmv(K, row_ptr, col_idx, a_re, x_re)
    cre, cim = ref.spmv(K, row_ptr, col_idx, a_re, x_re, a_im=zero_a, x_im=zero_x)
    assert np.array_equal(cre, yr) and np.all(cim == 0)
    # x -> i x  maps  y -> i y
    y_re, y_im = ref.spmv(K, row_ptr, col_idx, a_re, x_re, a_im=a_im, x_im=x_im)
    z_re, z_im = ref.spmv(K, row_ptr, col_idx, a_re, -x_im, a_im=a_im, x_im=x_re)
    assert np.array_equal(z_re, -y_im) and np.array_equal(z_im, y_re)
    # bounds on the real and imaginary parts (sum of |a_re||x_re| + |a_im||x_im| etc.)
    ys1, ss1 = exact.exact_row_products(row_ptr, col_idx, a_re, x_re)
    ys2, ss2 = exact.exact_row_products(row_ptr, col_idx, a_im, x_im)
    ys3, ss3 = exact.exact_row_products(row_ptr, col_idx, a_re, x_im)
    ys4, ss4 = exact.exact_row_products(row_ptr, col_idx, a_im, x_re)
    for i in range(50):
        L = int(row_ptr[i + 1] - row_ptr[i])
        assert exact.within_bound(exact.fixed_mp(y_re[:, i]), ys1[i] - ys2[i], ss1[i] + ss2[i], L + 1, BITS[K])
        assert exact.within_bound(exact.fixed_mp(y_im[:, i]), ys3[i] + ys4[i], ss3[i] + ss4[i], L + 1, BITS[K])
