"""Pins of the oracle's transpose (for A^T v, Sec. 3; CPU only).

* Pattern and values equal scipy's CSR transpose (sorted indices) bit for bit, for
  square and rectangular matrices with empty rows and columns and K = 1..4 components.
* Transposing twice gives A back exactly.
* The 5x5 example: A^T v with v = sqrt(2)[1..5] is sqrt(2)[25, 6, 17, -28, 32] to the
  K-component precision (tests/golden/csr_5x5.json).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref, exact
from workloads import random_csr, sqrt2_vector, csr_from_dense, paper_example_5x5

scipy_sparse = pytest.importorskip("scipy.sparse")


@pytest.mark.parametrize("K", [1, 2, 4])
@pytest.mark.parametrize("shape", [(300, 300), (200, 500), (500, 120)])
def test_matches_scipy_and_round_trips(K, shape):
    n, m = shape
    rng = np.random.default_rng(K * 1000 + n + m)
    lengths = rng.integers(0, 30, n)
    lengths[::17] = 0
    row_ptr, col_idx, a, _ = random_csr(n, m, lengths, max(K, 2), rng)
    a = a[:K] if K > 1 else a[0]
    rpt, cit, at = ref.transpose(row_ptr, col_idx, a, n_cols=m)
    comps = a.reshape(-1, col_idx.size)
    at2 = at.reshape(-1, col_idx.size)
    for c in range(comps.shape[0]):
        T = scipy_sparse.csr_matrix((comps[c], col_idx, row_ptr), shape=(n, m)).T.tocsr()
        T.sort_indices()
        assert np.array_equal(rpt, T.indptr) and np.array_equal(cit, T.indices)
        assert np.array_equal(at2[c], T.data)
    rp2, ci2, a2 = ref.transpose(rpt, cit, at, n_cols=n)
    assert np.array_equal(rp2, row_ptr) and np.array_equal(ci2, col_idx) and np.array_equal(a2, a)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_5x5_transpose_times_sqrt2(golden_dir, K):
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        g = json.load(f)
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    a = np.zeros((K, vals.size))
    a[0] = vals
    rpt, cit, at = ref.transpose(row_ptr, col_idx, a, n_cols=5)
    y = ref.spmv(K, rpt, cit, at, sqrt2_vector(5, K))
    mt = g["ATv_over_sqrt2_for_v_eq_sqrt2_times_1_to_n"]
    for i in range(5):
        got = exact.mp_value(y[:, i])
        tol = Fraction(abs(mt[i]) * 16, 2 ** (53 * K - 6))
        lo, hi = abs(got) - tol, abs(got) + tol
        assert got * mt[i] > 0 and lo * lo <= 2 * mt[i] * mt[i] <= hi * hi
