"""GPU checks of the device transpose (C ABI mp_csr_transpose) and A^T v built on it.

* Pattern and values equal the oracle's stable transpose bit for bit: square and
  rectangular ragged matrices with empty rows and columns, binary64 / DD / QD values,
  complex values, an empty matrix, and the full n = 1e6 power-law pattern (27e6 nnz).
* A^T v = SpMV of the transpose equals the oracle's SpMV of its transpose bitwise
  (plan-free and planned), including the 5x5 example of Sec. 3.
* Argument checks: overlapping outputs are refused.
"""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import random_csr, random_mp, sqrt2_vector, csr_from_dense, paper_example_5x5, powerlaw_pattern

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def same_transpose(mp, row_ptr, col_idx, a, n_cols, a_im=None, what=""):
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    At, at, at_im = mp.mp_csr_transpose(A, dev(a), dev(a_im) if a_im is not None else None)
    rpt, cit, want = ref.transpose(row_ptr, col_idx, a, n_cols=n_cols)
    assert np.array_equal(host(At.row_ptr), rpt), what
    assert np.array_equal(host(At.col_idx), cit), what
    assert_same_values(host(at), want, what + " values")
    if a_im is not None:
        assert_same_values(host(at_im), ref.transpose(row_ptr, col_idx, a_im, n_cols=n_cols)[2], what + " im")
    return A, At, at


@pytest.mark.parametrize("shape", [(700, 700), (300, 900), (900, 250)])
def test_transpose_matches_oracle(mp, shape):
    n, m = shape
    rng = np.random.default_rng(n * 7 + m)
    lengths = np.concatenate([[0, 1, min(600, m), 0], rng.integers(0, 40, n - 4)])
    row_ptr, col_idx, a4, a4i = random_csr(n, m, lengths, 4, rng, cplx=True)
    same_transpose(mp, row_ptr, col_idx, np.ascontiguousarray(a4[0]), m, what="binary64")
    same_transpose(mp, row_ptr, col_idx, np.ascontiguousarray(a4[:2]), m, what="DD")
    same_transpose(mp, row_ptr, col_idx, a4, m, a_im=a4i, what="QD complex")


def test_transpose_empty_and_powerlaw(mp):
    import torch
    A = mp.Csr(torch.zeros(4, dtype=torch.int32, device="cuda"), torch.zeros(0, dtype=torch.int32, device="cuda"),
               n_cols=6)
    At, at, _ = mp.mp_csr_transpose(A, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert np.array_equal(host(At.row_ptr), np.zeros(7, np.int32))
    row_ptr, col_idx = powerlaw_pattern(n=1_000_000, seed=1)
    a = np.random.default_rng(3).uniform(-1, 1, col_idx.size)
    same_transpose(mp, row_ptr, col_idx, a, row_ptr.size - 1, what="power-law")


@pytest.mark.parametrize("K", [2, 4])
def test_transpose_spmv(mp, K):
    import torch
    rng = np.random.default_rng(70 + K)
    n, m = 1200, 800
    lengths = np.concatenate([[0, 3000 % m, 1], rng.integers(0, 30, n - 3)])
    row_ptr, col_idx, a, _ = random_csr(n, m, lengths, K, rng)
    v = random_mp(n, K, rng)
    A, At, at = same_transpose(mp, row_ptr, col_idx, a, m, what="K=%d" % K)
    rpt, cit, want_at = ref.transpose(row_ptr, col_idx, a, n_cols=m)
    for plan in (None, mp.mp_plan_create(At, K), mp.mp_plan_create(At, K, False, 2, 8)):
        y = torch.full((K, m), float("nan"), dtype=torch.float64, device="cuda")
        mp.SPMV[(K, False)](At, at, dev(v), y, plan=plan)
        torch.cuda.synchronize()
        lw = None if plan is None else plan.row_log2w()
        assert_same_values(host(y), ref.spmv(K, rpt, cit, want_at, v, log2w=lw), "A^T v")
    # the paper's 5x5 example
    r5, c5, v5 = csr_from_dense(paper_example_5x5())
    a5 = np.zeros((K, v5.size))
    a5[0] = v5
    A5, At5, at5 = same_transpose(mp, r5, c5, a5, 5, what="5x5")
    x5 = sqrt2_vector(5, K)
    y = torch.empty((K, 5), dtype=torch.float64, device="cuda")
    mp.SPMV[(K, False)](At5, at5, dev(x5), y)
    rt, ct, vt = ref.transpose(r5, c5, a5, n_cols=5)
    assert_same_values(host(y), ref.spmv(K, rt, ct, vt, x5), "5x5 A^T v")


def test_transpose_alias_rejected(mp):
    import torch
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    a = dev(vals)
    buf = torch.zeros(32, dtype=torch.int32, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    from paper_2412_17510_amd._binding import _lib, _ptr
    import ctypes
    st = _lib.mp_csr_transpose(ctypes.byref(A.c), 1, _ptr(a), None, _ptr(buf[:6]), _ptr(buf[4:12]), _ptr(out), None,
                               None)
    assert st == -2
