"""GPU checks of the device transpose (C ABI mp_csr_transpose), A^T v built on it, and COO -> CSR.

* Pattern and values equal the oracle's stable transpose bit for bit: square and
  rectangular ragged matrices with empty rows and columns, binary64 / DD / QD values,
  complex values, an empty matrix, and the full n = 1e6 power-law pattern (27e6 nnz).
* A^T v = SpMV of the transpose equals the oracle's SpMV of its transpose bitwise
  (plan-free and planned), including the 5x5 example of Sec. 3.
* Argument checks: overlapping outputs are refused.
* COO -> CSR (C ABI mp_coo_to_csr) equals the oracle's conversion bit for bit on
  shuffled random COO with duplicate coordinates (binary64, DD, QD, complex DD) and
  reproduces the paper's printed 5x5 CSR arrays from its COO arrays; empty input;
  coordinates outside the matrix and overlapping buffers are refused.
"""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import configs
from workloads import random_csr, random_mp, sqrt2_vector, csr_from_dense, paper_example_5x5

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
    row_ptr, col_idx = configs.c1_pattern()
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


def coo_int(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


@pytest.mark.parametrize("ncomp,cplx", [(1, False), (2, False), (4, False), (2, True)])
def test_coo_to_csr_matches_oracle(mp, ncomp, cplx):
    """Device COO -> CSR equals the oracle's bit for bit on shuffled random COO with
    planted duplicate coordinates (their input order kept), over a rectangular matrix
    with empty rows; the result multiplies like the oracle's CSR."""
    rng = np.random.default_rng(40 + ncomp + 10 * cplx)
    n, m, nnz = 900, 700, 12000
    row = rng.integers(0, n, nnz).astype(np.int32)
    row[row % 13 == 0] += 1                          # some empty rows
    row = np.minimum(row, n - 1).astype(np.int32)
    col = rng.integers(0, m, nnz).astype(np.int32)
    dup = rng.choice(nnz, 600, replace=False)
    row[dup[300:]], col[dup[300:]] = row[dup[:300]], col[dup[:300]]
    v = rng.standard_normal((ncomp, nnz))
    vi = rng.standard_normal((ncomp, nnz)) if cplx else None
    A, a_re, a_im = mp.mp_coo_to_csr(n, m, coo_int(row), coo_int(col), dev(v), dev(vi) if cplx else None)
    rp, ci, want = ref.coo_to_csr(n, m, row, col, v)
    assert np.array_equal(host(A.row_ptr), rp) and np.array_equal(host(A.col_idx), ci)
    assert_same_values(host(a_re), want, "coo values")
    if cplx:
        assert_same_values(host(a_im), ref.coo_to_csr(n, m, row, col, vi)[2], "coo imaginary values")
    if ncomp == 2 and not cplx:
        x = random_mp(m, 2, rng)
        import torch
        y = torch.empty((2, n), dtype=torch.float64, device="cuda")
        mp.mpspmv_csr_dd(A, a_re, dev(x), y)
        assert_same_values(host(y), ref.spmv(2, rp, ci, want, x, n_cols=m), "SpMV of the converted matrix")


def test_coo_to_csr_paper_example_empty_and_errors(mp, golden_dir):
    import json
    import os
    import torch
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        g = json.load(f)
    perm = np.random.default_rng(2).permutation(8)
    A, a, _ = mp.mp_coo_to_csr(5, 5, coo_int(np.array(g["coo_row"])[perm]), coo_int(np.array(g["coo_col"])[perm]),
                               dev(np.array(g["coo_data"], float)[perm]))
    assert host(A.row_ptr).tolist() == g["csr_indptr"] and host(A.col_idx).tolist() == g["csr_indices"]
    assert host(a).tolist() == g["csr_data"]
    # empty
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    A0, a0, _ = mp.mp_coo_to_csr(4, 3, e, e, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert host(A0.row_ptr).tolist() == [0, 0, 0, 0, 0] and A0.nnz == 0
    # a coordinate outside the matrix, and an output overlapping an input
    with pytest.raises(mp.MpError) as ei:
        mp.mp_coo_to_csr(5, 5, coo_int([0, 5]), coo_int([1, 1]), dev(np.ones(2)))
    assert ei.value.status == -1
    rows = coo_int([0, 1, 2])
    v = dev(np.ones(3))
    with pytest.raises(mp.MpError) as ei:
        mp._check(mp._lib.mp_coo_to_csr(3, 3, 3, mp._ptr(rows), mp._ptr(rows), 1, mp._ptr(v), None,
                                        mp._ptr(rows), mp._ptr(rows), mp._ptr(v), None, None), "mp_coo_to_csr")
    assert ei.value.status == -2
