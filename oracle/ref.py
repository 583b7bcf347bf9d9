"""ctypes front end of the CPU oracle (libmpref.so).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
module.  Arrays follow the multi-component layout of the paper (Sec. 3): a
K-component array of length L is a C-contiguous (K, L) float64 array.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_eft.argtypes = [ctypes.c_int, i64, P, P, P, P]
        L.oracle_elementwise.argtypes = [ctypes.c_int, ctypes.c_int, i64, P, P, P]
        L.oracle_renorm5.argtypes = [i64, P, P]
        L.oracle_spmv.argtypes = [ctypes.c_int, i64, i64, i64, P, P, P, P, P, P, P, P, P, i64, P, ctypes.c_int]
        L.oracle_spmv_dmat.argtypes = [ctypes.c_int, i64, i64, i64, P, P, P, P, P, P, i64, P, ctypes.c_int]
        L.oracle_spmv_dmat_complex.argtypes = [ctypes.c_int, i64, i64, i64, P, P, P, P, P, P, P, P, P, i64, P,
                                               ctypes.c_int]
        L.oracle_transpose.argtypes = [i64, i64, i64, ctypes.c_int, P, P, P, P, P, P]
        L.oracle_coo_to_csr.argtypes = [i64, i64, i64, P, P, ctypes.c_int, P, P, P, P]
        L.oracle_canonical_log2w.argtypes = [i64]
        L.oracle_num_threads.argtypes = []
        L.oracle_exact_residual.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, P, P, P, P, P, P, P]
        L.oracle_exact_residual.restype = ctypes.c_int
        for name in ("oracle_eft", "oracle_elementwise", "oracle_renorm5", "oracle_spmv", "oracle_spmv_dmat",
                     "oracle_spmv_dmat_complex", "oracle_transpose", "oracle_coo_to_csr",
                     "oracle_canonical_log2w", "oracle_num_threads"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def eft(which, a, b):
    """which: 'two_sum' | 'quick_two_sum' | 'two_prod' -> (s, e) arrays."""
    code = {"two_sum": 0, "quick_two_sum": 1, "two_prod": 2}[which]
    a, b = _f64(a), _f64(b)
    s = np.empty_like(a)
    e = np.empty_like(a)
    assert lib().oracle_eft(code, a.size, _p(a), _p(b), _p(s), _p(e)) == 0
    return s, e


def elementwise(K, op, x, y):
    """op: 'add' | 'mul' | 'mul_d' (K-component times binary64, Algs 3-5).  x (K, n);
    y (K, n), or (n,) for mul_d."""
    code = {"add": 0, "mul": 1, "mul_d": 2}[op]
    x, y = _f64(x), _f64(y)
    n = x.shape[1]
    r = np.zeros((K, n))
    assert lib().oracle_elementwise(K, code, n, _p(x), _p(y), _p(r)) == 0
    return r


def renorm5(c):
    c = _f64(c)
    n = c.shape[1]
    r = np.zeros((4, n))
    lib().oracle_renorm5(n, _p(c), _p(r))
    return r


def canonical_log2w(lengths):
    lengths = np.asarray(lengths, dtype=np.int64)
    out = np.zeros(lengths.size, dtype=np.uint8)
    L = np.maximum(lengths, 1)
    # largest l <= 6 with 2^l <= len
    lw = np.floor(np.log2(L)).astype(np.int64)
    lw = np.where((1 << (lw + 1)) <= L, lw + 1, lw)
    lw = np.where((1 << lw) > L, lw - 1, lw)
    out[:] = np.minimum(6, lw)
    return out


def spmv(K, row_ptr, col_idx, a_re, x_re, a_im=None, x_im=None, log2w=None, rows=None,
         n_cols=None, nthreads=0):
    """y = A x in K-component arithmetic (Sec. 3).  Returns y_re or (y_re, y_im).

    log2w: per-row lane-width exponents (None = canonical order).  rows: subset of rows
    to compute (others are returned as NaN).  nthreads: OpenMP threads (0 = default).
    """
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.size - 1
    nnz = col_idx.size
    if n_cols is None:
        n_cols = x_re.shape[1]
    a_re, a_im, x_re, x_im = _f64(a_re), _f64(a_im), _f64(x_re), _f64(x_im)
    assert a_re.shape == (K, nnz) and x_re.shape == (K, n_cols)
    cplx = a_im is not None
    y_re = np.full((K, n), np.nan)
    y_im = np.full((K, n), np.nan) if cplx else None
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    rc = lib().oracle_spmv(K, n, n_cols, nnz, _p(row_ptr), _p(col_idx), _p(lw),
                           _p(a_re), _p(a_im), _p(x_re), _p(x_im), _p(y_re), _p(y_im),
                           0 if sel is None else sel.size, _p(sel), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_spmv: invalid argument (lane width larger than the row?)")
    return (y_re, y_im) if cplx else y_re


def spmv_dmat(K, row_ptr, col_idx, a, x, log2w=None, n_cols=None, rows=None, nthreads=0):
    """y = A x with a binary64 matrix a (nnz values) and a K-component x (Algs 3-5 for
    the products, the order of spmv).  Returns y (K, n); rows: optional subset (the
    other rows are NaN)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.size - 1
    nnz = col_idx.size
    a, x = _f64(a), _f64(x)
    if n_cols is None:
        n_cols = x.shape[1]
    assert a.shape == (nnz,) and x.shape == (K, n_cols)
    y = np.full((K, n), np.nan)
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    rc = lib().oracle_spmv_dmat(K, n, n_cols, nnz, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(x), _p(y),
                                0 if sel is None else sel.size, _p(sel), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_spmv_dmat: invalid argument")
    return y


def spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im, log2w=None, n_cols=None, rows=None,
                      nthreads=0):
    """Complex y = A x with a binary64 complex matrix (a_re, a_im: nnz values each) and a
    K-component complex x (Eq. 3, products by Algs 3-5, the order of spmv).  Returns
    (y_re, y_im), each (K, n); rows: optional subset (the other rows are NaN)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.size - 1
    nnz = col_idx.size
    a_re, a_im, x_re, x_im = _f64(a_re), _f64(a_im), _f64(x_re), _f64(x_im)
    if n_cols is None:
        n_cols = x_re.shape[1]
    assert a_re.shape == (nnz,) and a_im.shape == (nnz,)
    assert x_re.shape == (K, n_cols) and x_im.shape == (K, n_cols)
    y_re = np.full((K, n), np.nan)
    y_im = np.full((K, n), np.nan)
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    rc = lib().oracle_spmv_dmat_complex(K, n, n_cols, nnz, _p(row_ptr), _p(col_idx), _p(lw), _p(a_re), _p(a_im),
                                        _p(x_re), _p(x_im), _p(y_re), _p(y_im), 0 if sel is None else sel.size,
                                        _p(sel), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_spmv_dmat_complex: invalid argument")
    return y_re, y_im


def transpose(row_ptr, col_idx, a, n_cols=None):
    """CSR of A^T (stable: row j of A^T lists column j of A in increasing row order) and
    the values permuted with it.  a: (ncomp, nnz) or (nnz,).  Returns (row_ptr_t,
    col_idx_t, a_t) with a_t shaped like a."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.size - 1
    nnz = col_idx.size
    if n_cols is None:
        n_cols = int(col_idx.max()) + 1 if nnz else n
    a = _f64(a)
    a2 = a.reshape(-1, nnz)
    rpt = np.empty(n_cols + 1, dtype=np.int32)
    cit = np.empty(nnz, dtype=np.int32)
    at = np.empty_like(a2)
    assert lib().oracle_transpose(n, n_cols, nnz, a2.shape[0], _p(row_ptr), _p(col_idx), _p(a2), _p(rpt), _p(cit),
                                  _p(at)) == 0
    return rpt, cit, at.reshape(a.shape)


def coo_to_csr(n_rows, n_cols, row, col, v):
    """CSR of a COO matrix (0-based coordinates): elements ordered by row, then column;
    equal coordinates keep their input order.  v: (ncomp, nnz) or (nnz,).  Returns
    (row_ptr, col_idx, a) with a shaped like v; raises ValueError for a coordinate
    outside the matrix."""
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    nnz = row.size
    v = _f64(v)
    v2 = v.reshape(-1, nnz) if nnz else v.reshape(1 if v.ndim < 2 else v.shape[0], 0)
    rp = np.empty(n_rows + 1, dtype=np.int32)
    ci = np.empty(nnz, dtype=np.int32)
    a = np.empty_like(v2)
    st = lib().oracle_coo_to_csr(n_rows, n_cols, nnz, _p(row), _p(col), v2.shape[0], _p(v2), _p(rp), _p(ci), _p(a))
    if st == -2:
        raise ValueError("coordinate outside the %d x %d matrix" % (n_rows, n_cols))
    assert st == 0
    return rp, ci, a.reshape(v.shape)


def exact_residual(row_ptr, col_idx, a, b, x, want_vector=False):
    """Exact residual of A x = b (oracle_exact_residual): a (Ka, nnz) or (nnz,), b and x
    (Kx, n), every value the exact sum of its stored components.  Returns a dict with
    rr_upper >= ||b - A x||^2, bb_lower <= ||b||^2, relres_upper = sqrt of their ratio
    (rounded up), the informational rr / bb, and r (the exact residual rounded to
    binary64) when want_vector."""
    a = _f64(a)
    a2 = a.reshape(1, -1) if a.ndim == 1 else a
    b, x = _f64(b), _f64(x)
    n = b.shape[1]
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    norms = np.zeros(4)
    r = np.zeros(n) if want_vector else None
    st = lib().oracle_exact_residual(a2.shape[0], b.shape[0], n, ci.size, _p(rp), _p(ci), _p(a2), _p(b), _p(x),
                                     _p(r), _p(norms))
    if st != 0:
        raise ValueError("oracle_exact_residual failed (%d)" % st)
    ratio = norms[0] / norms[1] if norms[1] > 0 else (0.0 if norms[0] == 0 else np.inf)
    out = {"rr_upper": float(norms[0]), "bb_lower": float(norms[1]),
           "relres_upper": float(np.sqrt(ratio) * (1.0 + 2.0 ** -50)), "rr": float(norms[2]), "bb": float(norms[3])}
    if want_vector:
        out["r"] = r
    return out


def num_threads():
    return lib().oracle_num_threads()


def loaded_path():
    return os.path.abspath(_build.LIB)


# ---------------------------------------------------------------------------------------
# Krylov layer (DD): dot, division, Jacobi inverse diagonal, CG, BiCGSTAB
# ---------------------------------------------------------------------------------------

class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rr_true", ctypes.c_double * 2), ("bb", ctypes.c_double * 2)]


def _krylov_sigs():
    L = lib()
    if getattr(L, "_krylov_ready", False):
        return L
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    L.oracle_dd_dot.argtypes = [i64, P, P, P]
    L.oracle_dd_div.argtypes = [P, P, P]
    L.oracle_jacobi_minv.argtypes = [i64, P, P, P, P]
    for f in (L.oracle_cg, L.oracle_bicgstab, L.oracle_cgs, L.oracle_gpbicg):
        f.argtypes = [i64, i64, P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SolveInfo), P]
        f.restype = ctypes.c_int
    L.oracle_bicg.argtypes = [i64, i64, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                              ctypes.POINTER(SolveInfo), P]
    L.oracle_bicg.restype = ctypes.c_int
    for f in (L.oracle_cg_k, L.oracle_bicgstab_k, L.oracle_cgs_k, L.oracle_gpbicg_k):
        f.argtypes = [ctypes.c_int, i64, i64, P, P, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                      ctypes.POINTER(SolveInfo), P]
        f.restype = ctypes.c_int
    L.oracle_bicg_k.argtypes = [ctypes.c_int, i64, i64, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(SolveInfo), P]
    L.oracle_bicg_k.restype = ctypes.c_int
    L.oracle_mp_div.argtypes = [ctypes.c_int, P, P, P]
    L.oracle_mp_dot.argtypes = [ctypes.c_int, i64, P, P, P]
    L.oracle_mp_le.argtypes = [ctypes.c_int, P, P]
    L.oracle_mp_le.restype = ctypes.c_int
    L._krylov_ready = True
    return L


def dd_dot(x, y):
    L = _krylov_sigs()
    x, y = _f64(x), _f64(y)
    out = np.zeros(2)
    L.oracle_dd_dot(x.shape[1], _p(x), _p(y), _p(out))
    return out


def dd_div(a, b):
    L = _krylov_sigs()
    a, b = _f64(a), _f64(b)
    out = np.zeros(2)
    L.oracle_dd_div(_p(a), _p(b), _p(out))
    return out


def jacobi_minv(row_ptr, col_idx, a_hi):
    L = _krylov_sigs()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a_hi = _f64(a_hi)
    n = row_ptr.size - 1
    out = np.zeros(n)
    L.oracle_jacobi_minv(n, _p(row_ptr), _p(col_idx), _p(a_hi), _p(out))
    return out


def _solve(fn, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history):
    L = _krylov_sigs()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a, b = _f64(a), _f64(b)
    n = row_ptr.size - 1
    x = np.array(x0, dtype=np.float64, order="C", copy=True) if x0 is not None else np.zeros((2, n))
    minv = jacobi_minv(row_ptr, col_idx, a[0]) if precond == "jacobi" else None
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    hist = np.zeros(2 * (max_iter + 1)) if history else None
    info = SolveInfo()
    getattr(L, fn)(n, col_idx.size, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(b), _p(x), _p(minv),
                   float(rtol), int(max_iter), ctypes.byref(info), _p(hist))
    out = {"status": info.status, "iters": info.iters, "restarts": info.restarts,
           "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:])}
    if history:
        out["history"] = hist[:2 * (info.iters + 1)].reshape(-1, 2)
    return x, out


def mp_div(K, a, b):
    """K-component a / b (DD: Dekker; TD/QD: long division).  Returns K components."""
    L = _krylov_sigs()
    a, b = _f64(a), _f64(b)
    out = np.zeros(K)
    L.oracle_mp_div(K, _p(a), _p(b), _p(out))
    return out


def mp_le(K, a, b):
    """The solvers' stop comparison a <= b of K-component values (lexicographic)."""
    L = _krylov_sigs()
    return bool(L.oracle_mp_le(K, _p(_f64(a)), _p(_f64(b))))


def mp_dot(K, x, y):
    """K-component dot product of (K, n) vectors with the fixed tree."""
    L = _krylov_sigs()
    x, y = _f64(x), _f64(y)
    out = np.zeros(K)
    L.oracle_mp_dot(K, x.shape[1], _p(x), _p(y), _p(out))
    return out


def _solve_k(fn, K, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history):
    L = _krylov_sigs()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a, b = _f64(a), _f64(b)
    n = row_ptr.size - 1
    assert a.shape == (K, col_idx.size) and b.shape == (K, n)
    x = np.array(x0, dtype=np.float64, order="C", copy=True) if x0 is not None else np.zeros((K, n))
    minv = jacobi_minv(row_ptr, col_idx, a[0]) if precond == "jacobi" else None
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    hist = np.zeros(2 * (max_iter + 1)) if history else None
    info = SolveInfo()
    getattr(L, fn)(K, n, col_idx.size, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(b), _p(x), _p(minv),
                   float(rtol), int(max_iter), ctypes.byref(info), _p(hist))
    out = {"status": info.status, "iters": info.iters, "restarts": info.restarts,
           "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:])}
    if history:
        out["history"] = hist[:2 * (info.iters + 1)].reshape(-1, 2)
    return x, out


def cg_k(K, row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
         history=False):
    """K-component preconditioned CG (oracle; K = 2 is cg).  a, b, x: (K, len)."""
    return _solve_k("oracle_cg_k", K, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def bicgstab_k(K, row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
               history=False):
    """K-component BiCGSTAB (oracle; K = 2 is bicgstab).  a, b, x: (K, len)."""
    return _solve_k("oracle_bicgstab_k", K, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def cgs_k(K, row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
          history=False):
    """K-component CGS (oracle; K = 2 is cgs).  a, b, x: (K, len)."""
    return _solve_k("oracle_cgs_k", K, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def gpbicg_k(K, row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
             history=False):
    """K-component GPBiCG (oracle; K = 2 is gpbicg).  a, b, x: (K, len)."""
    return _solve_k("oracle_gpbicg_k", K, row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def bicg_k(K, row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
           log2w_t=None, history=False):
    """K-component BiCG (oracle; K = 2 is bicg); A^T from the oracle's stable transpose."""
    L = _krylov_sigs()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a, b = _f64(a), _f64(b)
    n = row_ptr.size - 1
    assert a.shape == (K, col_idx.size) and b.shape == (K, n)
    rpt, cit, at = transpose(row_ptr, col_idx, a, n_cols=n)
    x = np.array(x0, dtype=np.float64, order="C", copy=True) if x0 is not None else np.zeros((K, n))
    minv = jacobi_minv(row_ptr, col_idx, a[0]) if precond == "jacobi" else None
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    lwt = None if log2w_t is None else np.ascontiguousarray(log2w_t, dtype=np.uint8)
    hist = np.zeros(2 * (max_iter + 1)) if history else None
    info = SolveInfo()
    L.oracle_bicg_k(K, n, col_idx.size, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(rpt), _p(cit), _p(lwt), _p(at),
                    _p(b), _p(x), _p(minv), float(rtol), int(max_iter), ctypes.byref(info), _p(hist))
    out = {"status": info.status, "iters": info.iters, "restarts": info.restarts,
           "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:])}
    if history:
        out["history"] = hist[:2 * (info.iters + 1)].reshape(-1, 2)
    return x, out


def cg(row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
       history=False):
    """DD preconditioned CG (oracle).  Returns (x, info dict)."""
    return _solve("oracle_cg", row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def bicgstab(row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
             history=False):
    """DD BiCGSTAB (oracle).  Returns (x, info dict)."""
    return _solve("oracle_bicgstab", row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def cgs(row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
        history=False):
    """DD CGS (oracle).  Returns (x, info dict)."""
    return _solve("oracle_cgs", row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def gpbicg(row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
           history=False):
    """DD GPBiCG (oracle).  Returns (x, info dict)."""
    return _solve("oracle_gpbicg", row_ptr, col_idx, a, b, x0, precond, rtol, max_iter, log2w, history)


def bicg(row_ptr, col_idx, a, b, x0=None, precond="jacobi", rtol=1e-28, max_iter=10000, log2w=None,
         log2w_t=None, history=False):
    """DD BiCG (oracle); A^T from the oracle's stable transpose.  Returns (x, info dict)."""
    L = _krylov_sigs()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a, b = _f64(a), _f64(b)
    n = row_ptr.size - 1
    rpt, cit, at = transpose(row_ptr, col_idx, a, n_cols=n)
    x = np.array(x0, dtype=np.float64, order="C", copy=True) if x0 is not None else np.zeros((2, n))
    minv = jacobi_minv(row_ptr, col_idx, a[0]) if precond == "jacobi" else None
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    lwt = None if log2w_t is None else np.ascontiguousarray(log2w_t, dtype=np.uint8)
    hist = np.zeros(2 * (max_iter + 1)) if history else None
    info = SolveInfo()
    L.oracle_bicg(n, col_idx.size, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(rpt), _p(cit), _p(lwt), _p(at),
                  _p(b), _p(x), _p(minv), float(rtol), int(max_iter), ctypes.byref(info), _p(hist))
    out = {"status": info.status, "iters": info.iters, "restarts": info.restarts,
           "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:])}
    if history:
        out["history"] = hist[:2 * (info.iters + 1)].reshape(-1, 2)
    return x, out


class IrInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("rr_true", ctypes.c_double * 2), ("bb", ctypes.c_double * 2)]


def ir(row_ptr, col_idx, a, b, x0=None, inner="fp64", precond="jacobi", rtol=1e-28, inner_rtol=1e-8,
       inner_max_iter=1000, max_outer=50, max_iter=10000, log2w=None, m_values=None):
    """Mixed-precision iterative refinement (oracle).  Returns (x, info dict).

    ``m_values``: optional inner preconditioner M given by its binary64 values on A's
    pattern (z = M r); the stall fallback is then Jacobi DD CG."""
    L = _krylov_sigs()
    if not getattr(L, "_ir_ready", False):
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_ir.argtypes = [i64, i64, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(IrInfo)]
        L.oracle_ir.restype = ctypes.c_int
        L._ir_ready = True
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    a, b = _f64(a), _f64(b)
    n = row_ptr.size - 1
    x = np.array(x0, dtype=np.float64, order="C", copy=True) if x0 is not None else np.zeros((2, n))
    lw = None if log2w is None else np.ascontiguousarray(log2w, dtype=np.uint8)
    mv = None if m_values is None else _f64(m_values)
    if mv is not None and mv.shape != (col_idx.size,):
        raise ValueError("m_values must hold one value per stored element")
    info = IrInfo()
    L.oracle_ir(n, col_idx.size, _p(row_ptr), _p(col_idx), _p(lw), _p(a), _p(b), _p(x), int(inner == "fp32"),
                int(precond == "jacobi"), _p(mv), float(rtol), float(inner_rtol), int(inner_max_iter), int(max_outer),
                int(max_iter), ctypes.byref(info))
    return x, {"status": info.status, "iters": info.iters, "outer_iters": info.outer_iters,
               "fell_back": info.fell_back, "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:])}
