"""Thin ctypes binding of libmpsparse.so (the C ABI declared in include/mpsparse.h).

Argument marshalling only: tensors are torch CUDA tensors (device memory), streams
are torch CUDA streams, and every computation runs in the library's HIP kernels.
Multi-component arrays are C-contiguous float64 tensors of shape (K, L) (component
0 leading), exactly the K*L block layout of the C ABI.

Importing this module fails loudly if the library has not been built; there is no
fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsparse.so")

MP_OK = 0
STATUS_NAMES = {0: "MP_OK", -1: "MP_ERR_INVALID_ARG", -2: "MP_ERR_ALIAS", -3: "MP_ERR_HIP",
                -4: "MP_ERR_NO_MEMORY", -5: "MP_ERR_NOT_CONVERGED", -6: "MP_ERR_BREAKDOWN",
                -7: "MP_ERR_UNSUPPORTED"}


class MpError(RuntimeError):
    def __init__(self, status, func, message):
        self.status = status
        super().__init__("%s returned %s: %s" % (func, STATUS_NAMES.get(status, status), message))


class mp_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class mp_plan_opts(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int32), ("max_log2w", ctypes.c_int32), ("tile_nnz", ctypes.c_int32),
                ("row_groups", ctypes.c_int32)]


class mp_solve_opts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("inner", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("inner_max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32)]


class mp_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("rr_true", ctypes.c_double * 2), ("bb", ctypes.c_double * 2),
                ("relres", ctypes.c_double), ("seconds", ctypes.c_double), ("fell_back", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


PRECOND = {"none": 0, "jacobi": 1, "learned": 2}
INNER = {"fp64": 0, "fp32": 1}

if not os.path.exists(LIB_PATH):
    raise ImportError("libmpsparse.so is not built (expected at %s); run __graft_entry__.build()" % LIB_PATH)

# torch supplies device memory and streams, and ships its own HIP runtime under the
# soname the library links against (libamdhip64.so.7): whichever copy loads first serves
# the process.  Import torch first so that the library and torch share torch's runtime.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I = ctypes.c_int32
_CSR = ctypes.POINTER(mp_csr)

_SIGS = {
    "mp_last_error": ([], ctypes.c_char_p),
    "mp_version": ([], ctypes.c_char_p),
    "mp_csr_validate": ([_CSR, _P], ctypes.c_int),
    "mp_measure_rate": ([_I, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "mp_plan_create": ([_CSR, _I, _I, ctypes.POINTER(mp_plan_opts), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "mp_plan_create_explicit": ([_CSR, _I, _I, _P, _I, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "mp_plan_autotune": ([_CSR, _I, _I, _P, _P, _P, _P, _P, _P, _I, _P, ctypes.POINTER(_P),
                          ctypes.POINTER(mp_plan_opts)], ctypes.c_int),
    "mp_plan_destroy": ([_P], ctypes.c_int),
    "mp_plan_row_log2w": ([_P, _P], ctypes.c_int),
    "mp_plan_info": ([_P] + [ctypes.POINTER(_I)] * 5, ctypes.c_int),
}
_SIGS["mpspmv_workspace_bytes"] = ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int)
for _name in ("mpspmv_csr_dd", "mpspmv_csr_td", "mpspmv_csr_qd", "mpspmv_csr_dd_d", "mpspmv_csr_td_d",
              "mpspmv_csr_qd_d"):
    _SIGS[_name] = ([_CSR, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int)
for _name in ("mpspmv_csr_dd_complex", "mpspmv_csr_td_complex", "mpspmv_csr_qd_complex", "mpspmv_csr_dd_d_complex",
              "mpspmv_csr_td_d_complex", "mpspmv_csr_qd_d_complex"):
    _SIGS[_name] = ([_CSR, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int)

_SIGS["mpspmv_csr_dd_noalloc"] = ([_CSR, _P, _P, _P, _P, _P], ctypes.c_int)
_SIGS["mpvec_dd_sub"] = ([ctypes.c_int64, _P, _P, _P, _P], ctypes.c_int)
_SIGS["mpkrylov_workspace_bytes"] = ([_CSR, ctypes.POINTER(mp_solve_opts), ctypes.POINTER(ctypes.c_size_t)],
                                     ctypes.c_int)
for _name in ("mpkrylov_cg", "mpkrylov_bicgstab", "mpkrylov_cgs", "mpkrylov_gpbicg", "mpkrylov_ir"):
    _SIGS[_name] = ([_CSR, _P, _P, _P, ctypes.POINTER(mp_solve_opts), _P, _P, ctypes.c_size_t,
                     ctypes.POINTER(mp_solve_info), _P], ctypes.c_int)

for _name in ("mpkrylov_cg_td", "mpkrylov_cg_qd", "mpkrylov_bicgstab_td", "mpkrylov_bicgstab_qd", "mpkrylov_cgs_td",
              "mpkrylov_cgs_qd", "mpkrylov_gpbicg_td", "mpkrylov_gpbicg_qd"):
    _SIGS[_name] = ([_CSR, _P, _P, _P, ctypes.POINTER(mp_solve_opts), _P, _P, ctypes.c_size_t,
                     ctypes.POINTER(mp_solve_info), _P], ctypes.c_int)
for _name in ("mpkrylov_bicg_td", "mpkrylov_bicg_qd"):
    _SIGS[_name] = ([_CSR, _P, _CSR, _P, _P, _P, ctypes.POINTER(mp_solve_opts), _P, _P, _P, ctypes.c_size_t,
                     ctypes.POINTER(mp_solve_info), _P], ctypes.c_int)
_SIGS["mpkrylov_mp_workspace_bytes"] = ([_CSR, _I, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int)
_SIGS["mpkrylov_bicg"] = ([_CSR, _P, _CSR, _P, _P, _P, ctypes.POINTER(mp_solve_opts), _P, _P, _P, ctypes.c_size_t,
                           ctypes.POINTER(mp_solve_info), _P], ctypes.c_int)
_SIGS["mp_csr_transpose"] = ([_CSR, _I, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int)
_SIGS["mp_coo_to_csr"] = ([_I, _I, ctypes.c_int64, _P, _P, _I, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int)
_SIGS["mpkrylov_ir_learned"] = ([_CSR, _P, _P, _P, _P, ctypes.POINTER(mp_solve_opts), _P, _P, ctypes.c_size_t,
                                 ctypes.POINTER(mp_solve_info), _P], ctypes.c_int)
_SIGS["mp_mpnn_param_count"] = ([ctypes.POINTER(_I)], ctypes.c_int)
_SIGS["mp_mpnn_create"] = ([_I, ctypes.POINTER(_P)], ctypes.c_int)
_SIGS["mp_mpnn_destroy"] = ([_P], ctypes.c_int)
for _name in ("mp_mpnn_set_params", "mp_mpnn_get_params", "mp_mpnn_get_grads", "mp_mpnn_zero_grads"):
    _SIGS[_name] = ([_P, _P], ctypes.c_int)
_SIGS["mp_graph_create"] = ([_CSR, _P, _P, ctypes.POINTER(_P)], ctypes.c_int)
_SIGS["mp_graph_destroy"] = ([_P], ctypes.c_int)
_SIGS["mp_mpnn_forward"] = ([_P, _P, _P, _P], ctypes.c_int)
_SIGS["mp_mpnn_loss_grad"] = ([_P, _P, _P, _P, _I, _P, _P], ctypes.c_int)
_SIGS["mp_mpnn_adam_step"] = ([_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               _I, _P], ctypes.c_int)
_SIGS["mp_batch_plan_create"] = ([_CSR, _P, _I, _I, _I, _P, ctypes.POINTER(_P)], ctypes.c_int)
_SIGS["mp_batch_plan_autotune"] = ([_P, _CSR, _P, _P, _P, _I, _P, ctypes.POINTER(_I)], ctypes.c_int)
_SIGS["mp_batch_plan_destroy"] = ([_P], ctypes.c_int)
_SIGS["mp_batch_plan_set_schedule"] = ([_P, _I, _I, _I], ctypes.c_int)
_SIGS["mp_batch_plan_schedule"] = ([_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)], ctypes.c_int)
_SIGS["mpspmm_csr_dd_batched"] = ([_CSR, _P, _P, _P, _I, _P, _P], ctypes.c_int)
_SIGS["mpkrylov_batched_workspace_bytes"] = ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int)
_SIGS["mpkrylov_cg_batched"] = ([_CSR, _P, _P, _P, _I, ctypes.POINTER(mp_solve_opts), _P, _I, _P, ctypes.c_size_t,
                                 _P, _P], ctypes.c_int)

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _check(status, func):
    if status != MP_OK:
        raise MpError(status, func, _lib.mp_last_error().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_mp(t, K, L, name):
    import torch
    if t is None:
        raise ValueError("%s is required" % name)
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (K, L):
        raise ValueError("%s must be a contiguous CUDA float64 tensor of shape (%d, %d); got %s %s %s"
                         % (name, K, L, tuple(t.shape), t.dtype, t.device))


def version():
    return _lib.mp_version().decode()


def library_path():
    return LIB_PATH


class Csr:
    """A CSR pattern in device memory (int32 row_ptr / col_idx tensors, 0-based)."""

    def __init__(self, row_ptr, col_idx, n_cols=None):
        import torch
        for t, nm in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
            if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.dim() != 1:
                raise ValueError("%s must be a contiguous 1-D CUDA int32 tensor" % nm)
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.n_rows = row_ptr.numel() - 1
        self.n_cols = self.n_rows if n_cols is None else int(n_cols)
        self.nnz = col_idx.numel()
        self.c = mp_csr(self.n_rows, self.n_cols, self.nnz, row_ptr.data_ptr(),
                        col_idx.data_ptr() if self.nnz else None)

    @classmethod
    def from_numpy(cls, row_ptr, col_idx, n_cols=None, device="cuda"):
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(col_idx, dtype=np.int32)).to(device)
        return cls(rp, ci, n_cols)


class Plan:
    """Owns an mp_plan* (destroyed with the object)."""

    def __init__(self, handle, n_rows):
        self._h = handle
        self.n_rows = n_rows

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if self._h:
            _lib.mp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def row_log2w(self):
        out = np.zeros(self.n_rows, dtype=np.uint8)
        _check(_lib.mp_plan_row_log2w(self._h, out.ctypes.data_as(ctypes.c_void_p)), "mp_plan_row_log2w")
        return out

    def info(self):
        v = [ctypes.c_int32() for _ in range(5)]
        _check(_lib.mp_plan_info(self._h, *[ctypes.byref(x) for x in v]), "mp_plan_info")
        return dict(zip(("n_rows", "n_tiles", "tile_nnz", "ncomp", "is_complex"), (x.value for x in v)))


def _plan_handle(plan):
    return None if plan is None else plan.handle


def mpspmv_workspace_bytes(plan):
    """Bytes of SpMV workspace the plan needs (C ABI mpspmv_workspace_bytes; 0 for None)."""
    v = ctypes.c_size_t()
    _check(_lib.mpspmv_workspace_bytes(_plan_handle(plan), ctypes.byref(v)), "mpspmv_workspace_bytes")
    return v.value


def spmv_workspace(plan, stream=None):
    """A device tensor large enough for the plan's SpMV workspace (None if it needs none),
    allocated on `stream` (torch's current stream by default)."""
    import torch
    nb = mpspmv_workspace_bytes(plan)
    if nb == 0:
        return None
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
        return torch.empty((nb + 7) // 8, dtype=torch.float64, device="cuda")


def _spmv_ws(plan, ws, stream):
    """(workspace tensor or None, pointer, bytes) for one SpMV call: the caller's tensor,
    or a fresh one on the call's stream (kept alive by the caching allocator's stream
    order until the call completes)."""
    if plan is None:
        return None, None, 0
    if ws is None:
        ws = spmv_workspace(plan, stream)
        if ws is None:
            return None, None, 0
    return ws, _ptr(ws), ws.numel() * ws.element_size()


def mp_csr_validate(A, stream=None):
    _check(_lib.mp_csr_validate(ctypes.byref(A.c), _stream_ptr(stream)), "mp_csr_validate")


def mp_measure_rate(kind, stream=None):
    """Measured throughput (C ABI mp_measure_rate): kind 0 = binary64 FMA lane-instructions
    per second, kind K = 2, 3, 4 = K-component multiply-then-add steps per second."""
    v = ctypes.c_double()
    _check(_lib.mp_measure_rate(int(kind), ctypes.byref(v), _stream_ptr(stream)), "mp_measure_rate")
    return v.value


def mp_plan_create(A, ncomp, is_complex=False, shift=0, max_log2w=6, tile_nnz=0, row_groups=0, stream=None):
    """Plan for pattern A and variant (ncomp, is_complex); canonical order by default."""
    h = ctypes.c_void_p()
    opts = mp_plan_opts(shift, max_log2w, tile_nnz, int(row_groups))
    _check(_lib.mp_plan_create(ctypes.byref(A.c), ncomp, int(bool(is_complex)), ctypes.byref(opts),
                               _stream_ptr(stream), ctypes.byref(h)), "mp_plan_create")
    return Plan(h.value, A.n_rows)


def mp_plan_create_explicit(A, ncomp, is_complex, log2w, tile_nnz=0, stream=None):
    lw = np.ascontiguousarray(log2w, dtype=np.uint8)
    if lw.size != A.n_rows:
        raise ValueError("log2w must have n_rows entries")
    h = ctypes.c_void_p()
    _check(_lib.mp_plan_create_explicit(ctypes.byref(A.c), ncomp, int(bool(is_complex)),
                                        lw.ctypes.data_as(ctypes.c_void_p), tile_nnz, _stream_ptr(stream),
                                        ctypes.byref(h)), "mp_plan_create_explicit")
    return Plan(h.value, A.n_rows)


def mp_plan_autotune(A, ncomp, a_re, x_re, y_re, a_im=None, x_im=None, y_im=None, reps=3, stream=None):
    """Autotuned plan; returns (Plan, {"shift", "max_log2w", "tile_nnz", "row_groups"})."""
    cplx = a_im is not None
    h = ctypes.c_void_p()
    opts = mp_plan_opts()
    _check(_lib.mp_plan_autotune(ctypes.byref(A.c), ncomp, int(cplx), _ptr(a_re), _ptr(a_im), _ptr(x_re),
                                 _ptr(x_im), _ptr(y_re), _ptr(y_im), reps, _stream_ptr(stream), ctypes.byref(h),
                                 ctypes.byref(opts)), "mp_plan_autotune")
    return Plan(h.value, A.n_rows), {"shift": opts.shift, "max_log2w": opts.max_log2w, "tile_nnz": opts.tile_nnz,
                                     "row_groups": opts.row_groups}


def _spmv_real(name, K):
    fn = getattr(_lib, name)

    def call(A, a, x, y, plan=None, stream=None, ws=None):
        _check_mp(a, K, A.nnz, "a")
        _check_mp(x, K, A.n_cols, "x")
        _check_mp(y, K, A.n_rows, "y")
        _w, wp, wb = _spmv_ws(plan, ws, stream)
        _check(fn(ctypes.byref(A.c), _ptr(a), _ptr(x), _ptr(y), _plan_handle(plan), wp, wb, _stream_ptr(stream)),
               name)
        return y

    call.__name__ = name
    call.__doc__ = "y = A x in %d-component arithmetic (C ABI %s); tensors of shape (K, len)." % (K, name)
    return call


def mp_csr_transpose(A, a_re, a_im=None, stream=None):
    """A^T (C ABI mp_csr_transpose): returns (Csr of A^T, at_re, at_im or None), values
    shaped like a_re ((ncomp, nnz), or (nnz,) for a binary64 matrix)."""
    import torch
    for t, nm in ((a_re, "a_re"), (a_im, "a_im")):
        if t is None:
            continue
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() % max(A.nnz, 1):
            raise ValueError("%s must be a contiguous CUDA float64 tensor of ncomp * nnz values" % nm)
    ncomp = a_re.numel() // A.nnz if A.nnz else (a_re.shape[0] if a_re.dim() == 2 else 1)
    rpt = torch.empty(A.n_cols + 1, dtype=torch.int32, device="cuda")
    cit = torch.empty(A.nnz, dtype=torch.int32, device="cuda")
    at_re = torch.empty_like(a_re)
    at_im = torch.empty_like(a_im) if a_im is not None else None
    _check(_lib.mp_csr_transpose(ctypes.byref(A.c), int(ncomp), _ptr(a_re), _ptr(a_im), _ptr(rpt), _ptr(cit),
                                 _ptr(at_re), _ptr(at_im), _stream_ptr(stream)), "mp_csr_transpose")
    return Csr(rpt, cit, n_cols=A.n_rows), at_re, at_im


def mp_coo_to_csr(n_rows, n_cols, row, col, v_re, v_im=None, stream=None):
    """CSR of a COO matrix (C ABI mp_coo_to_csr).  row, col: CUDA int32 tensors of nnz
    0-based coordinates; v_re (v_im): CUDA float64 values, (ncomp, nnz) or (nnz,).
    Returns (Csr, a_re, a_im or None), values shaped like v_re, ordered by row then
    column (equal coordinates stay in input order)."""
    import torch
    nnz = row.numel()
    for t, nm in ((row, "row"), (col, "col")):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous() or t.numel() != nnz:
            raise ValueError("%s must be a contiguous CUDA int32 tensor of %d coordinates" % (nm, nnz))
    for t, nm in ((v_re, "v_re"), (v_im, "v_im")):
        if t is None:
            continue
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or (nnz and t.numel() % nnz):
            raise ValueError("%s must be a contiguous CUDA float64 tensor of ncomp * nnz values" % nm)
    ncomp = v_re.numel() // nnz if nnz else (v_re.shape[0] if v_re.dim() == 2 else 1)
    rp = torch.empty(n_rows + 1, dtype=torch.int32, device="cuda")
    ci = torch.empty(nnz, dtype=torch.int32, device="cuda")
    a_re = torch.empty_like(v_re)
    a_im = torch.empty_like(v_im) if v_im is not None else None
    _check(_lib.mp_coo_to_csr(int(n_rows), int(n_cols), int(nnz), _ptr(row), _ptr(col), int(ncomp), _ptr(v_re),
                              _ptr(v_im), _ptr(rp), _ptr(ci), _ptr(a_re), _ptr(a_im), _stream_ptr(stream)),
           "mp_coo_to_csr")
    return Csr(rp, ci, n_cols=n_cols), a_re, a_im


def _spmv_dmat(name, K):
    fn = getattr(_lib, name)

    def call(A, a, x, y, plan=None, stream=None, ws=None):
        import torch
        if not a.is_cuda or a.dtype != torch.float64 or not a.is_contiguous() or a.numel() != A.nnz:
            raise ValueError("a must be a contiguous CUDA float64 tensor of %d binary64 values" % A.nnz)
        _check_mp(x, K, A.n_cols, "x")
        _check_mp(y, K, A.n_rows, "y")
        _w, wp, wb = _spmv_ws(plan, ws, stream)
        _check(fn(ctypes.byref(A.c), _ptr(a), _ptr(x), _ptr(y), _plan_handle(plan), wp, wb, _stream_ptr(stream)),
               name)
        return y

    call.__name__ = name
    call.__doc__ = ("y = A x with a binary64 matrix and a %d-component vector (C ABI %s)." % (K, name))
    return call


def _spmv_complex(name, K):
    fn = getattr(_lib, name)

    def call(A, a_re, a_im, x_re, x_im, y_re, y_im, plan=None, stream=None, ws=None):
        for t, nm, L in ((a_re, "a_re", A.nnz), (a_im, "a_im", A.nnz), (x_re, "x_re", A.n_cols),
                         (x_im, "x_im", A.n_cols), (y_re, "y_re", A.n_rows), (y_im, "y_im", A.n_rows)):
            _check_mp(t, K, L, nm)
        _w, wp, wb = _spmv_ws(plan, ws, stream)
        _check(fn(ctypes.byref(A.c), _ptr(a_re), _ptr(a_im), _ptr(x_re), _ptr(x_im), _ptr(y_re), _ptr(y_im),
                  _plan_handle(plan), wp, wb, _stream_ptr(stream)), name)
        return y_re, y_im

    call.__name__ = name
    call.__doc__ = "complex y = A x in %d-component arithmetic (C ABI %s)." % (K, name)
    return call


mpspmv_csr_dd = _spmv_real("mpspmv_csr_dd", 2)
mpspmv_csr_td = _spmv_real("mpspmv_csr_td", 3)
mpspmv_csr_qd = _spmv_real("mpspmv_csr_qd", 4)
mpspmv_csr_dd_complex = _spmv_complex("mpspmv_csr_dd_complex", 2)
mpspmv_csr_td_complex = _spmv_complex("mpspmv_csr_td_complex", 3)
mpspmv_csr_qd_complex = _spmv_complex("mpspmv_csr_qd_complex", 4)

def _spmv_dmat_complex(name, K):
    fn = getattr(_lib, name)

    def call(A, a_re, a_im, x_re, x_im, y_re, y_im, plan=None, stream=None, ws=None):
        import torch
        for t, nm in ((a_re, "a_re"), (a_im, "a_im")):
            if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != A.nnz:
                raise ValueError("%s must be a contiguous CUDA float64 tensor of %d binary64 values" % (nm, A.nnz))
        for t, nm, L in ((x_re, "x_re", A.n_cols), (x_im, "x_im", A.n_cols), (y_re, "y_re", A.n_rows),
                         (y_im, "y_im", A.n_rows)):
            _check_mp(t, K, L, nm)
        _w, wp, wb = _spmv_ws(plan, ws, stream)
        _check(fn(ctypes.byref(A.c), _ptr(a_re), _ptr(a_im), _ptr(x_re), _ptr(x_im), _ptr(y_re), _ptr(y_im),
                  _plan_handle(plan), wp, wb, _stream_ptr(stream)), name)
        return y_re, y_im

    call.__name__ = name
    call.__doc__ = ("complex y = A x with a binary64 complex matrix and a %d-component complex vector (C ABI %s)."
                    % (K, name))
    return call


mpspmv_csr_dd_d = _spmv_dmat("mpspmv_csr_dd_d", 2)
mpspmv_csr_td_d = _spmv_dmat("mpspmv_csr_td_d", 3)
mpspmv_csr_qd_d = _spmv_dmat("mpspmv_csr_qd_d", 4)
SPMV_D = {2: mpspmv_csr_dd_d, 3: mpspmv_csr_td_d, 4: mpspmv_csr_qd_d}
mpspmv_csr_dd_d_complex = _spmv_dmat_complex("mpspmv_csr_dd_d_complex", 2)
mpspmv_csr_td_d_complex = _spmv_dmat_complex("mpspmv_csr_td_d_complex", 3)
mpspmv_csr_qd_d_complex = _spmv_dmat_complex("mpspmv_csr_qd_d_complex", 4)
SPMV_D_COMPLEX = {2: mpspmv_csr_dd_d_complex, 3: mpspmv_csr_td_d_complex, 4: mpspmv_csr_qd_d_complex}

def mpspmv_csr_dd_noalloc(A, a, x, y, plan=None, stream=None):
    """DD y = A x without workspace (C ABI mpspmv_csr_dd_noalloc: x is staged in the
    library's fixed device array, n_cols <= 1,048,576; overlapping calls race)."""
    _check_mp(a, 2, A.nnz, "a")
    _check_mp(x, 2, A.n_cols, "x")
    _check_mp(y, 2, A.n_rows, "y")
    _check(_lib.mpspmv_csr_dd_noalloc(ctypes.byref(A.c), _ptr(a), _ptr(x), _ptr(y), _plan_handle(plan),
                                      _stream_ptr(stream)), "mpspmv_csr_dd_noalloc")
    return y


SPMV = {(2, False): mpspmv_csr_dd, (3, False): mpspmv_csr_td, (4, False): mpspmv_csr_qd,
        (2, True): mpspmv_csr_dd_complex, (3, True): mpspmv_csr_td_complex, (4, True): mpspmv_csr_qd_complex}


# ---------------------------------------------------------------------------------------
# Krylov solvers
# ---------------------------------------------------------------------------------------

def mpvec_dd_sub(x, y, z, stream=None):
    """z = x - y in DD (C ABI mpvec_dd_sub); (2, n) CUDA float64 tensors."""
    n = x.shape[1] if x.dim() == 2 else 0
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _check_mp(t, 2, n, nm)
    _check(_lib.mpvec_dd_sub(n, _ptr(x), _ptr(y), _ptr(z), _stream_ptr(stream)), "mpvec_dd_sub")
    return z


def _opts(precond="jacobi", rtol=1e-28, max_iter=10000, check_every=32, inner="fp64", inner_rtol=1e-8,
          inner_max_iter=0, max_outer=50):
    return mp_solve_opts(PRECOND[precond], int(max_iter), float(rtol), int(check_every), INNER[inner],
                         float(inner_rtol), int(inner_max_iter), int(max_outer))


def _info_dict(info):
    return {"status": info.status, "iters": info.iters, "outer_iters": info.outer_iters,
            "restarts": info.restarts, "rr_true": np.array(info.rr_true[:]), "bb": np.array(info.bb[:]),
            "relres": info.relres, "seconds": info.seconds, "fell_back": info.fell_back}


def mpkrylov_workspace_bytes(A, **opts):
    o = _opts(**opts)
    nb = ctypes.c_size_t()
    _check(_lib.mpkrylov_workspace_bytes(ctypes.byref(A.c), ctypes.byref(o), ctypes.byref(nb)),
           "mpkrylov_workspace_bytes")
    return nb.value


def _workspace(A, ws, **opts):
    import torch
    need = mpkrylov_workspace_bytes(A, **opts)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    return ws


def _solver(name):
    fn = getattr(_lib, name)

    def call(A, a, b, x, plan=None, ws=None, stream=None, raise_on_failure=False, **opts):
        _check_mp(a, 2, A.nnz, "a")
        _check_mp(b, 2, A.n_rows, "b")
        _check_mp(x, 2, A.n_rows, "x")
        o = _opts(**opts)
        ws = _workspace(A, ws, **opts)
        info = mp_solve_info()
        st = fn(ctypes.byref(A.c), _ptr(a), _ptr(b), _ptr(x), ctypes.byref(o), _plan_handle(plan), _ptr(ws),
                ws.numel() * ws.element_size(), ctypes.byref(info), _stream_ptr(stream))
        if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
            _check(st, name)
        return _info_dict(info)

    call.__name__ = name
    call.__doc__ = "DD Krylov solve (C ABI %s); x is updated in place; returns the info record." % name
    return call


mpkrylov_cg = _solver("mpkrylov_cg")
mpkrylov_bicgstab = _solver("mpkrylov_bicgstab")
mpkrylov_cgs = _solver("mpkrylov_cgs")
mpkrylov_gpbicg = _solver("mpkrylov_gpbicg")


def _solver_k(name, K):
    fn = getattr(_lib, name)

    def call(A, a, b, x, plan=None, ws=None, stream=None, raise_on_failure=False, **opts):
        _check_mp(a, K, A.nnz, "a")
        _check_mp(b, K, A.n_rows, "b")
        _check_mp(x, K, A.n_rows, "x")
        o = _opts(**opts)
        ws = _mp_workspace(A, K, ws)
        info = mp_solve_info()
        st = fn(ctypes.byref(A.c), _ptr(a), _ptr(b), _ptr(x), ctypes.byref(o), _plan_handle(plan), _ptr(ws),
                ws.numel() * ws.element_size(), ctypes.byref(info), _stream_ptr(stream))
        if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
            _check(st, name)
        return _info_dict(info)

    call.__name__ = name
    call.__doc__ = "%d-component Krylov solve (C ABI %s); x is updated in place; returns the info record." % (K, name)
    return call


def _mp_workspace(A, K, ws):
    import torch
    nb = ctypes.c_size_t()
    _check(_lib.mpkrylov_mp_workspace_bytes(ctypes.byref(A.c), K, ctypes.byref(nb)), "mpkrylov_mp_workspace_bytes")
    return torch.empty(nb.value, dtype=torch.uint8, device="cuda") if ws is None else ws


def _bicg_k(name, K):
    fn = getattr(_lib, name)

    def call(A, a, At, at, b, x, plan=None, plan_t=None, ws=None, stream=None, raise_on_failure=False, **opts):
        _check_mp(a, K, A.nnz, "a")
        _check_mp(at, K, At.nnz, "at")
        _check_mp(b, K, A.n_rows, "b")
        _check_mp(x, K, A.n_rows, "x")
        o = _opts(**opts)
        ws = _mp_workspace(A, K, ws)
        info = mp_solve_info()
        st = fn(ctypes.byref(A.c), _ptr(a), ctypes.byref(At.c), _ptr(at), _ptr(b), _ptr(x), ctypes.byref(o),
                _plan_handle(plan), _plan_handle(plan_t), _ptr(ws), ws.numel() * ws.element_size(), ctypes.byref(info),
                _stream_ptr(stream))
        if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
            _check(st, name)
        return _info_dict(info)

    call.__name__ = name
    call.__doc__ = "%d-component BiCG (C ABI %s) with A^T given as (At, at); returns the info record." % (K, name)
    return call


mpkrylov_cg_td = _solver_k("mpkrylov_cg_td", 3)
mpkrylov_cg_qd = _solver_k("mpkrylov_cg_qd", 4)
mpkrylov_bicgstab_td = _solver_k("mpkrylov_bicgstab_td", 3)
mpkrylov_bicgstab_qd = _solver_k("mpkrylov_bicgstab_qd", 4)
mpkrylov_cgs_td = _solver_k("mpkrylov_cgs_td", 3)
mpkrylov_cgs_qd = _solver_k("mpkrylov_cgs_qd", 4)
mpkrylov_gpbicg_td = _solver_k("mpkrylov_gpbicg_td", 3)
mpkrylov_gpbicg_qd = _solver_k("mpkrylov_gpbicg_qd", 4)
mpkrylov_bicg_td = _bicg_k("mpkrylov_bicg_td", 3)
mpkrylov_bicg_qd = _bicg_k("mpkrylov_bicg_qd", 4)
mpkrylov_ir = _solver("mpkrylov_ir")


def mpkrylov_bicg(A, a, At, at, b, x, plan=None, plan_t=None, ws=None, stream=None, raise_on_failure=False, **opts):
    """DD BiCG (C ABI mpkrylov_bicg) with A^T given as (At, at), e.g. from
    mp_csr_transpose.  x is updated in place; returns the info record."""
    _check_mp(a, 2, A.nnz, "a")
    _check_mp(at, 2, At.nnz, "at")
    _check_mp(b, 2, A.n_rows, "b")
    _check_mp(x, 2, A.n_rows, "x")
    o = _opts(**opts)
    ws = _workspace(A, ws, **opts)
    info = mp_solve_info()
    st = _lib.mpkrylov_bicg(ctypes.byref(A.c), _ptr(a), ctypes.byref(At.c), _ptr(at), _ptr(b), _ptr(x),
                            ctypes.byref(o), _plan_handle(plan), _plan_handle(plan_t), _ptr(ws),
                            ws.numel() * ws.element_size(), ctypes.byref(info), _stream_ptr(stream))
    if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
        _check(st, "mpkrylov_bicg")
    return _info_dict(info)


def mpkrylov_ir_learned(A, a, m_values, b, x, plan=None, ws=None, stream=None, raise_on_failure=False, **opts):
    """Refinement with a learned inner preconditioner (C ABI mpkrylov_ir_learned).

    m_values: CUDA float64 tensor of A.nnz values of M on A's pattern.  x is updated in
    place; returns the info record."""
    import torch
    _check_mp(a, 2, A.nnz, "a")
    _check_mp(b, 2, A.n_rows, "b")
    _check_mp(x, 2, A.n_rows, "x")
    if (not m_values.is_cuda or m_values.dtype != torch.float64 or not m_values.is_contiguous()
            or m_values.numel() != A.nnz):
        raise ValueError("m_values must be a contiguous CUDA float64 tensor of %d values" % A.nnz)
    opts["precond"] = "learned"
    o = _opts(**opts)
    ws = _workspace(A, ws, **opts)
    info = mp_solve_info()
    st = _lib.mpkrylov_ir_learned(ctypes.byref(A.c), _ptr(a), _ptr(m_values), _ptr(b), _ptr(x), ctypes.byref(o),
                                  _plan_handle(plan), _ptr(ws), ws.numel() * ws.element_size(), ctypes.byref(info),
                                  _stream_ptr(stream))
    if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
        _check(st, "mpkrylov_ir_learned")
    return _info_dict(info)


# ---------------------------------------------------------------------------------------
# learned preconditioner network
# ---------------------------------------------------------------------------------------

def mp_mpnn_param_count():
    c = _I()
    _check(_lib.mp_mpnn_param_count(ctypes.byref(c)), "mp_mpnn_param_count")
    return c.value


class Mpnn:
    """Owns an mp_mpnn* (parameters, gradient accumulator, Adam moments on the device)."""

    def __init__(self, hidden=64):
        h = _P()
        _check(_lib.mp_mpnn_create(int(hidden), ctypes.byref(h)), "mp_mpnn_create")
        self._h = h
        self.n_params = mp_mpnn_param_count()

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if self._h:
            _lib.mp_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.shape != (self.n_params,):
            raise ValueError("expected %d parameters" % self.n_params)
        _check(_lib.mp_mpnn_set_params(self._h, t.ctypes.data_as(_P)), "mp_mpnn_set_params")

    def get_params(self):
        t = np.empty(self.n_params, dtype=np.float32)
        _check(_lib.mp_mpnn_get_params(self._h, t.ctypes.data_as(_P)), "mp_mpnn_get_params")
        return t

    def get_grads(self):
        t = np.empty(self.n_params, dtype=np.float32)
        _check(_lib.mp_mpnn_get_grads(self._h, t.ctypes.data_as(_P)), "mp_mpnn_get_grads")
        return t

    def zero_grads(self, stream=None):
        _check(_lib.mp_mpnn_zero_grads(self._h, _stream_ptr(stream)), "mp_mpnn_zero_grads")

    def adam_step(self, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0, stream=None):
        _check(_lib.mp_mpnn_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), float(grad_scale),
                                      int(step), _stream_ptr(stream)), "mp_mpnn_adam_step")


class Graph:
    """Owns an mp_graph* built from (A, a); keeps A and a alive while it exists."""

    def __init__(self, A, a, stream=None):
        _check_mp(a, 2, A.nnz, "a")
        h = _P()
        _check(_lib.mp_graph_create(ctypes.byref(A.c), _ptr(a), _stream_ptr(stream), ctypes.byref(h)),
               "mp_graph_create")
        self._h = h
        self.A, self.a = A, a

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if self._h:
            _lib.mp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def mp_mpnn_forward(net, g, m_values=None, stream=None):
    """M values of the network on g's pattern (CUDA float64 tensor of nnz values)."""
    import torch
    if m_values is None:
        m_values = torch.empty(g.A.nnz, dtype=torch.float64, device="cuda")
    _check(_lib.mp_mpnn_forward(net.handle, g.handle, _ptr(m_values), _stream_ptr(stream)), "mp_mpnn_forward")
    return m_values


def mp_mpnn_loss_grad(net, g, r, e, stream=None):
    """Add the gradients of the losses of the pairs (r[p], e[p]) to the accumulator.

    r, e: CUDA float64 tensors of shape (npairs, n).  Returns the losses (numpy)."""
    import torch
    n = g.A.n_rows
    for t, nm in ((r, "r"), (e, "e")):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != n:
            raise ValueError("%s must be a contiguous CUDA float64 tensor of shape (npairs, %d)" % (nm, n))
    npairs = r.shape[0]
    if e.shape[0] != npairs:
        raise ValueError("r and e hold different numbers of pairs")
    out = np.empty(npairs, dtype=np.float64)
    _check(_lib.mp_mpnn_loss_grad(net.handle, g.handle, _ptr(r), _ptr(e), int(npairs), out.ctypes.data_as(_P),
                                  _stream_ptr(stream)), "mp_mpnn_loss_grad")
    return out


# ---------------------------------------------------------------------------------------
# batched block-diagonal systems
# ---------------------------------------------------------------------------------------

class BatchPlan:
    """Owns an mp_batch_plan* (destroyed with the object)."""

    def __init__(self, handle, nsys, nrhs):
        self._h = handle
        self.nsys = nsys
        self.nrhs = nrhs

    @property
    def handle(self):
        return self._h

    def destroy(self):
        if self._h:
            _lib.mp_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _check_multi(t, N, R, name):
    import torch
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (2, N, R):
        raise ValueError("%s must be a contiguous CUDA float64 tensor of shape (2, %d, %d)" % (name, N, R))


def mp_batch_plan_create(A, sys_ptr, nrhs, threads_per_row=1, stream=None):
    sp = np.ascontiguousarray(sys_ptr, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(_lib.mp_batch_plan_create(ctypes.byref(A.c), sp.ctypes.data_as(ctypes.c_void_p), sp.size - 1, nrhs,
                                     threads_per_row, _stream_ptr(stream), ctypes.byref(h)), "mp_batch_plan_create")
    return BatchPlan(h.value, sp.size - 1, nrhs)


def mp_batch_plan_autotune(plan, A, a, X, Y, reps=3, stream=None):
    tpr = ctypes.c_int32()
    _check(_lib.mp_batch_plan_autotune(plan.handle, ctypes.byref(A.c), _ptr(a), _ptr(X), _ptr(Y), reps,
                                       _stream_ptr(stream), ctypes.byref(tpr)), "mp_batch_plan_autotune")
    return tpr.value


def mp_batch_plan_schedule(plan):
    """{"threads_per_row", "rows_per_tile", "chunk_order"} of a batch plan (C ABI mp_batch_plan_schedule)."""
    v = [ctypes.c_int32() for _ in range(3)]
    _check(_lib.mp_batch_plan_schedule(plan.handle, *[ctypes.byref(x) for x in v]), "mp_batch_plan_schedule")
    return dict(zip(("threads_per_row", "rows_per_tile", "chunk_order"), (x.value for x in v)))


def mp_batch_plan_set_schedule(plan, threads_per_row, rows_mult, chunk_order):
    """Explicit batch schedule (C ABI mp_batch_plan_set_schedule)."""
    _check(_lib.mp_batch_plan_set_schedule(plan.handle, int(threads_per_row), int(rows_mult), int(chunk_order)),
           "mp_batch_plan_set_schedule")


def mpspmm_csr_dd_batched(A, a, X, Y, nrhs, plan=None, stream=None):
    _check_mp(a, 2, A.nnz, "a")
    _check_multi(X, A.n_cols, nrhs, "X")
    _check_multi(Y, A.n_rows, nrhs, "Y")
    _check(_lib.mpspmm_csr_dd_batched(ctypes.byref(A.c), _ptr(a), _ptr(X), _ptr(Y), nrhs,
                                      None if plan is None else plan.handle, _stream_ptr(stream)),
           "mpspmm_csr_dd_batched")
    return Y


def mpkrylov_batched_workspace_bytes(plan):
    nb = ctypes.c_size_t()
    _check(_lib.mpkrylov_batched_workspace_bytes(plan.handle, ctypes.byref(nb)), "mpkrylov_batched_workspace_bytes")
    return nb.value


def mpkrylov_cg_batched(A, a, B, X, nrhs, plan, use_graph=True, ws=None, stream=None, raise_on_failure=False, **opts):
    """Batched DD Jacobi-CG; X updated in place; returns a list of nsys*nrhs info dicts."""
    import torch
    _check_mp(a, 2, A.nnz, "a")
    _check_multi(B, A.n_rows, nrhs, "B")
    _check_multi(X, A.n_rows, nrhs, "X")
    o = _opts(**opts)
    if ws is None:
        ws = torch.empty(mpkrylov_batched_workspace_bytes(plan), dtype=torch.uint8, device="cuda")
    npairs = plan.nsys * nrhs
    infos = (mp_solve_info * npairs)()
    st = _lib.mpkrylov_cg_batched(ctypes.byref(A.c), _ptr(a), _ptr(B), _ptr(X), nrhs, ctypes.byref(o), plan.handle,
                                  int(bool(use_graph)), _ptr(ws), ws.numel(), infos, _stream_ptr(stream))
    if st not in (MP_OK, -5, -6) or (raise_on_failure and st != MP_OK):
        _check(st, "mpkrylov_cg_batched")
    return [_info_dict(i) for i in infos]
