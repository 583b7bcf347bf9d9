"""Pins of the oracle's mixed-precision iterative refinement (CPU only).

* binary64 and binary32 inner solves refine to the DD target 1e-28, certified by an
  exact rational residual, and agree with the oracle's DD CG solution to the level the
  conditioning allows;
* a refinement that cannot progress (one inner iteration per step) is detected as a
  stall and finished by DD Jacobi-CG (fell_back = 1), still certified;
* max_outer = 0 falls back at once.
"""
import numpy as np
import pytest

from oracle import ref
from tests.test_oracle_krylov import _certify
from workloads import diffusion3d_7pt, random_mp, sqrt2_vector


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_ir_reaches_dd_target(inner):
    row_ptr, col_idx, a = diffusion3d_7pt(m=10, sigma=2.0, seed=21)
    n = row_ptr.size - 1
    v = sqrt2_vector(n, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    x, info = ref.ir(row_ptr, col_idx, a, b, inner=inner, inner_rtol=1e-6, inner_max_iter=2000, rtol=1e-28)
    assert info["status"] == 0 and info["fell_back"] == 0
    assert info["outer_iters"] >= 2
    ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
    assert ok, rel
    xc, _ = ref.cg(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=10000)
    diff = np.max(np.abs((x[0] - xc[0]) + (x[1] - xc[1]))) / np.max(np.abs(xc[0]))
    assert diff < 1e-22


def test_ir_stall_falls_back_to_dd_cg():
    row_ptr, col_idx, a = diffusion3d_7pt(m=8, sigma=2.0, seed=22)
    n = row_ptr.size - 1
    b = random_mp(n, 2, np.random.default_rng(22))
    x, info = ref.ir(row_ptr, col_idx, a, b, inner="fp64", inner_rtol=1e-12, inner_max_iter=1, rtol=1e-28)
    assert info["fell_back"] == 1 and info["status"] == 0
    ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
    assert ok, rel
    x0, info0 = ref.ir(row_ptr, col_idx, a, b, max_outer=0, rtol=1e-28)
    assert info0["fell_back"] == 1 and info0["outer_iters"] == 0 and info0["status"] == 0


def _jacobi_on_pattern(row_ptr, col_idx, a):
    rows = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    return np.where(rows == col_idx, 1.0 / np.where(rows == col_idx, a[0], 1.0), 0.0)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_ir_learned_m_equal_to_jacobi_reproduces_jacobi(inner):
    """M = D^-1 stored on A's pattern (zero off-diagonal values) gives the same iterates."""
    row_ptr, col_idx, a = diffusion3d_7pt(m=7, sigma=2.0, seed=23)
    n = row_ptr.size - 1
    b = random_mp(n, 2, np.random.default_rng(23))
    mv = _jacobi_on_pattern(row_ptr, col_idx, a)
    kw = dict(inner=inner, inner_rtol=1e-5, inner_max_iter=500, rtol=1e-28)
    xj, ij = ref.ir(row_ptr, col_idx, a, b, **kw)
    xm, im = ref.ir(row_ptr, col_idx, a, b, m_values=mv, **kw)
    assert ij["status"] == 0 and (ij["iters"], ij["outer_iters"]) == (im["iters"], im["outer_iters"])
    assert np.array_equal(xj, xm)


def test_ir_learned_exact_inverse_of_diagonal_matrix():
    """For a diagonal A and M = A^-1 every inner PCG converges in one iteration."""
    n = 300
    rng = np.random.default_rng(24)
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = np.arange(n, dtype=np.int32)
    a = np.zeros((2, n))
    a[0] = 2.0 ** rng.integers(0, 6, n)   # exact reciprocals
    b = random_mp(n, 2, rng)
    x, info = ref.ir(row_ptr, col_idx, a, b, inner="fp64", m_values=1.0 / a[0], inner_rtol=1e-12, rtol=1e-28)
    assert info["status"] == 0 and info["fell_back"] == 0
    assert info["iters"] == info["outer_iters"]
    ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
    assert ok, rel


def test_ir_with_network_preconditioner_converges():
    from oracle import mpnn
    row_ptr, col_idx, a = diffusion3d_7pt(m=6, sigma=2.0, seed=25)
    n = row_ptr.size - 1
    b = random_mp(n, 2, np.random.default_rng(25))
    g = mpnn.Graph(row_ptr, col_idx, a[0])
    mv, _ = mpnn.forward(g, mpnn.init_params(2, scale=2.0), bf=True)
    for inner in ("fp64", "fp32"):
        x, info = ref.ir(row_ptr, col_idx, a, b, inner=inner, m_values=mv, inner_rtol=1e-5, rtol=1e-28)
        assert info["status"] == 0 and info["fell_back"] == 0
        ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
        assert ok, rel
