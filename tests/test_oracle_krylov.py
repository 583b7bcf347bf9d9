"""Pins of the oracle's DD Krylov layer (CPU only).

* The DD dot product (fixed tree) is within n 2^-100 sum|x||y| of the exact value
  (Fractions), and exact on small integers; DD division is within 2^-100 of the exact
  quotient and exact where the quotient is representable.
* CG on a diagonal matrix with k distinct eigenvalues, unpreconditioned, converges in
  at most k iterations (a property of exact-arithmetic CG that DD keeps).
* CG / BiCGSTAB solve b = A v with the paper's v = sqrt(2)[1..n] (Sec. 4.2) on an SPD
  diffusion matrix and on a non-symmetric narrow-band matrix to relative residual
  1e-28; the returned x's residual is certified with exact rational arithmetic.
* Breakdown (NaN right-hand side) and iteration limit are reported; a warm start
  at the solution stops at once.
* GPBiCG: terminates within k steps on diagonal matrices with k distinct eigenvalues;
  certified 1e-28 on the non-symmetric band; its first step equals BiCGSTAB's to DD
  rounding (eta = 0); each step's recurrence residual equals the exact residual of
  that step's iterate to DD rounding.  Each of eleven plausible mistakes in its
  recursions (a dropped eta term in u, z or r, a sign in y, eta, w or p, beta without
  alpha/zeta, swapped dots in zeta, x without the preconditioner) fails three or more
  of these pins.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref, exact
from workloads import random_mp, diffusion3d_7pt, banded_nonsymmetric, sqrt2_vector, random_csr


def _fr(v):
    return Fraction(float(v[0])) + Fraction(float(v[1]))


@pytest.mark.parametrize("n", [0, 1, 255, 256, 4096, 4097, 9000])
def test_dd_dot_bound(n):
    rng = np.random.default_rng(n)
    x = random_mp(n, 2, rng)
    y = random_mp(n, 2, rng)
    d = ref.dd_dot(x, y)
    ex = sum((_fr(x[:, i]) * _fr(y[:, i]) for i in range(n)), Fraction(0))
    s = sum((abs(_fr(x[:, i]) * _fr(y[:, i])) for i in range(n)), Fraction(0))
    assert abs(_fr(d) - ex) <= max(n, 1) * s / 2 ** 100
    if n == 0:
        assert d[0] == 0 and d[1] == 0


def test_dd_dot_integers_exact():
    rng = np.random.default_rng(1)
    n = 10000
    x = np.zeros((2, n))
    y = np.zeros((2, n))
    x[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    y[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    d = ref.dd_dot(x, y)
    assert _fr(d) == int(np.dot(x[0].astype(object), y[0].astype(object)))


def test_dd_div():
    rng = np.random.default_rng(2)
    for _ in range(2000):
        a = random_mp(1, 2, rng)[:, 0] * 2.0 ** rng.integers(-30, 30)
        b = random_mp(1, 2, rng)[:, 0] * 2.0 ** rng.integers(-30, 30)
        q = ref.dd_div(a, b)
        ex = _fr(a) / _fr(b)
        assert abs(_fr(q) - ex) <= abs(ex) / 2 ** 100
    assert list(ref.dd_div(np.array([6.0, 0.0]), np.array([3.0, 0.0]))) == [2.0, 0.0]
    assert list(ref.dd_div(np.array([1.0, 0.0]), np.array([4.0, 0.0]))) == [0.25, 0.0]


def test_cg_k_distinct_eigenvalues():
    n = 400
    eig = np.array([1.0, 2.0, 3.0, 5.0, 8.0])
    diag = eig[np.arange(n) % eig.size]
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = np.arange(n, dtype=np.int32)
    a = np.zeros((2, n))
    a[0] = diag
    rng = np.random.default_rng(3)
    b = random_mp(n, 2, rng)
    x, info = ref.cg(row_ptr, col_idx, a, b, precond="none", rtol=1e-28, max_iter=50)
    assert info["status"] == 0
    assert info["iters"] <= eig.size


def _certify(row_ptr, col_idx, a, b, x, rtol):
    """Exact ||b - A x||^2 <= rtol^2 ||b||^2 (rationals)."""
    n = row_ptr.size - 1
    ys, _ = exact.exact_row_products(row_ptr, col_idx, a, x)
    scale = Fraction(1, 2 ** (-exact.E_SCALE))
    rr = Fraction(0)
    bb = Fraction(0)
    for i in range(n):
        bi = _fr(b[:, i])
        ri = bi - ys[i] * scale
        rr += ri * ri
        bb += bi * bi
    return rr <= Fraction(rtol) ** 2 * bb * Fraction(101, 100), float(rr / bb) ** 0.5


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_known_solution_certified(precond):
    row_ptr, col_idx, a = diffusion3d_7pt(m=8, sigma=1.0, seed=4)
    n = row_ptr.size - 1
    v = sqrt2_vector(n, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    x, info = ref.cg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=5000)
    assert info["status"] == 0
    ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
    assert ok, rel
    # forward error against the known v: within cond(A) times the residual level
    err = np.max(np.abs((x[0] - v[0]) + (x[1] - v[1]))) / np.max(np.abs(v[0]))
    assert err < 1e-24


def test_bicgstab_nonsymmetric_certified():
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=5)
    v = sqrt2_vector(200, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    for precond in ("none", "jacobi"):
        x, info = ref.bicgstab(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000)
        assert info["status"] == 0
        ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
        assert ok, rel


def test_failure_modes():
    row_ptr, col_idx, a = diffusion3d_7pt(m=6, sigma=1.0, seed=6)
    n = row_ptr.size - 1
    rng = np.random.default_rng(7)
    b = random_mp(n, 2, rng)
    bad = b.copy()
    bad[0, 5] = np.nan
    for solve in (ref.cg, ref.bicgstab):
        _, info = solve(row_ptr, col_idx, a, bad, rtol=1e-28, max_iter=50)
        assert info["status"] == -6
        _, info = solve(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=3)
        assert info["status"] == -5 and info["iters"] == 3
    # warm start at the solution: converged without iterating
    x, info = ref.cg(row_ptr, col_idx, a, b, rtol=1e-20, max_iter=5000)
    assert info["status"] == 0
    x2, info2 = ref.cg(row_ptr, col_idx, a, b, x0=x, rtol=1e-20, max_iter=5000)
    assert info2["status"] == 0 and info2["iters"] == 0 and np.array_equal(x, x2)


def test_bicg_equals_cg_on_symmetric_matrices():
    """With A = A^T exactly (values too) and a symmetric preconditioner the shadow
    recursion of BiCG repeats the primal one, so BiCG is CG step for step: same
    iterates bit for bit, same counts."""
    row_ptr, col_idx, a = diffusion3d_7pt(m=7, sigma=1.5, seed=8)
    n = row_ptr.size - 1
    b = random_mp(n, 2, np.random.default_rng(8))
    for precond in ("none", "jacobi"):
        xc, ic = ref.cg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=5000, history=True)
        xb, ib = ref.bicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=5000, history=True)
        assert ic["status"] == 0 and (ib["status"], ib["iters"], ib["restarts"]) == (0, ic["iters"], ic["restarts"])
        assert np.array_equal(xb, xc)
        assert np.array_equal(ib["history"], ic["history"])


def test_bicg_nonsymmetric_certified():
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=5)
    v = sqrt2_vector(200, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    for precond in ("none", "jacobi"):
        x, info = ref.bicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000)
        assert info["status"] == 0
        ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
        assert ok, rel
    bad = b.copy()
    bad[0, 5] = np.nan
    assert ref.bicg(row_ptr, col_idx, a, bad, rtol=1e-28, max_iter=50)[1]["status"] == -6
    _, info = ref.bicg(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=3)
    assert info["status"] == -5 and info["iters"] == 3


def test_cgs_k_distinct_eigenvalues_and_nonsymmetric_certified():
    """CGS squares the BiCG polynomial, so on a diagonal matrix with k distinct
    eigenvalues it also terminates within k steps; on the tub1000-shaped band it
    reaches 1e-28, certified by an exact residual; failures are reported."""
    n = 400
    eig = np.array([1.0, 2.0, 3.0, 5.0, 8.0])
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col_idx = np.arange(n, dtype=np.int32)
    a = np.zeros((2, n))
    a[0] = eig[np.arange(n) % eig.size]
    b = random_mp(n, 2, np.random.default_rng(3))
    _, info = ref.cgs(row_ptr, col_idx, a, b, precond="none", rtol=1e-28, max_iter=50)
    assert info["status"] == 0 and info["iters"] <= eig.size
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=5)
    v = sqrt2_vector(200, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    for precond in ("none", "jacobi"):
        x, info = ref.cgs(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000)
        assert info["status"] == 0
        ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
        assert ok, rel
    bad = b.copy()
    bad[0, 5] = np.nan
    assert ref.cgs(row_ptr, col_idx, a, bad, rtol=1e-28, max_iter=50)[1]["status"] == -6
    _, info = ref.cgs(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=3)
    assert info["status"] == -5 and info["iters"] == 3


def test_gpbicg_k_distinct_eigenvalues():
    """GPBiCG's residual polynomial carries the BiCG polynomial as a factor, so on a
    diagonal matrix with k distinct eigenvalues it terminates within k steps."""
    n = 400
    for eig in (np.array([1.0, 2.0, 3.0, 5.0, 8.0]), np.array([0.5, 4.0]), np.array([1.0, 1.5, 2.0, 7.0, 9.0, 12.0])):
        row_ptr = np.arange(n + 1, dtype=np.int32)
        col_idx = np.arange(n, dtype=np.int32)
        a = np.zeros((2, n))
        a[0] = eig[np.arange(n) % eig.size]
        b = random_mp(n, 2, np.random.default_rng(eig.size))
        _, info = ref.gpbicg(row_ptr, col_idx, a, b, precond="none", rtol=1e-28, max_iter=50)
        assert info["status"] == 0 and info["iters"] <= eig.size, (eig, info)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_gpbicg_nonsymmetric_certified(precond):
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=5)
    v = sqrt2_vector(200, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    x, info = ref.gpbicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000)
    assert info["status"] == 0
    ok, rel = _certify(row_ptr, col_idx, a, b, x, 1e-28)
    assert ok, rel


def test_gpbicg_first_step_is_bicgstab():
    """With eta = 0 (the first step) GPBiCG's step is BiCGSTAB's: zeta is BiCGSTAB's
    omega and alpha p + z = alpha p + omega s, so the first iterates agree to DD
    rounding."""
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=6)
    b = random_mp(200, 2, np.random.default_rng(6))
    for precond in ("none", "jacobi"):
        xg, ig = ref.gpbicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=1, history=True)
        xb, ib = ref.bicgstab(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=1, history=True)
        assert ig["iters"] == ib["iters"] == 1
        xs = np.abs(xb[0]).max()
        assert np.abs((xg[0] - xb[0]) + (xg[1] - xb[1])).max() <= 1e-28 * xs
        rg, rb = _fr(ig["history"][1]), _fr(ib["history"][1])
        assert abs(rg - rb) <= Fraction(1, 10 ** 26) * rb


def test_gpbicg_recurrence_tracks_true_residual():
    """Every step's recurrence residual equals the true residual of that step's iterate
    (exact rational b - A x) to DD rounding: x (through u and z) and r (through y, w
    and c) are updated consistently.  A dropped or mis-signed term in either
    recursion separates the two by the size of the residual itself."""
    row_ptr, col_idx, a = banded_nonsymmetric(n=120, seed=7)
    n = 120
    b = random_mp(n, 2, np.random.default_rng(7))
    bb = sum(_fr(b[:, i]) ** 2 for i in range(n))
    for precond in ("none", "jacobi"):
        _, full = ref.gpbicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=12, history=True)
        hist = full["history"]
        assert full["iters"] >= 8
        for k in range(1, 9):
            xk, ik = ref.gpbicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=k)
            assert ik["iters"] == k
            ys, _ = exact.exact_row_products(row_ptr, col_idx, a, xk)
            scale = Fraction(1, 2 ** (-exact.E_SCALE))
            rr_true = sum((_fr(b[:, i]) - ys[i] * scale) ** 2 for i in range(n))
            rr_rec = _fr(hist[k])
            gap = abs(float(rr_true) ** 0.5 - float(rr_rec) ** 0.5)
            assert gap <= 1e-24 * float(bb) ** 0.5, (precond, k, gap, float(rr_rec) ** 0.5)
            assert rr_rec < Fraction(1, 4) * bb or k < 3


def test_gpbicg_failures_and_warm_start():
    row_ptr, col_idx, a = banded_nonsymmetric(n=200, seed=5)
    b = random_mp(200, 2, np.random.default_rng(9))
    bad = b.copy()
    bad[0, 5] = np.nan
    assert ref.gpbicg(row_ptr, col_idx, a, bad, rtol=1e-28, max_iter=50)[1]["status"] == -6
    _, info = ref.gpbicg(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=3)
    assert info["status"] == -5 and info["iters"] == 3
    x, info = ref.gpbicg(row_ptr, col_idx, a, b, rtol=1e-24, max_iter=5000)
    assert info["status"] == 0
    x2, info2 = ref.gpbicg(row_ptr, col_idx, a, b, x0=x, rtol=1e-24, max_iter=5000)
    assert info2["iters"] == 0 and np.array_equal(x, x2)
