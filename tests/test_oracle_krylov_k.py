"""Pins of the oracle's K-component Krylov layer (TD and QD solvers; CPU only).

* Division: TD / QD quotients within 2^-150 / 2^-200 of the exact rational quotient on
  random full-tail operands over wide exponent ranges; exact quotients come out exact
  with zero tails; K = 2 is Dekker's DD division.
* The stop comparison equals the exact order of K-component values, including values
  that differ only in trailing components; NaN compares false.
* Dot product: K = 2 is the DD dot; TD / QD within n 2^-150 / 2^-200 sum|x||y| of the
  exact value; small integers exact.
* The K-generic CG and BiCGSTAB at K = 2 reproduce the pinned DD solvers bit for bit
  (iterates, counts, residual records) -- one code path for every K.
* TD / QD CG terminate within k steps on a diagonal matrix with k distinct
  eigenvalues; TD / QD CG (SPD diffusion) and BiCGSTAB (non-symmetric band) reach
  relative residuals 1e-44 / 1e-60, beyond DD, certified by an exact rational residual
  of b = A sqrt(2)[1..n] with K-component data; NaN input and iteration limits report.
* TD / QD BiCG equals TD / QD CG bit for bit on a symmetric matrix; CGS and GPBiCG
  terminate within k steps on k distinct eigenvalues; all three certify 1e-44 / 1e-60
  on the non-symmetric band; their K = 2 instances are the DD solvers.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref, exact
from workloads import random_mp, diffusion3d_7pt, banded_nonsymmetric, sqrt2_vector

BITS = {3: 150, 4: 200}
RTOL = {3: 1e-44, 4: 1e-60}


def _fr(v):
    return sum((Fraction(float(c)) for c in v), Fraction(0))


@pytest.mark.parametrize("K", [3, 4])
def test_mp_div_bound_and_exact(K):
    rng = np.random.default_rng(500 + K)
    for _ in range(1500):
        a = random_mp(1, K, rng)[:, 0] * 2.0 ** int(rng.integers(-60, 60))
        b = random_mp(1, K, rng)[:, 0] * 2.0 ** int(rng.integers(-60, 60))
        q = ref.mp_div(K, a, b)
        ex = _fr(a) / _fr(b)
        assert abs(_fr(q) - ex) <= abs(ex) / 2 ** BITS[K]
    for num, den, want in ((6.0, 3.0, 2.0), (1.0, 4.0, 0.25), (-10.0, 2.5, -4.0)):
        q = ref.mp_div(K, np.r_[num, np.zeros(K - 1)], np.r_[den, np.zeros(K - 1)])
        assert q.tolist() == [want] + [0.0] * (K - 1)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_mp_le_is_the_exact_order(K):
    """The stop comparison equals the exact order of the values, also when only the
    trailing components differ; NaN compares false."""
    rng = np.random.default_rng(40 + K)
    for _ in range(3000):
        a = random_mp(1, K, rng)[:, 0]
        b = a.copy()
        c = int(rng.integers(0, K))
        b[c:] = random_mp(1, K, rng)[:K - c, 0] * (2.0 ** (-53 * c) * abs(a[0]) if c else 1.0)
        if rng.random() < 0.1:
            b = a.copy()
        for u, v in ((a, b), (b, a)):
            assert ref.mp_le(K, u, v) == (_fr(u) <= _fr(v))
    nan = np.r_[np.nan, np.zeros(K - 1)]
    assert not ref.mp_le(K, nan, nan) and not ref.mp_le(K, nan, np.ones(K))


def test_mp_div_dd_is_dekker():
    rng = np.random.default_rng(7)
    for _ in range(200):
        a, b = random_mp(1, 2, rng)[:, 0], random_mp(1, 2, rng)[:, 0]
        assert np.array_equal(ref.mp_div(2, a, b), ref.dd_div(a, b))


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("n", [1, 300, 4096, 9001])
def test_mp_dot_bound(K, n):
    rng = np.random.default_rng(K * 100 + n)
    x, y = random_mp(n, K, rng), random_mp(n, K, rng)
    d = ref.mp_dot(K, x, y)
    ex = sum((_fr(x[:, i]) * _fr(y[:, i]) for i in range(n)), Fraction(0))
    s = sum((abs(_fr(x[:, i]) * _fr(y[:, i])) for i in range(n)), Fraction(0))
    assert abs(_fr(d) - ex) <= n * s / 2 ** BITS[K]
    xi = np.zeros((K, n))
    yi = np.zeros((K, n))
    xi[0] = rng.integers(-100, 100, n)
    yi[0] = rng.integers(-100, 100, n)
    assert ref.mp_dot(K, xi, yi).tolist() == [float(np.dot(xi[0], yi[0]))] + [0.0] * (K - 1)
    if n <= 300:
        assert np.array_equal(ref.mp_dot(2, x[:2], y[:2]), ref.dd_dot(x[:2], y[:2]))


def test_generic_solvers_at_K2_are_the_dd_solvers():
    rp, ci, a = diffusion3d_7pt(m=7, sigma=1.5, seed=8)
    n = rp.size - 1
    b = random_mp(n, 2, np.random.default_rng(8))
    for precond in ("none", "jacobi"):
        xd, idd = ref.cg(rp, ci, a, b, precond=precond, rtol=1e-28, history=True)
        xk, ik = ref.cg_k(2, rp, ci, a, b, precond=precond, rtol=1e-28, history=True)
        assert np.array_equal(xd, xk) and np.array_equal(idd["history"], ik["history"])
        assert (idd["status"], idd["iters"], idd["restarts"]) == (ik["status"], ik["iters"], ik["restarts"])
    rp, ci, a = banded_nonsymmetric(n=200, seed=5)
    b = random_mp(200, 2, np.random.default_rng(9))
    for precond in ("none", "jacobi"):
        xd, idd = ref.bicgstab(rp, ci, a, b, precond=precond, rtol=1e-28, max_iter=5000, history=True)
        xk, ik = ref.bicgstab_k(2, rp, ci, a, b, precond=precond, rtol=1e-28, max_iter=5000, history=True)
        assert np.array_equal(xd, xk) and np.array_equal(idd["history"], ik["history"])
        assert (idd["status"], idd["iters"], idd["restarts"]) == (ik["status"], ik["iters"], ik["restarts"])


@pytest.mark.parametrize("K", [3, 4])
def test_cg_k_distinct_eigenvalues(K):
    n = 400
    eig = np.array([1.0, 2.0, 3.0, 5.0, 8.0])
    a = np.zeros((K, n))
    a[0] = eig[np.arange(n) % eig.size]
    b = random_mp(n, K, np.random.default_rng(K))
    _, info = ref.cg_k(K, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), a, b, precond="none",
                       rtol=RTOL[K], max_iter=50)
    assert info["status"] == 0 and info["iters"] <= eig.size


def _certified(rp, ci, a, b, x, rtol):
    n = rp.size - 1
    ys, _ = exact.exact_row_products(rp, ci, a, x)
    scale = Fraction(1, 2 ** (-exact.E_SCALE))
    rr = sum(((_fr(b[:, i]) - ys[i] * scale) ** 2 for i in range(n)), Fraction(0))
    bb = sum((_fr(b[:, i]) ** 2 for i in range(n)), Fraction(0))
    return rr <= Fraction(rtol) ** 2 * bb * Fraction(101, 100), math.sqrt(float(rr / bb)) if bb else 0.0


@pytest.mark.parametrize("K", [3, 4])
def test_k_solvers_reach_beyond_dd_certified(K):
    rp, ci, a = diffusion3d_7pt(m=6, sigma=1.0, seed=4, K=K)
    n = rp.size - 1
    b = ref.spmv(K, rp, ci, a, sqrt2_vector(n, K))
    for precond in ("none", "jacobi"):
        x, info = ref.cg_k(K, rp, ci, a, b, precond=precond, rtol=RTOL[K], max_iter=5000)
        assert info["status"] == 0
        ok, rel = _certified(rp, ci, a, b, x, RTOL[K])
        assert ok, rel
    rp, ci, a = banded_nonsymmetric(n=150, seed=5, K=K)
    b = ref.spmv(K, rp, ci, a, sqrt2_vector(150, K))
    x, info = ref.bicgstab_k(K, rp, ci, a, b, precond="jacobi", rtol=RTOL[K], max_iter=20000)
    assert info["status"] == 0
    ok, rel = _certified(rp, ci, a, b, x, RTOL[K])
    assert ok, rel


@pytest.mark.parametrize("K", [3, 4])
def test_k_solver_failures(K):
    rp, ci, a = diffusion3d_7pt(m=5, sigma=1.0, seed=6, K=K)
    n = rp.size - 1
    b = random_mp(n, K, np.random.default_rng(6))
    bad = b.copy()
    bad[0, 3] = np.nan
    for solve in (ref.cg_k, ref.bicgstab_k):
        assert solve(K, rp, ci, a, bad, rtol=RTOL[K], max_iter=50)[1]["status"] == -6
        _, info = solve(K, rp, ci, a, b, rtol=RTOL[K], max_iter=3)
        assert info["status"] == -5 and info["iters"] == 3


@pytest.mark.parametrize("K", [3, 4])
def test_k_bicg_cgs_gpbicg(K):
    """TD / QD BiCG, CGS and GPBiCG: BiCG equals CG bit for bit on an exactly symmetric
    matrix; CGS and GPBiCG terminate within k steps on k distinct eigenvalues; all three
    reach 1e-44 / 1e-60 on the non-symmetric band, certified by an exact residual; the
    K = 2 instances are the DD solvers."""
    rp, ci, a = diffusion3d_7pt(m=6, sigma=1.5, seed=8, K=K)
    n = rp.size - 1
    b = random_mp(n, K, np.random.default_rng(31))
    for precond in ("none", "jacobi"):
        xc, ic = ref.cg_k(K, rp, ci, a, b, precond=precond, rtol=RTOL[K], max_iter=5000, history=True)
        xb, ib = ref.bicg_k(K, rp, ci, a, b, precond=precond, rtol=RTOL[K], max_iter=5000, history=True)
        assert ic["status"] == 0 and (ib["status"], ib["iters"], ib["restarts"]) == (0, ic["iters"], ic["restarts"])
        assert np.array_equal(xb, xc) and np.array_equal(ib["history"], ic["history"])
    nd = 400
    eig = np.array([1.0, 2.0, 3.0, 5.0, 8.0])
    ad = np.zeros((K, nd))
    ad[0] = eig[np.arange(nd) % eig.size]
    bd = random_mp(nd, K, np.random.default_rng(32))
    idx = np.arange(nd + 1, dtype=np.int32)
    for solve in (ref.cgs_k, ref.gpbicg_k):
        _, info = solve(K, idx, idx[:-1], ad, bd, precond="none", rtol=RTOL[K], max_iter=50)
        assert info["status"] == 0 and info["iters"] <= eig.size, solve.__name__
    rp, ci, a = banded_nonsymmetric(n=150, seed=5, K=K)
    b = ref.spmv(K, rp, ci, a, sqrt2_vector(150, K))
    for solve in (ref.bicg_k, ref.cgs_k, ref.gpbicg_k):
        x, info = solve(K, rp, ci, a, b, precond="jacobi", rtol=RTOL[K], max_iter=20000)
        assert info["status"] == 0, solve.__name__
        ok, rel = _certified(rp, ci, a, b, x, RTOL[K])
        assert ok, (solve.__name__, rel)


def test_k2_instances_are_the_dd_solvers():
    rp, ci, a = banded_nonsymmetric(n=200, seed=5)
    b = random_mp(200, 2, np.random.default_rng(33))
    for gen, dd in ((ref.bicg_k, ref.bicg), (ref.cgs_k, ref.cgs), (ref.gpbicg_k, ref.gpbicg)):
        xk, ik = gen(2, rp, ci, a, b, rtol=1e-28, max_iter=20000, history=True)
        xd, idd = dd(rp, ci, a, b, rtol=1e-28, max_iter=20000, history=True)
        assert np.array_equal(xk, xd) and np.array_equal(ik["history"], idd["history"])
        assert (ik["status"], ik["iters"]) == (idd["status"], idd["iters"])
