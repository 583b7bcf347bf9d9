"""Pins of the oracle's message-passing preconditioner network (CPU only).

* bfloat16 rounding equals torch's float32 -> bfloat16 conversion (round to nearest,
  ties to even), including exact ties;
* with every parameter zero the network's M is exactly the Jacobi inverse diagonal;
* for random (large) weights M is symmetric and positive definite, and v_ij = v_ji;
* with g_ij -> 1 and delta = 0 (readout bias bv large, every other weight zero) M is
  the first-order Neumann approximate inverse D^-1 + D^-1 N D^-1 (N = the negated
  off-diagonal part of A), entry for entry, and still positive definite on a strongly
  heterogeneous matrix;
* the analytic gradient equals central finite differences of the loss (binary64
  network, every parameter block, relative-or-absolute tolerance);
* the loss is 0 with a zero gradient when e = M r;
* the gradient summed over two pairs is the sum of the per-pair gradients (linearity
  used by the GPU's pair loop).
"""
import numpy as np
import pytest

from oracle import mpnn
from workloads import diffusion3d_7pt, random_mp


def graph(m=5, seed=31, sigma=2.0):
    rp, ci, a = diffusion3d_7pt(m=m, sigma=sigma, seed=seed)
    return mpnn.Graph(rp, ci, a[0]), rp, ci, a


def pair(g, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(g.n)
    r = g.spmv(g.a_hi, e)
    return r, e


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32) * np.float32(10.0) ** rng.integers(-8, 8, 5000),
                        np.float32([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0, 3.0e38])])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = mpnn.bf16(x)
    assert np.array_equal(got, want)
    assert mpnn.bf16(np.float32(1.0 + 2 ** -8)) == 1.0                 # tie -> even (down)
    assert mpnn.bf16(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6    # tie -> even (up)


def test_zero_network_is_jacobi():
    g, rp, ci, a = graph()
    theta = np.zeros(mpnn.n_params())
    for bf in (False, True):
        M, _ = mpnn.forward(g, theta, bf=bf)
        diag = g.rows == g.ci
        assert np.array_equal(M[diag], 1.0 / a[0][diag])
        assert np.all(M[~diag] == 0.0)
    assert mpnn.n_params() == 4 * 64 + 64 + 3 * (2 * 64 * 64 + 64) + 64 + 1 + 64 + 1


@pytest.mark.parametrize("scale", [0.5, 3.0])
def test_m_is_spd_and_symmetric(scale):
    g, rp, ci, a = graph(m=4, seed=32)
    theta = mpnn.init_params(7, scale=scale)
    M, c = mpnn.forward(g, theta, bf=True)
    n = g.n
    D = np.zeros((n, n))
    D[g.rows, g.ci] = M
    assert np.array_equal(D, D.T)
    Vd = np.zeros((n, n))
    Vd[g.rows, g.ci] = np.where(g.offd, c["v"], 0.0)
    assert np.array_equal(Vd, Vd.T)
    assert np.linalg.eigvalsh(D).min() > 0.0
    if scale >= 3.0:   # off-diagonal entries are really used (not a degenerate diagonal M)
        assert np.abs(M[g.offd]).max() > 1e-3 * np.abs(M[~g.offd]).max()


def test_neumann_limit():
    g, rp, ci, a = graph(m=5, seed=36, sigma=3.0)
    p = {name: np.zeros(shp) for name, shp in mpnn.param_shapes()}
    p["bv"] = np.array([20.0])           # tanh(20)^2 = 1 to binary64 precision
    theta = mpnn.pack(p)
    M, c = mpnn.forward(g, theta)
    hi = a[0]
    diag = np.zeros(g.n)
    diag[g.rows[~g.offd]] = hi[~g.offd]
    want = np.where(g.offd, -hi / (diag[g.rows] * diag[g.ci]), 1.0 / diag[g.rows])
    # w is held in float32 (the network's input), so agreement is to float32 rounding
    np.testing.assert_allclose(M, want, rtol=2e-7, atol=0)
    n = g.n
    D = np.zeros((n, n))
    D[g.rows, g.ci] = M
    assert np.linalg.eigvalsh(D).min() > 0.0


def test_gradient_matches_finite_differences():
    g, rp, ci, a = graph(m=4, seed=33)
    theta = mpnn.init_params(3, scale=1.0)
    r, e = pair(g, 5)
    L, grad = mpnn.backward(g, theta, r, e, bf=False)
    assert np.isfinite(L) and L > 0
    rng = np.random.default_rng(9)
    off = 0
    checked = 0
    for name, shp in mpnn.param_shapes():
        k = int(np.prod(shp))
        idx = np.unique(rng.integers(off, off + k, size=min(k, 6)))
        for i in idx:
            h = 1e-5 * max(1.0, abs(theta[i]))
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            Lp = mpnn.loss(g, mpnn.forward(g, tp)[0], r, e)[0]
            Lm = mpnn.loss(g, mpnn.forward(g, tm)[0], r, e)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-5 * abs(grad).max() + 1e-4 * abs(grad[i]), (name, i, fd, grad[i])
            checked += 1
        off += k
    assert checked > 40


def test_loss_zero_at_exact_pair():
    g, rp, ci, a = graph(m=4, seed=34)
    theta = mpnn.init_params(4, scale=1.0)
    M, _ = mpnn.forward(g, theta, bf=True)
    r = np.random.default_rng(1).standard_normal(g.n)
    e = g.spmv(M, r)
    L, grad = mpnn.backward(g, theta, r, e, bf=True)
    assert L == 0.0
    assert np.all(grad == 0.0)


def test_gradient_is_additive_over_pairs():
    g, rp, ci, a = graph(m=4, seed=35)
    theta = mpnn.init_params(5, scale=1.0)
    r1, e1 = pair(g, 1)
    r2, e2 = pair(g, 2)
    L1, g1 = mpnn.backward(g, theta, r1, e1, bf=True)
    L2, g2 = mpnn.backward(g, theta, r2, e2, bf=True)
    # loss of a pair depends on the pair only: scaling (r, e) together leaves it unchanged
    L3, g3 = mpnn.backward(g, theta, 4.0 * r1, 4.0 * e1, bf=True)
    assert L3 == pytest.approx(L1, rel=1e-12)
    np.testing.assert_allclose(g3, g1, rtol=1e-9, atol=1e-12 * abs(g1).max())
    assert L1 != L2


def test_adam_first_step_is_signed_learning_rate():
    """After bias correction the first step moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(100) * 10.0 ** rng.integers(-3, 3, 100)
    theta = rng.standard_normal(100)
    t1, m, v = mpnn.adam(theta, g, np.zeros(100), np.zeros(100), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(t1, theta - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    # a constant gradient keeps the step at lr (bias-corrected moments equal g and g^2)
    t, m, v = theta, np.zeros(100), np.zeros(100)
    for s in range(1, 6):
        t, m, v = mpnn.adam(t, g, m, v, s, lr=0.01, eps=0.0)
    np.testing.assert_allclose(t, theta - 0.05 * np.sign(g), rtol=0, atol=1e-12)
