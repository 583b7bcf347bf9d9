"""GPU checks of the learned refinement preconditioner (C ABI mp_mpnn_*, mp_graph_*,
mpkrylov_ir_learned).

* Forward: on a 24^3 graph every element of M is within a per-element bound derived
  from the readouts' magnitudes (forward_bound) of the oracle's; a matrix with a
  positive off-diagonal entry is refused (M is guaranteed SPD for Stieltjes matrices);
  on small graphs M
  from the GPU network equals the oracle network (bfloat16 mode) within
  1e-3 of max|M| (float32 accumulation against binary64; a rare float32 difference
  can move a value across a bfloat16 rounding boundary, one bfloat16 ulp = 2^-8
  relative, which the bound covers), with the median element error below 1e-5 of
  max|M|; with zero weights M equals the oracle's (the Jacobi inverse diagonal)
  bit for bit.
* Backward: summed gradients of two pairs equal the oracle's (bfloat16 mode) within
  1e-3 in norm per parameter block, losses within 1e-4 relative; Adam equals the
  oracle's step.
* Learned refinement: with M values computed by the oracle network and uploaded,
  iterates, counts and status equal the oracle's refinement with the same M bit for
  bit (binary64 and binary32 inner, and the Jacobi DD CG fallback after a stall);
  the zero-weight network reproduces Jacobi refinement exactly.
* Training on the GPU lowers the mean loss, and the trained network needs fewer inner
  iterations than Jacobi on held-out matrices (both certified to 1e-28); the committed
  network solves the benchmark's 64^3 system in less wall time than Jacobi refinement,
  forward pass included.
"""
import numpy as np
import pytest

from oracle import mpnn, ref
from tests.helpers import assert_same_values, dev, host
from workloads import diffusion3d_7pt, random_mp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def problem(m, seed, sigma=2.0):
    rp, ci, a = diffusion3d_7pt(m=m, sigma=sigma, seed=seed)
    return rp, ci, a, mpnn.Graph(rp, ci, a[0])


def gpu_graph(mp, rp, ci, a):
    A = mp.Csr.from_numpy(rp, ci)
    ad = dev(a)
    return A, ad, mp.Graph(A, ad)


def test_forward_matches_oracle(mp):
    import torch
    rp, ci, a, g = problem(6, 71)
    A, ad, gg = gpu_graph(mp, rp, ci, a)
    net = mp.Mpnn()
    for scale in (0.5, 2.0):
        theta = mpnn.init_params(11, scale=scale).astype(np.float32)
        net.set_params(theta)
        assert np.array_equal(net.get_params(), theta)
        Mg = host(mp.mp_mpnn_forward(net, gg))
        torch.cuda.synchronize()
        Mr, _ = mpnn.forward(g, theta.astype(np.float64), bf=True)
        err = np.abs(Mg - Mr)
        scale_m = np.abs(Mr).max()
        assert err.max() <= 1e-3 * scale_m, (scale, err.max() / scale_m)
        assert np.median(err) <= 1e-5 * scale_m
    net.set_params(np.zeros(net.n_params, np.float32))
    Mg = host(mp.mp_mpnn_forward(net, gg))
    Mr, _ = mpnn.forward(g, np.zeros(mpnn.n_params()), bf=True)
    assert_same_values(Mg, Mr, "zero network")


def forward_bound(g, c, theta):
    """Per-element bound on |M_gpu - M_oracle| (the network's forward pass on the GPU in
    float32 against the oracle's binary64 pass, both with bfloat16 weights and layer
    inputs).  The readouts u_i = h_i.wu + bu and v_ij = sum_k qv_k h_ik h_jk + bv of the
    two passes differ by at most 2^-6 of their absolute-term sums
        E_u,i = sum_k |wu_k h_ik| + |bu|,   E_v,ij = sum_k |qv_k h_ik h_jk| + |bv|
    (float32 accumulation contributes ~2^-17 of them; the rest covers isolated bfloat16
    rounding flips upstream, each moving one input by 2^-8 of itself).  Since
    g = tanh(v)^2 and delta = log(1 + u^2) have slopes at most 4/(3 sqrt 3) < 0.77 and 1,
    M_ij = g_ij w_ij sqrt(m_i m_j) and M_ii = (1 + delta_i) m_i (m = 1/a_ii) move by at
    most 0.77 2^-6 E_v,ij |w_ij| sqrt(m_i m_j) and 2^-6 E_u,i m_i, plus the float32
    rounding of the assembly on the GPU (2^-21 of |M|)."""
    p = mpnn.unpack(theta.astype(np.float64))
    H = np.abs(c["Hq"])
    qv = np.abs(mpnn.bf16(p["qv"]))
    wu = np.abs(mpnn.bf16(p["wu"]))
    Ev = (H[g.rows] * H[g.ci]) @ qv + abs(p["bv"][0])
    Eu = H @ wu + abs(p["bu"][0])
    eps = 2.0 ** -6
    Mr, _ = mpnn.forward(g, theta.astype(np.float64), bf=True)
    tau = np.where(g.offd, 0.77 * eps * Ev * np.abs(g.w) * np.sqrt(g.minv[g.rows] * g.minv[g.ci]), 0.0)
    dmask = ~g.offd
    tau[dmask] = (eps * Eu * g.minv)[g.rows[dmask]]
    return tau + 2.0 ** -21 * np.abs(Mr)


def test_forward_per_element_bound_24cubed(mp):
    """A 24^3 graph (13,824 nodes, 93,312 elements) of the training law: every element of
    the GPU's M within the per-element bound above of the oracle's, for random
    networks of two weight scales and for the trained network."""
    import os
    import torch
    rp, ci, a, g = problem(24, 73, sigma=2.5)
    A, ad, gg = gpu_graph(mp, rp, ci, a)
    net = mp.Mpnn()
    thetas = [mpnn.init_params(13, scale=0.5).astype(np.float32), mpnn.init_params(14, scale=2.0).astype(np.float32)]
    ckpt = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2412_17510_amd", "data",
                        "mpnn_diffusion.npz")
    if os.path.exists(ckpt):
        with np.load(ckpt, allow_pickle=False) as f:
            thetas.append(f["theta"].astype(np.float32))
    for k, theta in enumerate(thetas):
        net.set_params(theta)
        Mg = host(mp.mp_mpnn_forward(net, gg))
        torch.cuda.synchronize()
        Mr, c = mpnn.forward(g, theta.astype(np.float64), bf=True)
        tau = forward_bound(g, c, theta)
        ratio = np.abs(Mg - Mr) / tau
        print("network %d: max |dM| / bound %.3g, elements equal %.4f" % (k, ratio.max(), np.mean(Mg == Mr)),
              flush=True)
        assert np.all(np.abs(Mg - Mr) <= tau), (k, int(np.argmax(ratio)), ratio.max())


def test_graph_refuses_positive_off_diagonal(mp):
    rp, ci, a, g = problem(5, 75)
    bad = a.copy()
    k = int(np.nonzero(g.offd)[0][3])
    bad[0, k] = abs(bad[0, k])
    A = mp.Csr.from_numpy(rp, ci)
    with pytest.raises(mp.MpError) as ei:
        mp.Graph(A, dev(bad))
    assert ei.value.status == -1


def test_gradients_match_oracle(mp):
    import torch
    rp, ci, a, g = problem(5, 72)
    A, ad, gg = gpu_graph(mp, rp, ci, a)
    theta = mpnn.init_params(12, scale=1.0).astype(np.float32)
    rng = np.random.default_rng(72)
    E = rng.standard_normal((2, g.n))
    R = np.stack([g.spmv(g.a_hi, E[p]) for p in range(2)])
    net = mp.Mpnn()
    net.set_params(theta)
    net.zero_grads()
    losses = mp.mp_mpnn_loss_grad(net, gg, dev(R), dev(E))
    grads = net.get_grads().astype(np.float64)
    want_l, want_g = [], np.zeros(mpnn.n_params())
    for p in range(2):
        L, gr = mpnn.backward(g, theta.astype(np.float64), R[p], E[p], bf=True)
        want_l.append(L)
        want_g += gr
    np.testing.assert_allclose(losses, want_l, rtol=1e-4)
    off = 0
    for name, shp in mpnn.param_shapes():
        k = int(np.prod(shp))
        gw, gx = want_g[off:off + k], grads[off:off + k]
        assert np.linalg.norm(gx - gw) <= 1e-3 * np.linalg.norm(gw) + 1e-12, name
        off += k
    # the accumulator adds: a second call doubles the gradient
    mp.mp_mpnn_loss_grad(net, gg, dev(R), dev(E))
    np.testing.assert_allclose(net.get_grads(), 2.0 * grads, rtol=1e-6, atol=1e-30)
    # Adam against the oracle's step (float32 master weights)
    net.zero_grads()
    mp.mp_mpnn_loss_grad(net, gg, dev(R), dev(E))
    g32 = net.get_grads().astype(np.float64)
    net.adam_step(1, lr=1e-2, grad_scale=0.5)
    torch.cuda.synchronize()
    want, _, _ = mpnn.adam(theta.astype(np.float64), 0.5 * g32, 0.0, 0.0, 1, lr=1e-2)
    np.testing.assert_allclose(net.get_params(), want, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_learned_ir_matches_oracle(mp, inner):
    import torch
    rp, ci, a, g = problem(7, 73)
    n = g.n
    theta = mpnn.init_params(13, scale=2.0)
    Mr, _ = mpnn.forward(g, theta, bf=True)
    b = random_mp(n, 2, np.random.default_rng(73))
    kw = dict(inner=inner, inner_rtol=1e-5, rtol=1e-28)
    xo, io = ref.ir(rp, ci, a, b, m_values=Mr, inner_max_iter=400, **kw)
    A = mp.Csr.from_numpy(rp, ci)
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    ig = mp.mpkrylov_ir_learned(A, dev(a), dev(Mr), dev(b), x, inner_max_iter=400, **kw)
    assert io["status"] == 0 and io["fell_back"] == 0
    for k in ("status", "iters", "outer_iters", "fell_back"):
        assert ig[k] == io[k], k
    assert_same_values(host(x), xo, "learned IR x")
    assert_same_values(ig["rr_true"], io["rr_true"], "learned IR rr")
    # stall -> Jacobi DD CG fallback
    xo, io = ref.ir(rp, ci, a, b, m_values=Mr, inner_max_iter=1, **kw)
    x.zero_()
    ig = mp.mpkrylov_ir_learned(A, dev(a), dev(Mr), dev(b), x, inner_max_iter=1, **kw)
    assert io["fell_back"] == 1 and io["status"] == 0
    for k in ("status", "iters", "outer_iters", "fell_back"):
        assert ig[k] == io[k], k
    assert_same_values(host(x), xo, "fallback x")


def test_zero_network_reproduces_jacobi_ir(mp):
    import torch
    rp, ci, a, g = problem(8, 74)
    A, ad, gg = gpu_graph(mp, rp, ci, a)
    n = g.n
    net = mp.Mpnn()
    M = mp.mp_mpnn_forward(net, gg)
    bd = dev(random_mp(n, 2, np.random.default_rng(74)))
    for inner in ("fp64", "fp32"):
        xj = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        xl = torch.zeros_like(xj)
        ij = mp.mpkrylov_ir(A, ad, bd, xj, inner=inner, inner_rtol=1e-6, rtol=1e-28)
        il = mp.mpkrylov_ir_learned(A, ad, M, bd, xl, inner=inner, inner_rtol=1e-6, rtol=1e-28)
        assert ij["status"] == 0
        for k in ("status", "iters", "outer_iters", "fell_back"):
            assert ij[k] == il[k], (inner, k)
        assert_same_values(host(xl), host(xj), "zero network vs Jacobi (%s)" % inner)


def test_learned_ir_rejects_wrong_precond_and_alias(mp):
    import torch
    rp, ci, a, g = problem(4, 75)
    A = mp.Csr.from_numpy(rp, ci)
    n = g.n
    ad = dev(a)
    b = dev(random_mp(n, 2, np.random.default_rng(75)))
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError):
        mp.mpkrylov_ir(A, ad, b, x, precond="learned")
    big = torch.zeros(2 * n + A.nnz, dtype=torch.float64, device="cuda")
    xv = big[:2 * n].view(2, n)
    with pytest.raises(mp.MpError):   # M overlapping x
        mp.mpkrylov_ir_learned(A, ad, big[n:n + A.nnz], b, xv)


def test_training_beats_jacobi_on_held_out(mp):
    import torch
    from paper_2412_17510_amd import learned
    tr = learned.Trainer(learned.init_params(0, scale=0.1), lr=3e-3)
    keep = []
    for seed in (81, 82, 83):
        rp, ci, a = diffusion3d_7pt(m=10, sigma=2.0, seed=seed)
        A = mp.Csr.from_numpy(rp, ci)
        ad = dev(a)
        xt = dev(random_mp(rp.size - 1, 2, np.random.default_rng(seed)))
        R, E = learned.cg_pairs(A, ad, xt)
        tr.add(A, ad, R, E)
        keep.append((A, ad))
    l0 = tr.mean_loss()
    for _ in range(200):
        tr.step()
    l1 = tr.mean_loss()
    assert l1 < 0.8 * l0, (l0, l1)
    tot_l = tot_j = 0
    for seed in (91, 92):
        rp, ci, a = diffusion3d_7pt(m=12, sigma=2.0, seed=seed)
        n = rp.size - 1
        A = mp.Csr.from_numpy(rp, ci)
        ad = dev(a)
        bd = dev(random_mp(n, 2, np.random.default_rng(seed)))
        M = learned.m_values(tr.net, A, ad)
        xj = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        xl = torch.zeros_like(xj)
        ij = mp.mpkrylov_ir(A, ad, bd, xj, inner="fp64", inner_rtol=1e-8, rtol=1e-28)
        il = mp.mpkrylov_ir_learned(A, ad, M, bd, xl, inner="fp64", inner_rtol=1e-8, rtol=1e-28)
        assert ij["status"] == 0 and il["status"] == 0 and il["fell_back"] == 0
        assert il["relres"] <= 1e-28 * 1.01
        tot_l += il["iters"]
        tot_j += ij["iters"]
    assert tot_l < 0.9 * tot_j, (tot_l, tot_j)


def test_trained_network_wins_on_time(mp):
    """The committed network on the benchmark's sigma = 2.5 64^3 system: learned refinement
    (forward pass included) solves to 1e-28 in less wall time than Jacobi refinement
    (best of three each, binary64 inner), with under 0.7x its inner iterations, and
    both certified by the exact residual."""
    import os
    import time
    import torch
    from oracle import ref as oref
    from workloads.condition import load_law
    ckpt = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2412_17510_amd", "data",
                        "mpnn_diffusion.npz")
    with np.load(ckpt, allow_pickle=False) as f:
        theta = f["theta"].astype(np.float32)
    law = load_law()["systems"][0]
    rp, ci, a = diffusion3d_7pt(m=law["m"], sigma=law["sigma"], az=law["az"], seed=law["seed"])
    n = rp.size - 1
    b = random_mp(n, 2, np.random.default_rng(law["seed"]))
    A = mp.Csr.from_numpy(rp, ci)
    ad, bd = dev(a), dev(b)
    plan, _ = mp.mp_plan_autotune(A, 2, ad, bd, torch.empty((2, n), dtype=torch.float64, device="cuda"), reps=3)
    net = mp.Mpnn()
    net.set_params(theta)
    kw = dict(plan=plan, rtol=1e-28, inner="fp64", inner_rtol=1e-8, inner_max_iter=50000, max_outer=60)
    best_j = best_l = None
    for _ in range(3):
        xj = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        ij = mp.mpkrylov_ir(A, ad, bd, xj, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = mp.Graph(A, ad)
        M = mp.mp_mpnn_forward(net, g)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        g.destroy()
        xl = torch.zeros_like(xj)
        il = mp.mpkrylov_ir_learned(A, ad, M, bd, xl, **kw)
        tj, tl = ij["seconds"], il["seconds"] + t_fwd
        best_j = tj if best_j is None else min(best_j, tj)
        best_l = tl if best_l is None else min(best_l, tl)
    print("jacobi refinement %.4f s (%d inner), learned %.4f s (%d inner)" % (best_j, ij["iters"], best_l, il["iters"]),
          flush=True)
    assert ij["status"] == 0 and il["status"] == 0 and il["fell_back"] == 0
    assert il["iters"] < 0.7 * ij["iters"]
    assert best_l < best_j
    for x in (xj, xl):
        assert oref.exact_residual(rp, ci, a, b, host(x))["relres_upper"] <= 1e-28
