"""GPU parity of the TD / QD Krylov solvers (C ABI mpkrylov_{cg,bicgstab,cgs,gpbicg,bicg}_{td,qd}) with the
oracle's K-component solvers: same status, iteration count and restarts, bitwise
identical x and identical leading components of the true residual, with and without
Jacobi preconditioning and with a non-canonical plan, on an SPD 3D diffusion matrix
(also over several 4096-row chunks), the non-symmetric band, a one-eigenvalue diagonal
system (BiCGSTAB's half step), iteration limits, a NaN right-hand side, and argument
errors (a plan of the wrong precision, a short workspace)."""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import diffusion3d_7pt, banded_nonsymmetric, random_mp

pytestmark = pytest.mark.gpu

RTOL = {3: 1e-44, 4: 1e-60}


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def solvers(mp, K):
    return {"cg": (mp.mpkrylov_cg_td if K == 3 else mp.mpkrylov_cg_qd, ref.cg_k),
            "bicgstab": (mp.mpkrylov_bicgstab_td if K == 3 else mp.mpkrylov_bicgstab_qd, ref.bicgstab_k)}


def compare(mp, K, kind, rp, ci, a, b, precond, rtol, max_iter, plan=None, what="", values=True):
    import torch
    gfn, ofn = solvers(mp, K)[kind]
    A = mp.Csr.from_numpy(rp, ci)
    x = torch.zeros((K, rp.size - 1), dtype=torch.float64, device="cuda")
    ig = gfn(A, dev(a), dev(b), x, plan=plan, precond=precond, rtol=rtol, max_iter=max_iter, check_every=8)
    lw = None if plan is None else plan.row_log2w()
    xo, io = ofn(K, rp, ci, a, b, precond=precond, rtol=rtol, max_iter=max_iter, log2w=lw)
    assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), what
    if values:   # a NaN right-hand side leaves NaN iterates on both sides
        assert_same_values(host(x), xo, what + " x")
        assert_same_values(ig["rr_true"], io["rr_true"], what + " rr")
    return io


@pytest.mark.parametrize("K", [3, 4])
def test_cg_matches_oracle(mp, K):
    rp, ci, a = diffusion3d_7pt(m=6, sigma=1.0, seed=9, K=K)
    A = mp.Csr.from_numpy(rp, ci)
    b = random_mp(rp.size - 1, K, np.random.default_rng(21))
    for precond in ("none", "jacobi"):
        for plan in (None, mp.mp_plan_create(A, K, False, 2, 6)):
            io = compare(mp, K, "cg", rp, ci, a, b, precond, RTOL[K], 5000, plan, "cg K=%d %s" % (K, precond))
            assert io["status"] == 0
    rp, ci, a = diffusion3d_7pt(m=21, sigma=1.0, seed=10, K=K)   # 9261 rows: three chunks, ragged
    b = random_mp(rp.size - 1, K, np.random.default_rng(22))
    io = compare(mp, K, "cg", rp, ci, a, b, "jacobi", RTOL[K], 5000, None, "cg chunks K=%d" % K)
    assert io["status"] == 0


@pytest.mark.parametrize("K", [3, 4])
def test_bicgstab_matches_oracle(mp, K):
    rp, ci, a = banded_nonsymmetric(n=300, seed=6, K=K)
    A = mp.Csr.from_numpy(rp, ci)
    b = random_mp(300, K, np.random.default_rng(23))
    for precond in ("none", "jacobi"):
        for plan in (None, mp.mp_plan_create(A, K, False, 1, 6)):
            io = compare(mp, K, "bicgstab", rp, ci, a, b, precond, RTOL[K], 20000, plan,
                         "bicgstab K=%d %s" % (K, precond))
            assert io["status"] == 0
    rp, ci, a = diffusion3d_7pt(m=21, sigma=1.0, seed=11, K=K)
    b = random_mp(rp.size - 1, K, np.random.default_rng(24))
    io = compare(mp, K, "bicgstab", rp, ci, a, b, "jacobi", RTOL[K], 5000, None, "bicgstab chunks K=%d" % K)
    assert io["status"] == 0


@pytest.mark.parametrize("K", [3, 4])
def test_limits_half_step_breakdown_and_errors(mp, K):
    import torch
    rp, ci, a = banded_nonsymmetric(n=300, seed=6, K=K)
    b = random_mp(300, K, np.random.default_rng(25))
    for kind in ("cg", "bicgstab"):
        for lim in (1, 5, 11):
            io = compare(mp, K, kind, rp, ci, a, b, "none", RTOL[K], lim, None, "%s limit %d" % (kind, lim))
            assert io["status"] == -5 and io["iters"] == lim
        bad = b.copy()
        bad[0, 4] = np.nan
        io = compare(mp, K, kind, rp, ci, a, bad, "jacobi", RTOL[K], 50, None, "%s nan" % kind, values=False)
        assert io["status"] == -6
    # one distinct eigenvalue: BiCGSTAB's s vanishes after the first alpha (half step)
    n = 5000
    rpd = np.arange(n + 1, dtype=np.int32)
    cid = np.arange(n, dtype=np.int32)
    ad = np.zeros((K, n))
    ad[0] = 3.0
    bd = random_mp(n, K, np.random.default_rng(26))
    io = compare(mp, K, "bicgstab", rpd, cid, ad, bd, "none", RTOL[K], 50, None, "half step")
    assert io["status"] == 0 and io["iters"] == 1
    # argument errors
    A = mp.Csr.from_numpy(rp, ci)
    gfn = solvers(mp, K)["cg"][0]
    x = torch.zeros((K, 300), dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError):
        gfn(A, dev(a), dev(b), x, plan=mp.mp_plan_create(A, 2), rtol=RTOL[K])
    with pytest.raises(mp.MpError) as ei:
        gfn(A, dev(a), dev(b), x, ws=torch.empty(4096, dtype=torch.uint8, device="cuda"), rtol=RTOL[K])
    assert ei.value.status == -4


@pytest.mark.parametrize("K", [3, 4])
def test_cgs_gpbicg_bicg_match_oracle(mp, K):
    """TD / QD CGS, GPBiCG and BiCG (with the device transpose) equal the oracle's
    K-component solvers bit for bit on the non-symmetric band (with and without
    Jacobi, with a plan), over several chunks of a diffusion matrix, at iteration
    limits, and BiCG equals CG on a symmetric matrix."""
    import torch
    rp, ci, a = banded_nonsymmetric(n=300, seed=6, K=K)
    n = 300
    A = mp.Csr.from_numpy(rp, ci)
    ad = dev(a)
    b = random_mp(n, K, np.random.default_rng(40 + K))
    At, at, _ = mp.mp_csr_transpose(A, ad)
    cases = [("cgs", mp.mpkrylov_cgs_td if K == 3 else mp.mpkrylov_cgs_qd, ref.cgs_k),
             ("gpbicg", mp.mpkrylov_gpbicg_td if K == 3 else mp.mpkrylov_gpbicg_qd, ref.gpbicg_k)]
    bicg = mp.mpkrylov_bicg_td if K == 3 else mp.mpkrylov_bicg_qd
    for precond in ("none", "jacobi"):
        for plan in (None, mp.mp_plan_create(A, K, False, 1, 6)):
            lw = None if plan is None else plan.row_log2w()
            for name, gfn, ofn in cases:
                x = torch.zeros((K, n), dtype=torch.float64, device="cuda")
                ig = gfn(A, ad, dev(b), x, plan=plan, precond=precond, rtol=RTOL[K], max_iter=20000, check_every=8)
                xo, io = ofn(K, rp, ci, a, b, precond=precond, rtol=RTOL[K], max_iter=20000, log2w=lw)
                assert io["status"] == 0, name
                assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), name
                assert_same_values(host(x), xo, "%s x" % name)
                assert_same_values(ig["rr_true"], io["rr_true"], "%s rr" % name)
            x = torch.zeros((K, n), dtype=torch.float64, device="cuda")
            ig = bicg(A, ad, At, at, dev(b), x, plan=plan, precond=precond, rtol=RTOL[K], max_iter=20000,
                      check_every=8)
            xo, io = ref.bicg_k(K, rp, ci, a, b, precond=precond, rtol=RTOL[K], max_iter=20000, log2w=lw)
            assert io["status"] == 0
            assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"])
            assert_same_values(host(x), xo, "bicg x")
    # iteration limits inside a check chunk
    for name, gfn, ofn in cases:
        for lim in (1, 5):
            x = torch.zeros((K, n), dtype=torch.float64, device="cuda")
            ig = gfn(A, ad, dev(b), x, precond="none", rtol=RTOL[K], max_iter=lim, check_every=4)
            xo, io = ofn(K, rp, ci, a, b, precond="none", rtol=RTOL[K], max_iter=lim)
            assert io["status"] == -5 and (ig["status"], ig["iters"]) == (io["status"], io["iters"]), name
            assert_same_values(host(x), xo, "%s limit x" % name)
    # several chunks of rows
    rpd, cid, adf = diffusion3d_7pt(m=21, sigma=1.0, seed=12, K=K)
    nd = rpd.size - 1
    bd = random_mp(nd, K, np.random.default_rng(50 + K))
    Ad = mp.Csr.from_numpy(rpd, cid)
    for name, gfn, ofn in cases:
        x = torch.zeros((K, nd), dtype=torch.float64, device="cuda")
        ig = gfn(Ad, dev(adf), dev(bd), x, precond="jacobi", rtol=RTOL[K], max_iter=5000)
        xo, io = ofn(K, rpd, cid, adf, bd, precond="jacobi", rtol=RTOL[K], max_iter=5000)
        assert io["status"] == 0 and (ig["status"], ig["iters"], ig["restarts"]) == (0, io["iters"], io["restarts"])
        assert_same_values(host(x), xo, "%s chunks x" % name)
    # BiCG = CG on a symmetric matrix
    Atd, atd, _ = mp.mp_csr_transpose(Ad, dev(adf))
    xb = torch.zeros((K, nd), dtype=torch.float64, device="cuda")
    xc = torch.zeros((K, nd), dtype=torch.float64, device="cuda")
    ib = bicg(Ad, dev(adf), Atd, atd, dev(bd), xb, precond="jacobi", rtol=RTOL[K], max_iter=5000)
    cg = mp.mpkrylov_cg_td if K == 3 else mp.mpkrylov_cg_qd
    ic = cg(Ad, dev(adf), dev(bd), xc, precond="jacobi", rtol=RTOL[K], max_iter=5000)
    assert ib["status"] == ic["status"] == 0 and ib["iters"] == ic["iters"]
    assert_same_values(host(xb), host(xc), "bicg = cg")
