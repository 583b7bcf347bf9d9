"""GPU checks of the batched block-diagonal layer (C ABI mpspmm_csr_dd_batched,
mpkrylov_cg_batched).

* SpMM: every right-hand side equals the oracle's single-vector SpMV with W = 1 order,
  bitwise, for every threads-per-row mapping (the autotuner's search space), and at the
  benchmark's full size (256 systems, 17.7 M rows, 8 right-hand sides) in every row.
* Batched CG: every (system, rhs) pair equals a separate oracle DD CG solve with the
  same order (status, iterations, restarts, bitwise x and true residual); the hipGraph
  replay path equals the eager path bitwise; a pair equals the GPU's own single-system
  mpkrylov_cg with a W = 1 plan.
* Systems of several 4096-row dot chunks (grid edges 12..33, 1,728..35,937 rows, 8
  right-hand sides): every pair after a capped number of iterations, and every pair of
  two multi-chunk systems solved to 1e-28, equal to separate oracle solves, in the
  graph and the eager path.
* A matrix with an entry outside its system's block is refused.
"""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import batched_diffusion, random_mp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def multi(rng, N, R):
    """(2, N, R) DD multi-vector with random leads and tails."""
    v = random_mp(N * R, 2, rng)
    return np.ascontiguousarray(v.reshape(2, N, R))


@pytest.mark.parametrize("R", [1, 4, 8])
def test_batched_spmm_matches_single_spmv(mp, R):
    import torch
    rp, ci, a, sp = batched_diffusion([5, 7, 4, 9], sigma=2.0, seed=41)
    N = rp.size - 1
    rng = np.random.default_rng(41 + R)
    X = multi(rng, N, R)
    A = mp.Csr.from_numpy(rp, ci)
    want = [ref.spmv(2, rp, ci, a, np.ascontiguousarray(X[:, :, r]), log2w=np.zeros(N, np.uint8)) for r in range(R)]
    for tpr in [t for t in (1, 2, 4, 8) if t <= R]:
        plan = mp.mp_batch_plan_create(A, sp, R, tpr)
        Y = torch.full((2, N, R), float("nan"), dtype=torch.float64, device="cuda")
        mp.mpspmm_csr_dd_batched(A, dev(a), dev(X), Y, R, plan=plan)
        torch.cuda.synchronize()
        Yh = host(Y)
        for r in range(R):
            assert_same_values(Yh[:, :, r], want[r], "spmm tpr=%d rhs %d" % (tpr, r))
    plan = mp.mp_batch_plan_create(A, sp, R, 1)
    Y = torch.empty((2, N, R), dtype=torch.float64, device="cuda")
    tpr = mp.mp_batch_plan_autotune(plan, A, dev(a), dev(X), Y)
    assert tpr in (1, 2, 4, 8) and tpr <= R


def test_batched_spmm_full_size(mp):
    """The benchmark's 256 systems (edges U{12..60}, 17.7 M rows, 122 M nnz) x 8
    right-hand sides: every row of every right-hand side equal to the oracle's W = 1
    SpMV, under the autotuned schedule and under one and eight threads per row."""
    import torch
    from workloads import configs
    from workloads.condition import load_law
    az = load_law()["systems"][0]["az"]
    rp, ci, a, sp = configs.c3_systems(az)
    N, R = rp.size - 1, configs.load("c3")["nrhs"]
    print("batched full size: N=%d nnz=%d" % (N, ci.size), flush=True)
    X = configs.c3_rhs(N)
    A = mp.Csr.from_numpy(rp, ci)
    ad, Xd = dev(a), dev(X)
    Y = torch.empty((2, N, R), dtype=torch.float64, device="cuda")
    plan = mp.mp_batch_plan_create(A, sp, R, 1)
    tuned = mp.mp_batch_plan_autotune(plan, A, ad, Xd, Y)
    got = {}
    for tpr in sorted({tuned, 1, 8}):
        pl = mp.mp_batch_plan_create(A, sp, R, tpr)
        Y.fill_(float("nan"))
        mp.mpspmm_csr_dd_batched(A, ad, Xd, Y, R, plan=pl)
        torch.cuda.synchronize()
        got[tpr] = host(Y)
    del Y, Xd, ad
    zero = np.zeros(N, np.uint8)
    for r in range(R):
        want = ref.spmv(2, rp, ci, a, np.ascontiguousarray(X[:, :, r]), log2w=zero)
        for tpr, Yh in got.items():
            assert_same_values(Yh[:, :, r], want, "full-size spmm tpr=%d rhs %d" % (tpr, r))


@pytest.mark.parametrize("precond", ["jacobi", "none"])
def test_batched_cg_matches_single_solves(mp, precond):
    import torch
    edges = [4, 6, 5, 7, 3, 6]
    rp, ci, a, sp = batched_diffusion(edges, sigma=2.0, seed=42)
    N = rp.size - 1
    R = 4
    rng = np.random.default_rng(42)
    B = multi(rng, N, R)
    A = mp.Csr.from_numpy(rp, ci)
    plan = mp.mp_batch_plan_create(A, sp, R, 2)
    results = {}
    for use_graph in (True, False):
        X = torch.zeros((2, N, R), dtype=torch.float64, device="cuda")
        infos = mp.mpkrylov_cg_batched(A, dev(a), dev(B), X, R, plan, use_graph=use_graph, precond=precond,
                                       rtol=1e-28, max_iter=3000, check_every=8)
        results[use_graph] = (host(X), infos)
    assert_same_values(results[True][0], results[False][0], "graph vs eager")
    Xg, infos = results[True]
    for s in range(len(edges)):
        r0, r1 = sp[s], sp[s + 1]
        rps = (rp[r0:r1 + 1] - rp[r0]).astype(np.int32)
        cis = (ci[rp[r0]:rp[r1]] - r0).astype(np.int32)
        a_s = np.ascontiguousarray(a[:, rp[r0]:rp[r1]])
        for r in range(R):
            b_s = np.ascontiguousarray(B[:, r0:r1, r])
            xo, io = ref.cg(rps, cis, a_s, b_s, precond=precond, rtol=1e-28, max_iter=3000,
                            log2w=np.zeros(r1 - r0, np.uint8))
            ig = infos[s * R + r]
            assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), (s, r)
            assert_same_values(Xg[:, r0:r1, r], xo, "pair (%d, %d) x" % (s, r))
            assert_same_values(ig["rr_true"], io["rr_true"], "pair (%d, %d) rr" % (s, r))
            assert ig["status"] == 0
    # one pair against the GPU's own single-system solver with a W = 1 plan
    s, r = 3, 2
    r0, r1 = sp[s], sp[s + 1]
    rps = (rp[r0:r1 + 1] - rp[r0]).astype(np.int32)
    cis = (ci[rp[r0]:rp[r1]] - r0).astype(np.int32)
    As = mp.Csr.from_numpy(rps, cis)
    p1 = mp.mp_plan_create(As, 2, False, 0, 0)
    xs = torch.zeros((2, r1 - r0), dtype=torch.float64, device="cuda")
    mp.mpkrylov_cg(As, dev(np.ascontiguousarray(a[:, rp[r0]:rp[r1]])), dev(np.ascontiguousarray(B[:, r0:r1, r])),
                   xs, plan=p1, precond=precond, rtol=1e-28, max_iter=3000)
    assert_same_values(host(xs), Xg[:, r0:r1, r], "batched vs single GPU solve")


def compare_pairs(mp, edges, R, seed, max_iter, precond="jacobi", converged=False):
    import torch
    rp, ci, a, sp = batched_diffusion(edges, sigma=2.5, seed=seed)
    N = rp.size - 1
    rng = np.random.default_rng(seed)
    B = multi(rng, N, R)
    A = mp.Csr.from_numpy(rp, ci)
    plan = mp.mp_batch_plan_create(A, sp, R, 2)
    results = {}
    for use_graph in (True, False):
        print("batched edges=%s R=%d max_iter=%d graph=%s" % (edges, R, max_iter, use_graph), flush=True)
        X = torch.zeros((2, N, R), dtype=torch.float64, device="cuda")
        infos = mp.mpkrylov_cg_batched(A, dev(a), dev(B), X, R, plan, use_graph=use_graph, precond=precond,
                                       rtol=1e-28, max_iter=max_iter, check_every=8)
        results[use_graph] = (host(X), infos)
    assert_same_values(results[True][0], results[False][0], "graph vs eager")
    for g in (True, False):
        assert [i["iters"] for i in results[True][1]] == [i["iters"] for i in results[g][1]]
    Xg, infos = results[True]
    for s in range(len(edges)):
        r0, r1 = sp[s], sp[s + 1]
        rps = (rp[r0:r1 + 1] - rp[r0]).astype(np.int32)
        cis = (ci[rp[r0]:rp[r1]] - r0).astype(np.int32)
        a_s = np.ascontiguousarray(a[:, rp[r0]:rp[r1]])
        for r in range(R):
            b_s = np.ascontiguousarray(B[:, r0:r1, r])
            xo, io = ref.cg(rps, cis, a_s, b_s, precond=precond, rtol=1e-28, max_iter=max_iter,
                            log2w=np.zeros(r1 - r0, np.uint8))
            ig = infos[s * R + r]
            assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), (s, r)
            assert_same_values(Xg[:, r0:r1, r], xo, "pair (%d, %d) x" % (s, r))
            assert_same_values(ig["rr_true"], io["rr_true"], "pair (%d, %d) rr" % (s, r))
            assert_same_values(ig["bb"], io["bb"], "pair (%d, %d) bb" % (s, r))
            if converged:
                assert ig["status"] == 0
    return infos


def test_batched_cg_multi_chunk_capped(mp):
    """Five systems of 1..9 dot chunks, 8 right-hand sides each, 40 iterations: every
    pair's iterate equals the oracle's (the per-system chunk boundaries and the
    multi-chunk reduction trees of every scalar)."""
    infos = compare_pairs(mp, [12, 17, 20, 24, 33], 8, 44, 40)
    assert all(i["status"] == -5 and i["iters"] == 40 for i in infos)


def test_batched_cg_multi_chunk_converged(mp):
    """Two multi-chunk systems (4,913 and 8,000 rows), 8 right-hand sides, solved to
    1e-28: every pair equals the oracle's solve, status and iteration count included."""
    compare_pairs(mp, [17, 20], 8, 45, 20000, converged=True)


def test_batched_schedules_give_the_same_solves(mp):
    """Every schedule of the persistent step (threads per row, SpMM tile rows, chunk
    order) and the autotuned one give the same pairs bit for bit (graph path), on
    systems of several dot chunks; the schedule setter refuses bad values."""
    import torch
    rp, ci, a, sp = batched_diffusion([20, 12, 17, 9], sigma=2.5, seed=46)
    N = rp.size - 1
    R = 8
    B = multi(np.random.default_rng(46), N, R)
    A = mp.Csr.from_numpy(rp, ci)
    ad, Bd = dev(a), dev(B)
    plan = mp.mp_batch_plan_create(A, sp, R, 1)
    ref_x, ref_it = None, None
    for sched in ((1, 1, 0), (2, 4, 1), (8, 2, 1), (4, 1, 0), None):
        if sched is None:
            mp.mp_batch_plan_autotune(plan, A, ad, Bd, torch.empty((2, N, R), dtype=torch.float64, device="cuda"))
        else:
            mp.mp_batch_plan_set_schedule(plan, *sched)
        got = mp.mp_batch_plan_schedule(plan)
        print("schedule", got, flush=True)
        X = torch.zeros((2, N, R), dtype=torch.float64, device="cuda")
        infos = mp.mpkrylov_cg_batched(A, ad, Bd, X, R, plan, use_graph=True, precond="jacobi", rtol=1e-28,
                                       max_iter=300, check_every=16)
        xh = host(X)
        its = [i["iters"] for i in infos]
        if ref_x is None:
            ref_x, ref_it = xh, its
        else:
            assert_same_values(xh, ref_x, "schedule %s" % (got,))
            assert its == ref_it
    for bad in ((3, 1, 0), (16, 1, 0), (1, 3, 0), (1, 1, 2)):
        with pytest.raises(mp.MpError):
            mp.mp_batch_plan_set_schedule(plan, *bad)


def test_batched_rejects_off_block_entries(mp):
    rp, ci, a, sp = batched_diffusion([4, 4], sigma=1.0, seed=43)
    bad = ci.copy()
    bad[3] = sp[1] + 2   # row 0 of system 0 pointing into system 1
    A = mp.Csr.from_numpy(rp, bad)
    with pytest.raises(mp.MpError):
        mp.mp_batch_plan_create(A, sp, 2, 1)
