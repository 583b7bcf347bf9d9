"""GPU parity of the DD Krylov solvers (C ABI mpkrylov_cg / _bicgstab / _bicg / _cgs / _gpbicg) with the
CPU oracle: same status, iteration count and restarts, bitwise identical x and
identical DD true residual, with and without Jacobi preconditioning and with a
non-canonical plan order.  Cases: SPD 3D diffusion (to 1e-28, and a 100-iteration
run at the full 64^3 size), the non-symmetric tub1000-shaped matrix (iteration
limit), NaN right-hand side (breakdown), warm start, and argument errors."""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import diffusion3d_7pt, banded_nonsymmetric, sqrt2_vector, random_mp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def gpu_solve(mp, kind, row_ptr, col_idx, a, b, x0=None, plan_opts=None, **opts):
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    plan = None if plan_opts is None else mp.mp_plan_create(A, 2, False, *plan_opts)
    n = row_ptr.size - 1
    x = dev(np.zeros((2, n)) if x0 is None else x0)
    fn = mp.mpkrylov_cg if kind == "cg" else mp.mpkrylov_bicgstab
    info = fn(A, dev(a), dev(b), x, plan=plan, **opts)
    return host(x), info, (None if plan is None else plan.row_log2w())


def compare(mp, kind, row_ptr, col_idx, a, b, precond, rtol, max_iter, plan_opts=None, x0=None, what=""):
    xg, ig, lw = gpu_solve(mp, kind, row_ptr, col_idx, a, b, x0=x0, plan_opts=plan_opts, precond=precond,
                           rtol=rtol, max_iter=max_iter, check_every=16)
    solve = ref.cg if kind == "cg" else ref.bicgstab
    xo, io = solve(row_ptr, col_idx, a, b, x0=x0, precond=precond, rtol=rtol, max_iter=max_iter, log2w=lw)
    assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), (what, ig, io)
    assert_same_values(xg, xo, what + " x")
    assert_same_values(ig["rr_true"], io["rr_true"], what + " rr_true")
    assert_same_values(ig["bb"], io["bb"], what + " bb")
    return ig


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_cg_diffusion_converged_parity(mp, precond):
    row_ptr, col_idx, a = diffusion3d_7pt(m=16, sigma=1.0, seed=11)
    n = row_ptr.size - 1
    v = sqrt2_vector(n, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    info = compare(mp, "cg", row_ptr, col_idx, a, b, precond, 1e-28, 5000, what="cg " + precond)
    assert info["status"] == 0 and info["relres"] <= 1.01e-28


@pytest.mark.parametrize("row_groups", [0, 1, 2])
def test_cg_with_plan_order(mp, row_groups):
    """CG under a plan's order, its SpMV in tiles or in row groups (the step stages p for
    either kernel)."""
    row_ptr, col_idx, a = diffusion3d_7pt(m=12, sigma=1.5, seed=12)
    rng = np.random.default_rng(12)
    b = random_mp(row_ptr.size - 1, 2, rng)
    compare(mp, "cg", row_ptr, col_idx, a, b, "jacobi", 1e-28, 5000, plan_opts=(1, 2, 256, row_groups),
            what="cg plan, row groups %d" % row_groups)


def test_cg_full_size_100_iterations(mp):
    row_ptr, col_idx, a = diffusion3d_7pt(m=64, sigma=2.5, seed=2)
    rng = np.random.default_rng(2)
    b = random_mp(row_ptr.size - 1, 2, rng)
    info = compare(mp, "cg", row_ptr, col_idx, a, b, "jacobi", 1e-28, 100, what="cg 64^3")
    assert info["status"] == -5 and info["iters"] == 100


@pytest.mark.parametrize("which", [0, 1])
def test_cg_64cubed_converged_parity(mp, which):
    """The benchmark's 64^3 solver systems (the calibrated law: sigma 2.5 at the
    anisotropy of largest condition number, and the sigma of condition number 1e10),
    solved to 1e-28 by Jacobi DD CG under the plan the benchmark autotunes for them: the
    GPU's whole solve equals the oracle's (status, iterations, restarts, every component
    of x, the DD true residual), and the exact residual certifies 1e-28."""
    import torch
    from workloads.condition import load_law
    law = load_law()["systems"][which]
    print("64^3 system %s sigma %g az %g" % (law["name"], law["sigma"], law["az"]), flush=True)
    row_ptr, col_idx, a = diffusion3d_7pt(m=law["m"], sigma=law["sigma"], az=law["az"], seed=law["seed"])
    n = row_ptr.size - 1
    b = random_mp(n, 2, np.random.default_rng(law["seed"]))
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    ad, bd = dev(a), dev(b)
    plan, _ = mp.mp_plan_autotune(A, 2, ad, bd, torch.empty((2, n), dtype=torch.float64, device="cuda"), reps=3)
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    ig = mp.mpkrylov_cg(A, ad, bd, x, plan=plan, precond="jacobi", rtol=1e-28, max_iter=100000, check_every=32)
    xo, io = ref.cg(row_ptr, col_idx, a, b, precond="jacobi", rtol=1e-28, max_iter=100000, log2w=plan.row_log2w())
    assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"])
    assert_same_values(host(x), xo, "64^3 x")
    assert_same_values(ig["rr_true"], io["rr_true"], "64^3 rr_true")
    assert ig["status"] == 0
    assert ref.exact_residual(row_ptr, col_idx, a, b, xo)["relres_upper"] <= 1e-28


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_bicgstab_parity(mp, precond):
    row_ptr, col_idx, a = banded_nonsymmetric(n=1000, seed=3)
    v = sqrt2_vector(1000, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    info = compare(mp, "bicgstab", row_ptr, col_idx, a, b, precond, 1e-28, 400, what="bicgstab " + precond)
    assert info["iters"] == 400
    # a well-conditioned system converges fully
    row_ptr, col_idx, a = banded_nonsymmetric(n=3000, seed=4, lower=-1.3, upper=-0.5, upper2=0.05)
    v = sqrt2_vector(3000, 2)
    b = ref.spmv(2, row_ptr, col_idx, a, v)
    info = compare(mp, "bicgstab", row_ptr, col_idx, a, b, precond, 1e-28, 5000, what="bicgstab conv")
    assert info["status"] == 0


def test_bicgstab_on_spd_with_plan(mp):
    row_ptr, col_idx, a = diffusion3d_7pt(m=10, sigma=1.0, seed=13)
    rng = np.random.default_rng(13)
    b = random_mp(row_ptr.size - 1, 2, rng)
    compare(mp, "bicgstab", row_ptr, col_idx, a, b, "jacobi", 1e-26, 3000, plan_opts=(0, 6, 512), what="bicg spd")


def test_breakdown_warm_start_and_errors(mp):
    import torch
    row_ptr, col_idx, a = diffusion3d_7pt(m=6, sigma=1.0, seed=6)
    n = row_ptr.size - 1
    rng = np.random.default_rng(7)
    b = random_mp(n, 2, rng)
    bad = b.copy()
    bad[0, 5] = np.nan
    for kind in ("cg", "bicgstab"):
        xg, ig, _ = gpu_solve(mp, kind, row_ptr, col_idx, a, bad, precond="jacobi", rtol=1e-28, max_iter=50)
        assert ig["status"] == -6
    xs, info = ref.cg(row_ptr, col_idx, a, b, rtol=1e-20, max_iter=5000)
    compare(mp, "cg", row_ptr, col_idx, a, b, "jacobi", 1e-20, 5000, x0=xs, what="warm start")
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    ad, bd = dev(a), dev(b)
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(mp.MpError) as ei:
        mp.mpkrylov_cg(A, ad, bd, x, ws=small)
    assert ei.value.status == -4
    with pytest.raises(mp.MpError) as ei:
        mp.mpkrylov_cg(A, ad, bd, bd)
    assert ei.value.status == -2
    with pytest.raises(mp.MpError):
        qplan = mp.mp_plan_create(A, 4)
        mp.mpkrylov_cg(A, ad, bd, x, plan=qplan)


def test_bicg_matches_oracle_and_cg(mp):
    """GPU BiCG (with the device transpose) equals the oracle's BiCG bit for bit on a
    non-symmetric band and on a symmetric diffusion matrix, where it also equals CG."""
    import torch
    from workloads import banded_nonsymmetric, diffusion3d_7pt
    for name, (row_ptr, col_idx, a) in (("band", banded_nonsymmetric(n=300, seed=5)),
                                        ("diffusion", diffusion3d_7pt(m=7, sigma=1.5, seed=8))):
        n = row_ptr.size - 1
        b = random_mp(n, 2, np.random.default_rng(11))
        A = mp.Csr.from_numpy(row_ptr, col_idx)
        ad, bd = dev(a), dev(b)
        At, at, _ = mp.mp_csr_transpose(A, ad)
        for precond in ("none", "jacobi"):
            for plans in ((None, None), (mp.mp_plan_create(A, 2, False, 2, 6), mp.mp_plan_create(At, 2, False, 1, 4))):
                x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
                ig = mp.mpkrylov_bicg(A, ad, At, at, bd, x, plan=plans[0], plan_t=plans[1], precond=precond,
                                      rtol=1e-28, max_iter=20000, check_every=16)
                lw = None if plans[0] is None else plans[0].row_log2w()
                lwt = None if plans[1] is None else plans[1].row_log2w()
                xo, io = ref.bicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000, log2w=lw,
                                  log2w_t=lwt)
                assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), name
                assert io["status"] == 0
                assert_same_values(host(x), xo, "%s bicg x" % name)
                assert_same_values(ig["rr_true"], io["rr_true"], "%s bicg rr" % name)
                if name == "diffusion" and plans[0] is None:
                    xc = torch.zeros_like(x)
                    ic = mp.mpkrylov_cg(A, ad, bd, xc, precond=precond, rtol=1e-28, max_iter=20000, check_every=16)
                    assert ic["iters"] == ig["iters"]
                    assert_same_values(host(xc), host(x), "bicg = cg on a symmetric matrix")


def test_cgs_matches_oracle(mp):
    """GPU CGS equals the oracle's CGS bit for bit (status, counts, x, residual) on a
    non-symmetric band and a diffusion matrix, with and without plans."""
    import torch
    from workloads import banded_nonsymmetric, diffusion3d_7pt
    for name, (row_ptr, col_idx, a) in (("band", banded_nonsymmetric(n=300, seed=6)),
                                        ("diffusion", diffusion3d_7pt(m=6, sigma=1.0, seed=9))):
        n = row_ptr.size - 1
        b = random_mp(n, 2, np.random.default_rng(12))
        A = mp.Csr.from_numpy(row_ptr, col_idx)
        ad, bd = dev(a), dev(b)
        for precond in ("none", "jacobi"):
            for plan in (None, mp.mp_plan_create(A, 2, False, 2, 6)):
                x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
                ig = mp.mpkrylov_cgs(A, ad, bd, x, plan=plan, precond=precond, rtol=1e-28, max_iter=20000,
                                     check_every=8)
                lw = None if plan is None else plan.row_log2w()
                xo, io = ref.cgs(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000, log2w=lw)
                assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), name
                assert io["status"] == 0
                assert_same_values(host(x), xo, "%s cgs x" % name)
                assert_same_values(ig["rr_true"], io["rr_true"], "%s cgs rr" % name)


def test_gpbicg_matches_oracle(mp):
    """GPU GPBiCG equals the oracle's GPBiCG bit for bit (status, counts, x, residual)
    on a non-symmetric band and a diffusion matrix, with and without plans, and over
    several chunks of 4096 rows (a ragged last chunk)."""
    import torch
    from workloads import banded_nonsymmetric, diffusion3d_7pt
    for name, (row_ptr, col_idx, a) in (("band", banded_nonsymmetric(n=300, seed=6)),
                                        ("diffusion", diffusion3d_7pt(m=6, sigma=1.0, seed=9)),
                                        ("diffusion-chunks", diffusion3d_7pt(m=21, sigma=1.0, seed=10))):
        n = row_ptr.size - 1
        b = random_mp(n, 2, np.random.default_rng(13))
        A = mp.Csr.from_numpy(row_ptr, col_idx)
        ad, bd = dev(a), dev(b)
        for precond in ("none", "jacobi"):
            for plan in (None, mp.mp_plan_create(A, 2, False, 2, 6)):
                if name == "diffusion-chunks" and (precond == "none" or plan is None):
                    continue
                x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
                ig = mp.mpkrylov_gpbicg(A, ad, bd, x, plan=plan, precond=precond, rtol=1e-28, max_iter=20000,
                                        check_every=8)
                lw = None if plan is None else plan.row_log2w()
                xo, io = ref.gpbicg(row_ptr, col_idx, a, b, precond=precond, rtol=1e-28, max_iter=20000, log2w=lw)
                assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]), name
                assert io["status"] == 0
                assert_same_values(host(x), xo, "%s gpbicg x" % name)
                assert_same_values(ig["rr_true"], io["rr_true"], "%s gpbicg rr" % name)


def test_gpbicg_limits_half_step_and_breakdown(mp):
    """Iteration limits (ending inside a check chunk), a half step that meets the
    tolerance (a diagonal system with one distinct eigenvalue converges when t is
    formed), a warm start at the solution, and a NaN right-hand side (breakdown)
    report the oracle's status and counts."""
    import torch
    from workloads import banded_nonsymmetric
    row_ptr, col_idx, a = banded_nonsymmetric(n=300, seed=6)
    n = row_ptr.size - 1
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    ad = dev(a)
    b = random_mp(n, 2, np.random.default_rng(14))
    for lim in (1, 2, 5, 11):
        x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        ig = mp.mpkrylov_gpbicg(A, ad, dev(b), x, rtol=1e-28, max_iter=lim, check_every=4)
        xo, io = ref.gpbicg(row_ptr, col_idx, a, b, rtol=1e-28, max_iter=lim)
        assert io["status"] == -5 and io["iters"] == lim
        assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"])
        assert_same_values(ig["rr_true"], io["rr_true"], "limit %d rr" % lim)
        assert_same_values(host(x), xo, "limit %d x" % lim)
    # one distinct eigenvalue: t = 0 after the first alpha -> half step, then confirmed
    nd = 5000
    rp = np.arange(nd + 1, dtype=np.int32)
    ci = np.arange(nd, dtype=np.int32)
    ad_diag = np.zeros((2, nd))
    ad_diag[0] = 3.0
    bdg = random_mp(nd, 2, np.random.default_rng(15))
    Ad = mp.Csr.from_numpy(rp, ci)
    x = torch.zeros((2, nd), dtype=torch.float64, device="cuda")
    ig = mp.mpkrylov_gpbicg(Ad, dev(ad_diag), dev(bdg), x, precond="none", rtol=1e-28, max_iter=50)
    xo, io = ref.gpbicg(rp, ci, ad_diag, bdg, precond="none", rtol=1e-28, max_iter=50)
    assert (ig["status"], ig["iters"], ig["restarts"]) == (io["status"], io["iters"], io["restarts"]) == (0, 1, 0)
    assert_same_values(host(x), xo, "half step x")
    # warm start at the solution: no step
    xw = x.clone()
    iw = mp.mpkrylov_gpbicg(Ad, dev(ad_diag), dev(bdg), xw, precond="none", rtol=1e-28, max_iter=50)
    assert iw["iters"] == 0 and torch.equal(xw, x)
    bad = b.copy()
    bad[0, 7] = np.nan
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    ig = mp.mpkrylov_gpbicg(A, ad, dev(bad), x, rtol=1e-28, max_iter=50)
    io = ref.gpbicg(row_ptr, col_idx, a, bad, rtol=1e-28, max_iter=50)[1]
    assert ig["status"] == io["status"] == -6 and ig["iters"] == io["iters"]
    with pytest.raises(mp.MpError) as ei:
        mp.mpkrylov_gpbicg(A, ad, dev(bad), x, rtol=1e-28, max_iter=50, raise_on_failure=True)
    assert ei.value.status == -6


def test_dd_sub_keeps_both_components(mp):
    """mpvec_dd_sub equals the oracle's DD addition of x and -y (negation is exact), also
    in place; the result carries the trailing component that a leading-only difference
    would drop."""
    import torch
    rng = np.random.default_rng(21)
    n = 100_003
    x = random_mp(n, 2, rng)
    y = x.copy()
    y[1] = random_mp(n, 2, rng)[1] * 1e-3   # same leading parts, different tails
    y[0, ::7] = random_mp(n, 2, rng)[0, ::7]
    want = ref.elementwise(2, "add", x, -y)
    xd, yd = dev(x), dev(y)
    z = torch.full((2, n), float("nan"), dtype=torch.float64, device="cuda")
    mp.mpvec_dd_sub(xd, yd, z)
    torch.cuda.synchronize()
    assert_same_values(host(z), want, "dd_sub")
    mp.mpvec_dd_sub(xd, yd, xd)
    torch.cuda.synchronize()
    assert_same_values(host(xd), want, "dd_sub in place")
    same_lead = np.ones(n, dtype=bool)
    same_lead[::7] = False
    assert np.all(want[0][same_lead] == x[1][same_lead] - y[1][same_lead])
    buf = torch.zeros(2 * n + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError) as ei:
        mp.mpvec_dd_sub(buf[:2 * n].view(2, n), yd, buf[1:].view(2, n))
    assert ei.value.status == -2
