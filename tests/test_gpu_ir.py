"""GPU parity of mixed-precision iterative refinement (C ABI mpkrylov_ir) with the CPU
oracle: same status, inner-iteration total, refinement steps and fallback flag,
bitwise identical x and DD true residual.  binary64 and binary32 inner solves, a plan
order, a forced stall (fallback to DD CG), and the 64^3 sigma = 2.5 diffusion system to
relative residual 1e-28 (with the solution's distance from the oracle's DD CG answer
reported)."""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import diffusion3d_7pt, random_mp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def compare_ir(mp, row_ptr, col_idx, a, b, plan_opts=None, **kw):
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    plan = None if plan_opts is None else mp.mp_plan_create(A, 2, False, *plan_opts)
    n = row_ptr.size - 1
    x = dev(np.zeros((2, n)))
    ig = mp.mpkrylov_ir(A, dev(a), dev(b), x, plan=plan, check_every=16, **kw)
    xo, io = ref.ir(row_ptr, col_idx, a, b, log2w=None if plan is None else plan.row_log2w(), **kw)
    got = (ig["status"], ig["iters"], ig["outer_iters"], ig["fell_back"])
    assert got == (io["status"], io["iters"], io["outer_iters"], io["fell_back"]), (got, io)
    assert_same_values(host(x), xo, "ir x")
    assert_same_values(ig["rr_true"], io["rr_true"], "ir rr_true")
    return ig, xo


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_ir_parity(mp, inner):
    row_ptr, col_idx, a = diffusion3d_7pt(m=16, sigma=2.0, seed=31)
    b = random_mp(row_ptr.size - 1, 2, np.random.default_rng(31))
    ig, _ = compare_ir(mp, row_ptr, col_idx, a, b, inner=inner, inner_rtol=1e-6, inner_max_iter=3000, rtol=1e-28)
    assert ig["status"] == 0 and ig["relres"] <= 1.01e-28


def test_ir_plan_and_fallback(mp):
    row_ptr, col_idx, a = diffusion3d_7pt(m=12, sigma=2.0, seed=32)
    b = random_mp(row_ptr.size - 1, 2, np.random.default_rng(32))
    compare_ir(mp, row_ptr, col_idx, a, b, plan_opts=(1, 3, 256), inner="fp64", inner_rtol=1e-8,
               inner_max_iter=3000, rtol=1e-28)
    ig, _ = compare_ir(mp, row_ptr, col_idx, a, b, inner="fp64", inner_rtol=1e-12, inner_max_iter=1, rtol=1e-28)
    assert ig["fell_back"] == 1


def test_ir_full_size_64cubed(mp):
    row_ptr, col_idx, a = diffusion3d_7pt(m=64, sigma=2.5, seed=2)
    b = random_mp(row_ptr.size - 1, 2, np.random.default_rng(2))
    ig, xo = compare_ir(mp, row_ptr, col_idx, a, b, inner="fp64", inner_rtol=1e-8, inner_max_iter=20000,
                        max_iter=20000, rtol=1e-28)
    assert ig["status"] == 0
    print("64^3 IR(fp64): outer %d inner %d, %.3f s on the GPU, relres %.3g" % (
        ig["outer_iters"], ig["iters"], ig["seconds"], ig["relres"]))
