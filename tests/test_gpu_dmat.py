"""GPU parity of the binary64-matrix SpMV (C ABI mpspmv_csr_{dd,td,qd}_d and _d_complex) with the
oracle: bitwise equality of every component under the plan's exported order, on
ragged random matrices spanning several tiles and every lane width 1..1024 (plan-free
kernel, canonical plans of every tile size, width policies, explicit orders), the
paper's 5x5 example, and every row of the full n = 1e6 power-law workload; for DD
the result equals the DD SpMV of the zero-tail matrix on the GPU too; argument
checks."""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import configs
from workloads import (random_csr, random_mp, sqrt2_vector, csr_from_dense, paper_example_5x5)

pytestmark = pytest.mark.gpu

TILES = {2: (256, 512, 1024, 2048), 3: (256, 512, 1024), 4: (256, 512, 1024)}


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def run(mp, K, A, a, x, plan=None):
    import torch
    y = torch.full((K, A.n_rows), float("nan"), dtype=torch.float64, device="cuda")
    mp.SPMV_D[K](A, dev(a), dev(x), y, plan=plan)
    torch.cuda.synchronize()
    return host(y)


def check(mp, K, row_ptr, col_idx, a, x, A, plan=None, what=""):
    got = run(mp, K, A, a, x, plan)
    lw = None if plan is None else plan.row_log2w()
    assert_same_values(got, ref.spmv_dmat(K, row_ptr, col_idx, a, x, log2w=lw), what)
    return got


@pytest.mark.parametrize("K", [2, 3, 4])
def test_ragged_random_every_width(mp, K):
    rng = np.random.default_rng(2000 + K)
    lengths = np.concatenate([[0, 1, 2, 3, 5, 63, 64, 65, 127, 128, 255, 256, 511, 512, 1023, 1024, 2049, 0],
                              rng.integers(0, 40, 700), rng.integers(40, 300, 60)])
    n_cols = 3000
    row_ptr, col_idx, _, _ = random_csr(lengths.size, n_cols, lengths, K, rng)
    a = rng.uniform(-1, 1, col_idx.size) * 2.0 ** rng.integers(-20, 20, col_idx.size)
    x = random_mp(n_cols, K, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    check(mp, K, row_ptr, col_idx, a, x, A, what="plan-free")
    for tile in TILES[K]:
        check(mp, K, row_ptr, col_idx, a, x, A, plan=mp.mp_plan_create(A, K, False, tile_nnz=tile),
              what="canonical tile %d" % tile)
    for sh, mx in ((2, 4), (0, 8), (2, 8)):
        check(mp, K, row_ptr, col_idx, a, x, A, plan=mp.mp_plan_create(A, K, False, sh, mx), what="policy")
    fl = np.array([0 if L == 0 else int(np.floor(np.log2(L))) for L in lengths])
    lw = np.array([rng.integers(0, min(10, f) + 1) for f in fl], dtype=np.uint8)
    lw[lengths >= 1024] = 10
    lw[(lengths >= 512) & (lengths < 1024)] = 9
    for tile in TILES[K]:
        check(mp, K, row_ptr, col_idx, a, x, A, plan=mp.mp_plan_create_explicit(A, K, False, lw, tile),
              what="explicit wide tile %d" % tile)
    if K == 2:
        # equal to the DD SpMV of the same matrix with zero trailing components
        import torch
        padded = np.zeros((2, a.size))
        padded[0] = a
        plan = mp.mp_plan_create(A, 2, False, 2, 8)
        yd = torch.empty((2, A.n_rows), dtype=torch.float64, device="cuda")
        mp.mpspmv_csr_dd(A, dev(padded), dev(x), yd, plan=plan)
        assert_same_values(run(mp, 2, A, a, x, plan), host(yd), "dmat vs zero-tail DD")


@pytest.mark.parametrize("K", [2, 3, 4])
def test_paper_5x5(mp, K):
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    v = sqrt2_vector(5, K)
    check(mp, K, row_ptr, col_idx, vals, v, A, what="5x5 plan-free")
    check(mp, K, row_ptr, col_idx, vals, v, A, plan=mp.mp_plan_create(A, K), what="5x5 canonical")


@pytest.mark.parametrize("K", [2, 3, 4])
def test_powerlaw_full_size(mp, K):
    """Every one of the 1e6 rows, under an autotuned-style plan and the plan-free kernel."""
    import torch
    row_ptr, col_idx = configs.c1_pattern()
    n = row_ptr.size - 1
    rng = np.random.default_rng([7, K])
    a = rng.uniform(-1, 1, col_idx.size)
    x = random_mp(n, K, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    y = torch.empty((K, n), dtype=torch.float64, device="cuda")
    ad, xd = dev(a), dev(x)
    for plan in (mp.mp_plan_create(A, K, False, 2, 8, 512), None):
        y.fill_(float("nan"))
        mp.SPMV_D[K](A, ad, xd, y, plan=plan)
        torch.cuda.synchronize()
        want = ref.spmv_dmat(K, row_ptr, col_idx, a, x, log2w=None if plan is None else plan.row_log2w())
        assert_same_values(host(y), want, "powerlaw dmat K=%d plan %s" % (K, plan is not None))


def test_argument_checks(mp):
    import torch
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    x = dev(sqrt2_vector(5, 2))
    y = torch.empty((2, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        mp.mpspmv_csr_dd_d(A, dev(np.zeros((2, vals.size))), x, y)
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError):   # y overlapping a
        mp.mpspmv_csr_dd_d(A, buf[:8], x, buf[6:16].view(2, 5))


# ---------------------------------------------------------------------------
# complex: binary64 complex matrix times a K-component complex vector
# ---------------------------------------------------------------------------

TILES_C = {2: (256, 512), 3: (256, 512), 4: (256,)}


def run_c(mp, K, A, a_re, a_im, x_re, x_im, plan=None):
    import torch
    y_re = torch.full((K, A.n_rows), float("nan"), dtype=torch.float64, device="cuda")
    y_im = torch.full((K, A.n_rows), float("nan"), dtype=torch.float64, device="cuda")
    mp.SPMV_D_COMPLEX[K](A, dev(a_re), dev(a_im), dev(x_re), dev(x_im), y_re, y_im, plan=plan)
    torch.cuda.synchronize()
    return host(y_re), host(y_im)


def check_c(mp, K, row_ptr, col_idx, a_re, a_im, x_re, x_im, A, plan=None, what=""):
    gr, gi = run_c(mp, K, A, a_re, a_im, x_re, x_im, plan)
    lw = None if plan is None else plan.row_log2w()
    wr, wi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im, log2w=lw)
    assert_same_values(gr, wr, what + " re")
    assert_same_values(gi, wi, what + " im")
    return gr, gi


@pytest.mark.parametrize("K", [2, 3, 4])
def test_complex_ragged_random_every_width(mp, K):
    rng = np.random.default_rng(2100 + K)
    lengths = np.concatenate([[0, 1, 2, 3, 5, 63, 64, 65, 127, 128, 255, 256, 511, 512, 1023, 1024, 2049, 0],
                              rng.integers(0, 40, 500), rng.integers(40, 300, 40)])
    n_cols = 3000
    row_ptr, col_idx, _, _ = random_csr(lengths.size, n_cols, lengths, K, rng)
    a_re = rng.uniform(-1, 1, col_idx.size) * 2.0 ** rng.integers(-20, 20, col_idx.size)
    a_im = rng.uniform(-1, 1, col_idx.size)
    x_re = random_mp(n_cols, K, rng)
    x_im = random_mp(n_cols, K, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    args = (mp, K, row_ptr, col_idx, a_re, a_im, x_re, x_im, A)
    check_c(*args, what="plan-free")
    for tile in TILES_C[K]:
        check_c(*args, plan=mp.mp_plan_create(A, K, True, tile_nnz=tile), what="canonical tile %d" % tile)
    for sh, mx in ((2, 4), (0, 8), (2, 8)):
        check_c(*args, plan=mp.mp_plan_create(A, K, True, sh, mx), what="policy")
    fl = np.array([0 if L == 0 else int(np.floor(np.log2(L))) for L in lengths])
    lw = np.array([rng.integers(0, min(10, f) + 1) for f in fl], dtype=np.uint8)
    lw[lengths >= 1024] = 10
    lw[(lengths >= 512) & (lengths < 1024)] = 9
    for tile in TILES_C[K]:
        check_c(*args, plan=mp.mp_plan_create_explicit(A, K, True, lw, tile), what="explicit wide tile %d" % tile)
    # a_im = x_im = 0: the real binary64-matrix product and a zero imaginary part
    z = np.zeros_like(a_im)
    plan = mp.mp_plan_create(A, K, True, 2, 8)
    gr, gi = run_c(mp, K, A, a_re, z, x_re, np.zeros_like(x_im), plan)
    assert np.all(gi == 0)
    plan_r = mp.mp_plan_create_explicit(A, K, False, plan.row_log2w())
    assert_same_values(gr, run(mp, K, A, a_re, x_re, plan_r), "complex with zero imaginary parts vs real")


@pytest.mark.parametrize("K", [2, 3, 4])
def test_complex_powerlaw_full_size(mp, K):
    """Every one of the 1e6 rows of the binary64 complex matrix product."""
    import torch
    row_ptr, col_idx = configs.c1_pattern()
    n = row_ptr.size - 1
    rng = np.random.default_rng([8, K])
    a_re = rng.uniform(-1, 1, col_idx.size)
    a_im = rng.uniform(-1, 1, col_idx.size)
    x_re = random_mp(n, K, rng)
    x_im = random_mp(n, K, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    y_re = torch.empty((K, n), dtype=torch.float64, device="cuda")
    y_im = torch.empty((K, n), dtype=torch.float64, device="cuda")
    plan = mp.mp_plan_create(A, K, True, 2, 8, 256)
    mp.SPMV_D_COMPLEX[K](A, dev(a_re), dev(a_im), dev(x_re), dev(x_im), y_re, y_im, plan=plan)
    torch.cuda.synchronize()
    wr, wi = ref.spmv_dmat_complex(K, row_ptr, col_idx, a_re, a_im, x_re, x_im, log2w=plan.row_log2w())
    assert_same_values(host(y_re), wr, "powerlaw complex dmat re K=%d" % K)
    assert_same_values(host(y_im), wi, "powerlaw complex dmat im K=%d" % K)


def test_complex_argument_checks(mp):
    import torch
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    x = dev(sqrt2_vector(5, 2))
    y = torch.empty((2, 5), dtype=torch.float64, device="cuda")
    yi = torch.empty((2, 5), dtype=torch.float64, device="cuda")
    a = dev(vals)
    with pytest.raises(ValueError):   # a K-component matrix where binary64 values are expected
        mp.mpspmv_csr_dd_d_complex(A, dev(np.zeros((2, vals.size))), a, x, x, y, yi)
    with pytest.raises(mp.MpError):   # y_re overlapping y_im
        buf = torch.zeros(20, dtype=torch.float64, device="cuda")
        mp.mpspmv_csr_dd_d_complex(A, a, a, x, x, buf[:10].view(2, 5), buf[5:15].view(2, 5))
    with pytest.raises(mp.MpError):   # a real plan for the complex product
        mp.mpspmv_csr_dd_d_complex(A, a, a, x, x, y, yi, plan=mp.mp_plan_create(A, 2, False))
