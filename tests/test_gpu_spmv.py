"""GPU parity of the multi-component CSR SpMV (C ABI) with the CPU oracle.

Bar: bitwise equality of every component (+0 == -0, no NaN) when the GPU plan's
lane widths (the summation order, exported with mp_plan_row_log2w) are given to the
oracle.  Cases: the 2D 5-point workload (n = 10,000, 49,600 nnz), ragged random
matrices spanning several tiles and every lane width 1..1024, the paper's 5x5
example, empty rows / empty matrices / a single 5,000-element row, every plan kind
(plan-free kernel, canonical plan, width policies, row groups, explicit orders, autotuned), run
to run determinism, argument errors, concurrent calls that share one plan on two
streams, and the full n = 1e6 power-law workload compared on every row.
"""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import configs
from workloads import (laplace2d_5pt, random_csr, random_mp, sqrt2_vector, csr_from_dense,
                       paper_example_5x5, mp_from_leads)

pytestmark = pytest.mark.gpu

VARIANTS = [(2, False), (3, False), (4, False), (2, True), (3, True), (4, True)]
# tile sizes (elements staged in LDS per workgroup) each variant supports
TILES = {(2, False): (256, 512, 1024, 2048), (3, False): (256, 512, 1024), (4, False): (256, 512, 1024),
         (2, True): (256, 512), (3, True): (256, 512), (4, True): (256,)}


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2412_17510_amd import mp as binding
    return binding


def run_gpu(mp, K, cplx, A, a_re, x_re, a_im=None, x_im=None, plan=None):
    import torch
    n = A.n_rows
    y_re = torch.full((K, n), float("nan"), dtype=torch.float64, device="cuda")
    if not cplx:
        mp.SPMV[(K, False)](A, dev(a_re), dev(x_re), y_re, plan=plan)
        torch.cuda.synchronize()
        return host(y_re), None
    y_im = torch.full((K, n), float("nan"), dtype=torch.float64, device="cuda")
    mp.SPMV[(K, True)](A, dev(a_re), dev(a_im), dev(x_re), dev(x_im), y_re, y_im, plan=plan)
    torch.cuda.synchronize()
    return host(y_re), host(y_im)


def check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im=None, x_im=None, plan=None, A=None, what=""):
    if A is None:
        A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=x_re.shape[1])
    y_re, y_im = run_gpu(mp, K, cplx, A, a_re, x_re, a_im, x_im, plan)
    lw = None if plan is None else plan.row_log2w()
    want = ref.spmv(K, row_ptr, col_idx, a_re, x_re, a_im=a_im, x_im=x_im, log2w=lw)
    if cplx:
        assert_same_values(y_re, want[0], what + " re")
        assert_same_values(y_im, want[1], what + " im")
    else:
        assert_same_values(y_re, want, what)
    return y_re, y_im


def test_laplace2d_dd_all_plans(mp):
    row_ptr, col_idx, a = laplace2d_5pt(100, K=2, seed=0)
    rng = np.random.default_rng(0)
    x = random_mp(10000, 2, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    mp.mp_csr_validate(A)
    check(mp, 2, False, row_ptr, col_idx, a, x, A=A, what="plan-free")
    canon = mp.mp_plan_create(A, 2)
    assert np.array_equal(canon.row_log2w(), ref.canonical_log2w(np.diff(row_ptr)))
    y1, _ = check(mp, 2, False, row_ptr, col_idx, a, x, plan=canon, A=A, what="canonical plan")
    y0, _ = run_gpu(mp, 2, False, A, a, x)
    assert_same_values(y0, y1, "plan-free vs canonical plan")
    for shift, mx in ((0, 1), (2, 6), (1, 0)):
        check(mp, 2, False, row_ptr, col_idx, a, x, plan=mp.mp_plan_create(A, 2, False, shift, mx), A=A,
              what="policy %d,%d" % (shift, mx))
        check(mp, 2, False, row_ptr, col_idx, a, x, plan=mp.mp_plan_create(A, 2, False, shift, mx, 0, 1), A=A,
              what="row groups %d,%d" % (shift, mx))
    for tile in (256, 512, 1024, 2048):
        check(mp, 2, False, row_ptr, col_idx, a, x, plan=mp.mp_plan_create(A, 2, False, 0, 6, tile), A=A,
              what="tile %d" % tile)


@pytest.mark.parametrize("K,cplx", VARIANTS)
def test_ragged_random_every_width(mp, K, cplx):
    rng = np.random.default_rng(1000 + 10 * K + cplx)
    # every length class: empty, short, around wavefront and tile sizes, long
    # (7, 8, 15, 16, 17: the plan-free kernel's boundary between rows on eight-lane groups and
    # rows on the whole wavefront)
    lengths = np.concatenate([[0, 1, 2, 3, 5, 7, 8, 15, 16, 17, 63, 64, 65, 127, 128, 255, 256, 511, 512, 1023, 1024,
                               2049, 0],
                              rng.integers(0, 40, 700), rng.integers(40, 300, 60)])
    n_cols = 3000
    row_ptr, col_idx, a_re, a_im = random_csr(lengths.size, n_cols, lengths, K, rng, cplx)
    x_re = random_mp(n_cols, K, rng)
    x_im = random_mp(n_cols, K, rng) if cplx else None
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, A=A, what="plan-free")
    for tile in TILES[(K, cplx)]:
        check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, plan=mp.mp_plan_create(A, K, cplx, tile_nnz=tile),
              A=A, what="canonical tile %d" % tile)
    check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, plan=mp.mp_plan_create(A, K, cplx, 2, 4), A=A,
          what="policy 2,4")
    check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, plan=mp.mp_plan_create(A, K, cplx, 0, 8), A=A,
          what="policy 0,8")
    # row groups (rows with W <= 64 and at most 16 elements per lane; the rest LONG or wide)
    for rg in (1, 2):
        for shift, mx in ((0, 6), (2, 6), (2, 4), (1, 3), (0, 0), (0, 10)):
            plan = mp.mp_plan_create(A, K, cplx, shift, mx, 0, row_groups=rg)
            check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, plan=plan, A=A,
                  what="row groups %d: %d,%d" % (rg, shift, mx))
    # explicit random orders, including every wide (multi-wavefront) width
    fl = np.array([0 if L == 0 else int(np.floor(np.log2(L))) for L in lengths])
    lw = np.array([rng.integers(0, min(10, f) + 1) for f in fl], dtype=np.uint8)
    lw[lengths >= 1024] = 10
    lw[(lengths >= 512) & (lengths < 1024)] = 9
    lw[(lengths >= 256) & (lengths < 512)] = 8
    lw[(lengths >= 128) & (lengths < 256)] = 7
    for tile in TILES[(K, cplx)]:
        check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im,
              plan=mp.mp_plan_create_explicit(A, K, cplx, lw, tile), A=A, what="explicit wide tile %d" % tile)
    lw2 = np.array([rng.integers(0, min(10, f) + 1) for f in fl], dtype=np.uint8)
    check(mp, K, cplx, row_ptr, col_idx, a_re, x_re, a_im, x_im, plan=mp.mp_plan_create_explicit(A, K, cplx, lw2),
          A=A, what="explicit random")


@pytest.mark.parametrize("K", [2, 3, 4])
def test_paper_5x5_example(mp, K):
    row_ptr, col_idx, vals = csr_from_dense(paper_example_5x5())
    a = np.zeros((K, vals.size))
    a[0] = vals
    v = sqrt2_vector(5, K)
    check(mp, K, False, row_ptr, col_idx, a, v, what="5x5 plan-free")
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    check(mp, K, False, row_ptr, col_idx, a, v, plan=mp.mp_plan_create(A, K), A=A, what="5x5 canonical")


@pytest.mark.parametrize("K,cplx", [(2, False), (4, True)])
def test_edge_cases(mp, K, cplx):
    import torch
    rng = np.random.default_rng(7)
    # all rows empty
    row_ptr = np.zeros(9, dtype=np.int32)
    col_idx = np.zeros(0, dtype=np.int32)
    a = np.zeros((K, 0))
    x = random_mp(4, K, rng)
    xi = random_mp(4, K, rng) if cplx else None
    check(mp, K, cplx, row_ptr, col_idx, a, x, a if cplx else None, xi, what="all empty")
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=4)
    check(mp, K, cplx, row_ptr, col_idx, a, x, a if cplx else None, xi, plan=mp.mp_plan_create(A, K, cplx), A=A,
          what="all empty, plan")
    check(mp, K, cplx, row_ptr, col_idx, a, x, a if cplx else None, xi,
          plan=mp.mp_plan_create(A, K, cplx, row_groups=1), A=A, what="all empty, row groups")
    # no rows at all
    A0 = mp.Csr.from_numpy(np.zeros(1, dtype=np.int32), col_idx, n_cols=4)
    y0 = torch.zeros((K, 0), dtype=torch.float64, device="cuda")
    if cplx:
        mp.SPMV[(K, True)](A0, dev(a), dev(a), dev(x), dev(xi), y0, y0.clone())
    else:
        mp.SPMV[(K, False)](A0, dev(a), dev(x), y0)
    torch.cuda.synchronize()
    # one long row and a 1-element row
    lengths = np.array([5000, 1])
    row_ptr, col_idx, a_re, a_im = random_csr(2, 6000, lengths, K, rng, cplx)
    x = random_mp(6000, K, rng)
    xi = random_mp(6000, K, rng) if cplx else None
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=6000)
    for plan in (None, mp.mp_plan_create(A, K, cplx), mp.mp_plan_create(A, K, cplx, 0, 10),
                 mp.mp_plan_create(A, K, cplx, 0, 8), mp.mp_plan_create(A, K, cplx, 3, 4),
                 mp.mp_plan_create_explicit(A, K, cplx, np.array([10, 0], dtype=np.uint8)),
                 mp.mp_plan_create_explicit(A, K, cplx, np.array([9, 0], dtype=np.uint8)),
                 mp.mp_plan_create(A, K, cplx, 0, 6, 0, 1), mp.mp_plan_create(A, K, cplx, 0, 10, 0, 1),
                 mp.mp_plan_create(A, K, cplx, 7, 6, 0, 1), mp.mp_plan_create(A, K, cplx, 0, 6, 0, 2),
                 mp.mp_plan_create(A, K, cplx, 0, 10, 0, 2)):
        check(mp, K, cplx, row_ptr, col_idx, a_re, x, a_im, xi, plan=plan, A=A, what="long row")


def test_zero_tail_inputs_take_general_renorm_path(mp):
    """Integer-valued inputs give exact zero errors inside the QD renormalisation (the
    select-based path); results must still match the oracle and be exact."""
    rng = np.random.default_rng(9)
    lengths = rng.integers(0, 90, 300)
    row_ptr, col_idx, _, _ = random_csr(300, 500, lengths, 4, rng)
    for K in (3, 4):
        a = np.zeros((K, col_idx.size))
        a[0] = rng.integers(-2 ** 20, 2 ** 20, col_idx.size)
        x = np.zeros((K, 500))
        x[0] = rng.integers(-2 ** 20, 2 ** 20, 500)
        y, _ = check(mp, K, False, row_ptr, col_idx, a, x, what="integers K=%d" % K)
        assert np.all(y[1:] == 0)


def test_determinism_and_errors(mp):
    import torch
    rng = np.random.default_rng(3)
    lengths = rng.integers(0, 200, 2000)
    row_ptr, col_idx, a, _ = random_csr(2000, 2500, lengths, 2, rng)
    x = random_mp(2500, 2, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=2500)
    plan = mp.mp_plan_create(A, 2, False, 1, 5)
    ad, xd = dev(a), dev(x)
    y = torch.empty((2, 2000), dtype=torch.float64, device="cuda")
    mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan)
    first = host(y).copy()
    for _ in range(10):
        y.fill_(float("nan"))
        mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan)
        assert np.array_equal(host(y), first)
    # aliasing: y is x (square 5x5 example)
    rp5, ci5, v5 = csr_from_dense(paper_example_5x5())
    A5 = mp.Csr.from_numpy(rp5, ci5)
    a5 = np.zeros((2, v5.size))
    a5[0] = v5
    x5 = dev(random_mp(5, 2, rng))
    with pytest.raises(mp.MpError) as ei:
        mp.mpspmv_csr_dd(A5, dev(a5), x5, x5)
    assert ei.value.status == -2
    # a plan built for another pattern is rejected
    with pytest.raises(mp.MpError):
        mp.mpspmv_csr_dd(A5, dev(a5), x5, torch.empty((2, 5), dtype=torch.float64, device="cuda"), plan=plan)
    # malformed patterns are reported by validate
    bad_cols = col_idx.copy()
    bad_cols[5] = 2500
    with pytest.raises(mp.MpError):
        mp.mp_csr_validate(mp.Csr.from_numpy(row_ptr, bad_cols, n_cols=2500))
    bad_rp = row_ptr.copy()
    bad_rp[10] = bad_rp[11] + 1
    with pytest.raises(mp.MpError):
        mp.mp_csr_validate(mp.Csr.from_numpy(bad_rp, col_idx, n_cols=2500))
    with pytest.raises(mp.MpError):
        mp.mp_plan_create(mp.Csr.from_numpy(bad_rp, col_idx, n_cols=2500), 2)
    with pytest.raises(mp.MpError):
        mp.mp_plan_create_explicit(A, 2, False, np.full(2000, 10, dtype=np.uint8))
    # a plan made for another variant is rejected
    with pytest.raises(mp.MpError):
        mp.mpspmv_csr_qd(A, dev(np.zeros((4, a.shape[1]))), dev(np.zeros((4, 2500))),
                         torch.empty((4, 2000), dtype=torch.float64, device="cuda"), plan=plan)
    # tile sizes beyond the variant's LDS budget are refused
    with pytest.raises(mp.MpError) as ei:
        mp.mp_plan_create(A, 4, True, tile_nnz=2048)
    assert ei.value.status == -7


# ---------------------------------------------------------------------------------------
# full-size power-law workload (n = 1e6, mean 27 nnz/row), sampled rows
# ---------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def powerlaw():
    row_ptr, col_idx = configs.c1_pattern()
    return row_ptr, col_idx


@pytest.mark.parametrize("K,cplx", VARIANTS)
def test_powerlaw_full_size(mp, powerlaw, K, cplx):
    """Every one of the 1e6 rows, under the autotuned plan (the launch configuration the
    benchmark times) and the plan-free kernel."""
    import torch
    row_ptr, col_idx = powerlaw
    n = row_ptr.size - 1
    nnz = col_idx.size
    rng = np.random.default_rng([5, K, int(cplx)])
    a_re = mp_from_leads(rng.uniform(-1, 1, nnz), K, rng)
    a_im = mp_from_leads(rng.uniform(-1, 1, nnz), K, rng) if cplx else None
    x_re = random_mp(n, K, rng)
    x_im = random_mp(n, K, rng) if cplx else None
    A = mp.Csr.from_numpy(row_ptr, col_idx)
    ad_re, xd_re = dev(a_re), dev(x_re)
    ad_im = dev(a_im) if cplx else None
    xd_im = dev(x_im) if cplx else None
    y_re = torch.empty((K, n), dtype=torch.float64, device="cuda")
    y_im = torch.empty((K, n), dtype=torch.float64, device="cuda") if cplx else None
    args = (ad_re, ad_im, xd_re, xd_im, y_re, y_im) if cplx else (ad_re, xd_re, y_re)
    plan, pol = mp.mp_plan_autotune(A, K, ad_re, xd_re, y_re, ad_im, xd_im, y_im, reps=2)
    ws = mp.spmv_workspace(plan)
    # the autotuned plan, the other plan kind under the same order, and the plan-free kernel
    others = [mp.mp_plan_create(A, K, cplx, pol["shift"], pol["max_log2w"], pol["tile_nnz"], rg)
              for rg in (0, 1, 2) if rg != pol["row_groups"]]
    for p in (plan, *others, None):
        if cplx:
            y_im.fill_(float("nan"))
        y_re.fill_(float("nan"))
        mp.SPMV[(K, cplx)](A, *args, plan=p, ws=ws if p is plan else None)
        torch.cuda.synchronize()
        lw = None if p is None else p.row_log2w()
        want = ref.spmv(K, row_ptr, col_idx, a_re, x_re, a_im=a_im, x_im=x_im, log2w=lw)
        if cplx:
            assert_same_values(host(y_re), want[0], "powerlaw re %s" % (pol,))
            assert_same_values(host(y_im), want[1], "powerlaw im %s" % (pol,))
        else:
            assert_same_values(host(y_re), want, "powerlaw %s" % (pol,))
    assert plan.info()["tile_nnz"] == pol["tile_nnz"]


@pytest.mark.parametrize("K,cplx", [(2, False), (3, True)])
def test_shared_plan_concurrent_streams(mp, K, cplx):
    """A plan is read-only: two SpMVs that share it, each with its own workspace, run
    concurrently on two streams (different x, different y) and both equal the oracle
    bit for bit; repeated with the calls interleaved many times."""
    import torch
    rng = np.random.default_rng([11, K, int(cplx)])
    n_cols = 60000
    lengths = np.concatenate([rng.integers(0, 60, 40000), rng.integers(200, 3000, 40)])
    row_ptr, col_idx, a_re, a_im = random_csr(lengths.size, n_cols, lengths, K, rng, cplx)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    plan = mp.mp_plan_create(A, K, cplx, 1, 6)
    xs = [(random_mp(n_cols, K, rng), random_mp(n_cols, K, rng) if cplx else None) for _ in range(2)]
    wants = [ref.spmv(K, row_ptr, col_idx, a_re, xr, a_im=a_im, x_im=xi, log2w=plan.row_log2w()) for xr, xi in xs]
    ad_re = dev(a_re)
    ad_im = dev(a_im) if cplx else None
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    ins, outs, wss = [], [], []
    for j, st in enumerate(streams):
        with torch.cuda.stream(st):
            xr, xi = xs[j]
            ins.append((dev(xr), dev(xi) if cplx else None))
            outs.append((torch.empty((K, A.n_rows), dtype=torch.float64, device="cuda"),
                         torch.empty((K, A.n_rows), dtype=torch.float64, device="cuda") if cplx else None))
            wss.append(mp.spmv_workspace(plan, st))
    torch.cuda.synchronize()
    for _ in range(20):
        for j, st in enumerate(streams):
            (xr, xi), (yr, yi) = ins[j], outs[j]
            if cplx:
                mp.SPMV[(K, True)](A, ad_re, ad_im, xr, xi, yr, yi, plan=plan, stream=st, ws=wss[j])
            else:
                mp.SPMV[(K, False)](A, ad_re, xr, yr, plan=plan, stream=st, ws=wss[j])
    torch.cuda.synchronize()
    for j in range(2):
        yr, yi = outs[j]
        if cplx:
            assert_same_values(host(yr), wants[j][0], "stream %d re" % j)
            assert_same_values(host(yi), wants[j][1], "stream %d im" % j)
        else:
            assert_same_values(host(yr), wants[j], "stream %d" % j)


def test_workspace_errors(mp):
    """A planned SpMV refuses a workspace that is too small, misaligned or overlapping an
    operand; the plan-free call needs none."""
    import torch
    rng = np.random.default_rng(12)
    lengths = rng.integers(1, 50, 3000)
    row_ptr, col_idx, a, _ = random_csr(3000, 3000, lengths, 2, rng)
    x = random_mp(3000, 2, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=3000)
    plan = mp.mp_plan_create(A, 2)
    need = mp.mpspmv_workspace_bytes(plan)
    assert need == 16 * 3000 and mp.mpspmv_workspace_bytes(None) == 0
    ad, xd = dev(a), dev(x)
    y = torch.empty((2, 3000), dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError) as ei:
        mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan, ws=torch.empty(need // 8 - 1, dtype=torch.float64, device="cuda"))
    assert ei.value.status == -4
    big = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpError) as ei:
        mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan, ws=big[1:])
    assert ei.value.status == -1
    with pytest.raises(mp.MpError) as ei:
        mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan, ws=y.view(-1))
    assert ei.value.status == -2
    mp.mpspmv_csr_dd(A, ad, xd, y, plan=plan, ws=big)
    torch.cuda.synchronize()
    assert_same_values(host(y), ref.spmv(2, row_ptr, col_idx, a, x, log2w=plan.row_log2w()), "workspace")
