"""The allocation-free DD SpMV (C ABI mpspmv_csr_dd_noalloc) against the workspace
entry point mpspmv_csr_dd and the oracle: bitwise equal on two calls in a row, the
second with a smaller matrix, and the size limit of its fixed staging array."""
import numpy as np
import pytest

from oracle import ref
from tests.helpers import assert_same_values, dev, host
from workloads import random_csr, random_mp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available()
    from paper_2412_17510_amd import mp as binding
    return binding


def one_case(mp, rng, n_rows, n_cols, max_len, plan_opts):
    import torch
    print("noalloc case n_rows=%d n_cols=%d plan=%s" % (n_rows, n_cols, plan_opts), flush=True)
    lengths = np.concatenate([rng.integers(0, max_len, n_rows - 3), [0, min(1500, n_cols), min(3000, n_cols)]])
    row_ptr, col_idx, a, _ = random_csr(n_rows, n_cols, lengths, 2, rng)
    x = random_mp(n_cols, 2, rng)
    A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
    plan = None if plan_opts is None else mp.mp_plan_create(A, 2, False, *plan_opts)
    ad, xd = dev(a), dev(x)
    y_ws = torch.full((2, n_rows), float("nan"), dtype=torch.float64, device="cuda")
    y_na = torch.full((2, n_rows), float("nan"), dtype=torch.float64, device="cuda")
    mp.mpspmv_csr_dd(A, ad, xd, y_ws, plan=plan)
    mp.mpspmv_csr_dd_noalloc(A, ad, xd, y_na, plan=plan)
    torch.cuda.synchronize()
    assert_same_values(host(y_na), host(y_ws), "noalloc vs workspace entry")
    want = ref.spmv(2, row_ptr, col_idx, a, x, log2w=None if plan is None else plan.row_log2w())
    assert_same_values(host(y_na), want, "noalloc vs oracle")


def test_noalloc_matches_workspace_entry_twice(mp):
    rng = np.random.default_rng(31)
    one_case(mp, rng, 200_000, 1_000_000, 60, (1, 6, 1024))
    one_case(mp, rng, 3_000, 5_000, 40, (0, 6, 512))
    one_case(mp, rng, 2_000, 2_500, 30, None)


def test_noalloc_size_limit(mp):
    """Largest staged x it holds: 1,048,576 DD columns; one more is refused before any
    launch with MP_ERR_NO_MEMORY."""
    import torch
    rng = np.random.default_rng(32)
    for n_cols, ok in ((1 << 20, True), ((1 << 20) + 1, False)):
        lengths = rng.integers(1, 20, 1000)
        row_ptr, col_idx, a, _ = random_csr(1000, n_cols, lengths, 2, rng)
        A = mp.Csr.from_numpy(row_ptr, col_idx, n_cols=n_cols)
        plan = mp.mp_plan_create(A, 2)
        x = torch.zeros((2, n_cols), dtype=torch.float64, device="cuda")
        y = torch.empty((2, 1000), dtype=torch.float64, device="cuda")
        if ok:
            mp.mpspmv_csr_dd_noalloc(A, dev(a), x, y, plan=plan)
            torch.cuda.synchronize()
            assert np.all(host(y) == 0)
        else:
            with pytest.raises(mp.MpError) as ei:
                mp.mpspmv_csr_dd_noalloc(A, dev(a), x, y, plan=plan)
            assert ei.value.status == -4 and b"1048576" in mp._lib.mp_last_error()
