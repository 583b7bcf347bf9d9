"""Host logic of bench.py (no GPU): the roofline classification and arithmetic, the
measured-ceiling fields attached to each variant, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_and_ops():
    n, nnz = 1000, 27000
    # CSR row pointers, int32 columns, K components of each value, x read and y written once
    assert bench.algo_bytes(n, nnz, 2, False) == 4 * (n + 1) + nnz * (4 + 16) + 2 * 16 * n
    assert bench.algo_bytes(n, nnz, 4, True) == 4 * (n + 1) + nnz * (4 + 64) + 2 * 64 * n
    assert bench.algo_bytes(n, nnz, 3, False, dmat=True) == 4 * (n + 1) + nnz * 12 + 2 * 24 * n
    assert bench.ops_per_nnz(2, False) == 20
    assert bench.ops_per_nnz(4, True) == 4 * (118 + 82)
    assert bench.ops_per_nnz(3, False, dmat=True) == 66 + 82
    # complex with a binary64 matrix: two binary64 values per element, four mixed products
    assert bench.algo_bytes(n, nnz, 4, True, dmat=True) == 4 * (n + 1) + nnz * (4 + 16) + 2 * 64 * n
    assert bench.ops_per_nnz(4, True, dmat=True) == 4 * (66 + 82)


def test_roofline_picks_the_binding_resource():
    n, nnz = 1_000_000, 26_865_804
    dd = bench.roofline(n, nnz, 2, False, 0.25)
    assert dd["bound"] == "hbm" and dd["unit"] == "GB/s" and dd["peak"] == 8000.0
    assert dd["achieved"] == pytest.approx(bench.algo_bytes(n, nnz, 2, False) / 0.25e-3 / 1e9, rel=1e-3)
    assert dd["frac"] == pytest.approx(dd["achieved"] / 8000.0, rel=1e-3)
    qdc = bench.roofline(n, nnz, 4, True, 2.3)
    assert qdc["bound"] == "alu" and qdc["peak"] == pytest.approx(39.32, rel=1e-3)
    assert qdc["achieved"] == pytest.approx(800 * nnz / 2.3e-3 / 1e12, rel=1e-2)


class _FakeMp:
    """Stands in for the binding: fixed measured rates."""
    RATES = {0: 32e12, 2: 1.6e12, 3: 1.9e11, 4: 1.9e11}

    def mp_measure_rate(self, kind):
        return self.RATES[kind]


def test_measured_ceilings_fields():
    results = {"dd": {"gnnz_s": 100.0}, "dd_d": {"gnnz_s": 120.0}, "td": {"gnnz_s": 63.0},
               "qd_complex": {"gnnz_s": 11.4}}
    out = bench.measured_ceilings(_FakeMp(), results)
    assert out["fp64_fma_lane_instr_per_s"] == pytest.approx(32e12)
    assert out["fp64_fma_frac_of_spec"] == pytest.approx(32e12 / bench.FP64_INSTR_PEAK, rel=1e-3)
    assert results["dd"]["arith_ceiling_gnnz_s"] == pytest.approx(1600.0)
    assert results["td"]["frac_of_arith_ceiling"] == pytest.approx(63.0 / 190.0, rel=1e-3)
    # complex: four multiply-add steps per element
    assert results["qd_complex"]["arith_ceiling_gnnz_s"] == pytest.approx(190.0 / 4, rel=1e-3)
    # binary64-matrix variants carry no step ceiling (their product is a different operation)
    assert "arith_ceiling_gnnz_s" not in results["dd_d"]


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""
