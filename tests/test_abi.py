"""The C-ABI library builds for gfx950, loads, and exports every entry point the header
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpsparse.h")
LIB = os.path.join(ROOT, "paper_2412_17510_amd", "libmpsparse.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mp_status|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2412_17510_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_spmv_entry_points():
    names = declared_functions()
    for n in ("mpspmv_csr_dd", "mpspmv_csr_td", "mpspmv_csr_qd", "mpspmv_csr_dd_complex",
              "mpspmv_csr_td_complex", "mpspmv_csr_qd_complex", "mp_last_error", "mpkrylov_cg",
              "mpkrylov_bicgstab", "mpkrylov_ir", "mpkrylov_ir_learned", "mpspmm_csr_dd_batched",
              "mpkrylov_cg_batched", "mp_mpnn_forward", "mp_mpnn_loss_grad", "mp_mpnn_adam_step"):
        assert n in names


def test_every_declared_symbol_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_library_is_gfx950(lib):
    """The embedded device code object targets gfx950 (target id string in our own build)."""
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_version_and_error_calls_are_host_only(lib):
    lib.mp_version.restype = ctypes.c_char_p
    lib.mp_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mp_version()
    assert isinstance(lib.mp_last_error(), bytes)


def test_null_arguments_rejected_without_gpu(lib):
    """O(1) host checks fire before any HIP call."""
    lib.mpspmv_csr_dd.restype = ctypes.c_int
    lib.mp_last_error.restype = ctypes.c_char_p
    assert lib.mpspmv_csr_dd(None, None, None, None, None, None, ctypes.c_size_t(0), None) == -1
    assert b"NULL" in lib.mp_last_error()
    nb = ctypes.c_size_t(123)
    assert lib.mpspmv_workspace_bytes(None, ctypes.byref(nb)) == 0 and nb.value == 0
    assert lib.mpspmv_workspace_bytes(None, None) == -1
    assert lib.mpvec_dd_sub(ctypes.c_int64(-1), None, None, None, None) == -1
    assert lib.mpvec_dd_sub(ctypes.c_int64(0), None, None, None, None) == 0
    assert lib.mpvec_dd_sub(ctypes.c_int64(4), None, None, None, None) == -1


def test_learned_entry_points_host_checks(lib):
    """Parameter count agrees with the oracle network; NULL / unsupported arguments fail
    before any HIP call."""
    from oracle import mpnn
    lib.mp_last_error.restype = ctypes.c_char_p
    c = ctypes.c_int32()
    assert lib.mp_mpnn_param_count(ctypes.byref(c)) == 0 and c.value == mpnn.n_params()
    h = ctypes.c_void_p()
    assert lib.mp_mpnn_create(32, ctypes.byref(h)) == -7 and not h.value
    assert lib.mp_mpnn_create(64, None) == -1
    assert lib.mpkrylov_ir_learned(None, None, None, None, None, None, None, None, ctypes.c_size_t(0), None,
                                   None) == -1
    assert lib.mp_graph_create(None, None, None, ctypes.byref(h)) == -1
    d = ctypes.c_double()
    assert lib.mp_measure_rate(1, ctypes.byref(d), None) == -1
    assert lib.mp_measure_rate(5, ctypes.byref(d), None) == -1
    assert lib.mp_measure_rate(0, None, None) == -1


def test_traffic_record_is_usable_by_the_bench():
    """Each committed counter record carries what bench.py matches before it reports the
    traffic figure: the kernel-source hash, the plan and the matrix size, and a
    positive copy-calibrated byte count per call; one record per plan, all taken on the
    same kernel sources."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "spmv_dd_powerlaw_traffic.json")
    with open(path) as f:
        recs = json.load(f)["records"]
    assert recs
    plans = [json.dumps(r["plan"], sort_keys=True) for r in recs]
    assert len(set(plans)) == len(plans)
    for rec in recs:
        for key in ("source_hash", "plan", "n", "nnz", "traffic_bytes", "commands"):
            assert key in rec, key
        assert set(rec["plan"]) == {"shift", "max_log2w", "tile_nnz", "row_groups"} and rec["n"] == 1_000_000
        assert rec["traffic_bytes"] > 0 and len(rec["source_hash"]) == 16
        assert rec["source_hash"] == recs[0]["source_hash"]
        # read bytes are the counted requests at their sizes, scaled by a plain copy
        for k in rec["kernels"].values():
            q = k["read_requests"]
            assert k["read_bytes"] == 32 * q["32B"] + 64 * q["64B"] + 128 * q["128B"]


def test_traffic_records_merge_and_match(tmp_path):
    """The per-plan merge keeps one record per plan, drops records of other kernel
    sources, and the bench's lookup matches plan, size and source hash exactly."""
    from paper_2412_17510_amd.profiling import find_record, merge_record
    import json
    p = str(tmp_path / "t.json")
    pa = {"shift": 2, "max_log2w": 6, "tile_nnz": 512}
    pb = {"shift": 2, "max_log2w": 8, "tile_nnz": 512}

    def write(recs):
        with open(p, "w") as f:
            json.dump({"records": recs}, f)

    write(merge_record(p, {"plan": pa, "n": 10, "source_hash": "h1", "traffic_bytes": 1}))
    write(merge_record(p, {"plan": pb, "n": 10, "source_hash": "h1", "traffic_bytes": 2}))
    r3 = {"plan": pa, "n": 10, "source_hash": "h1", "traffic_bytes": 3}
    recs = merge_record(p, r3)
    assert [r["traffic_bytes"] for r in recs] == [3, 2]
    write(recs)
    assert find_record(p, pa, 10, "h1")["traffic_bytes"] == 3
    assert find_record(p, pb, 10, "h1")["traffic_bytes"] == 2
    assert find_record(p, pa, 11, "h1") is None
    assert find_record(p, pa, 10, "h2") is None
    assert find_record(p, {"shift": 0, "max_log2w": 6, "tile_nnz": 512}, 10, "h1") is None
    r4 = {"plan": pb, "n": 10, "source_hash": "h2", "traffic_bytes": 4}
    assert [r["traffic_bytes"] for r in merge_record(p, r4)] == [4]
    assert find_record(str(tmp_path / "missing.json"), pa, 10, "h1") is None
