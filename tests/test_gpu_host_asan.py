"""Host code of the HIP library under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (GPU).

`tests/host_asan_build.py` (run by `__graft_entry__.build()`) compiles the library's
sources with the host half of every translation unit instrumented and links them with
`tests/host_asan_driver.cpp`, which calls every C-ABI entry point on small inputs (plan
kinds, SpMV variants, argument and workspace checks, transpose, COO -> CSR, the DD and
K-component solvers, refinement, the batched layer, the network, the allocation-free
SpMV) and checks status codes and exact identities.  The run must end with "ok" and no
sanitizer report.  Allocations made inside the HIP and HSA runtimes that live until exit
are suppressed for the leak check (stacks through libamdhip64 or libhsa-runtime64); the
library's own host allocations are checked.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2412_17510_amd", "_build", "asan", "host_asan_driver")


def test_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(EXE):
        pytest.skip("sanitizer driver not built (python tests/host_asan_build.py)")
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libhsa-runtime64.so\nleak:libamdhip64.so\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    env["LSAN_OPTIONS"] = "suppressions=%s" % supp
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert "runtime error" not in out, "UndefinedBehaviorSanitizer report"
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, "AddressSanitizer / LeakSanitizer report"
    assert r.returncode == 0, "driver exit status %d" % r.returncode
    assert r.stdout.strip().splitlines()[-1] == "ok"
