"""Builds the host-sanitizer check of the HIP library (test infrastructure).

The library's sources are compiled again with the host half of every translation unit
under AddressSanitizer and UndefinedBehaviorSanitizer (device code as in the library
build), and linked with `tests/host_asan_driver.cpp` into one executable,
`paper_2412_17510_amd/_build/asan/host_asan_driver`, which `tests/test_gpu_host_asan.py`
runs on a GPU.  `__graft_entry__.build()` calls build().
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
from paper_2412_17510_amd import build as lib_build  # noqa: E402

OUT = os.path.join(lib_build.BUILD, "asan")
EXE = os.path.join(OUT, "host_asan_driver")
DRIVER = os.path.join(HERE, "host_asan_driver.cpp")
# each sanitizer flag applies to the host compilation only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _compile(src):
    obj = os.path.join(OUT, os.path.splitext(os.path.basename(src))[0] + ".o")
    flags = [f for f in lib_build.FLAGS if f != "-fPIC"]
    cmd = [lib_build.HIPCC, *flags, *SAN, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build():
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(lib_build.CSRC, s) for s in lib_build.SOURCES] + [DRIVER]
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [lib_build.HIPCC, "--offload-arch=" + lib_build.ARCH, *SAN, *objs, "-o", EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    return EXE


if __name__ == "__main__":
    print(build())
