"""Builds the CPU oracle (``libmpref.so``) from ``mpref.c`` and ``exact_resid.c`` with gcc.

TEST INFRASTRUCTURE ONLY: the oracle is loaded by the tests, the smoke check and
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpref.c")
SOURCES = [SRC, os.path.join(HERE, "exact_resid.c")]
LIB = os.path.join(HERE, "libmpref.so")

# No contraction, no fast-math: each + and * is one IEEE binary64 operation.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra"]


def build(force=True):
    """Compile the oracle; with force=False only when the library is missing or stale."""
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(s) for s in SOURCES):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, *SOURCES, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
