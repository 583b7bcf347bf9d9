"""MI355X-native multi-component-precision (DD/TD/QD) sparse kernels and solvers.

The computation lives in the gfx950 HIP library ``libmpsparse.so`` (C ABI in
``include/mpsparse.h``); this package is its Python binding.  Import the binding
with ``from paper_2412_17510_amd import mp`` -- it raises ImportError when the
library has not been built (there is no fallback path).
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libmpsparse.so")


def __getattr__(name):
    if name == "mp":
        from . import _binding
        return _binding
    raise AttributeError(name)
