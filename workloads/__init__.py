"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and by the CPU oracle.

This package only draws inputs (sparsity patterns, values, vectors).  It holds none
of the sparse-product or solver arithmetic.
"""
from .gen import (  # noqa: F401
    mp_from_leads, is_nonoverlapping, sqrt2_vector, sqrt_2p3i_vector,
    laplace2d_5pt, powerlaw_pattern, powerlaw_csr, random_csr, random_mp,
    diffusion3d_7pt, powerlaw_xmin, csr_from_dense, paper_example_5x5, banded_nonsymmetric,
    batched_diffusion,
)
