"""The benchmark configurations as data (`workloads/configs.json`) and the generators
that build each from its entry.  Draws only: no arithmetic of the method."""
import json
import os

import numpy as np

from .gen import batched_diffusion, laplace2d_5pt, mp_from_leads, powerlaw_pattern, random_mp

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "configs.json")


def load(name=None):
    """The whole table, or the entry of one configuration ("c0" .. "c4")."""
    with open(PATH) as f:
        table = json.load(f)
    return table if name is None else table[name]


def c0(K=2):
    """(row_ptr, col_idx, a (K, nnz), x (K, n)) of the parity case."""
    e = load("c0")
    rp, ci, a = laplace2d_5pt(e["grid"], K=K, seed=e["seed"])
    x = random_mp(rp.size - 1, K, np.random.default_rng(e["x_seed"]))
    return rp, ci, a, x


def c1_pattern(n=None, **overrides):
    """(row_ptr, col_idx) of the power-law matrix (n rows; default the configured n)."""
    e = load("c1")
    kw = dict(n=e["n"] if n is None else n, mean=e["mean_row"], alpha=e["alpha"], maxlen=e["max_row"],
              band=e["band"], p_band=e["p_band"], seed=e["seed"])
    kw.update(overrides)
    return powerlaw_pattern(**kw)


def c1_operands(K, cplx, nnz, n):
    """(a_re, a_im, x_re, x_im) of one variant (a_im, x_im None when real): leads U(-1, 1)
    with K-component tails, drawn from the variant's own stream."""
    rng = np.random.default_rng([load("c1")["value_seed"], K, int(cplx)])
    a_re = mp_from_leads(rng.uniform(-1, 1, nnz), K, rng)
    a_im = mp_from_leads(rng.uniform(-1, 1, nnz), K, rng) if cplx else None
    x_re = random_mp(n, K, rng)
    x_im = random_mp(n, K, rng) if cplx else None
    return a_re, a_im, x_re, x_im


def c3_edges(systems=None):
    """Grid edges of the batched systems (the first `systems` of the configured draw)."""
    e = load("c3")
    return np.random.default_rng(e["edge_seed"]).integers(e["edge_lo"], e["edge_hi"] + 1,
                                                          e["systems"] if systems is None else systems)


def c3_systems(az, systems=None):
    """(row_ptr, col_idx, a (2, nnz), sys_ptr) of the block-diagonal batch."""
    e = load("c3")
    return batched_diffusion(c3_edges(systems), sigma=e["sigma"], seed=e["seed"], az=az)


def c3_rhs(N):
    """The (2, N, nrhs) DD right-hand sides of the batch."""
    e = load("c3")
    R = e["nrhs"]
    return np.ascontiguousarray(random_mp(N * R, 2, np.random.default_rng(e["rhs_seed"])).reshape(2, N, R))
