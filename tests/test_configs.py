"""The configuration table (workloads/configs.json) against what its generators build:
sizes of every configuration, and the draws bench.py and the tests take from it."""
import numpy as np

from workloads import configs, diffusion3d_7pt, laplace2d_5pt, mp_from_leads, powerlaw_pattern, random_mp


def test_c0_sizes_and_draws():
    e = configs.load("c0")
    rp, ci, a, x = configs.c0(K=2)
    assert rp.size - 1 == e["n"] and ci.size == e["nnz"] and a.shape == (2, e["nnz"]) and x.shape == (2, e["n"])
    rp2, ci2, a2 = laplace2d_5pt(100, K=2, seed=0)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2) and np.array_equal(a, a2)


def test_c1_sizes_and_draws():
    e = configs.load("c1")
    rp, ci = configs.c1_pattern()
    assert rp.size - 1 == e["n"] and ci.size == e["nnz"]
    assert np.diff(rp).max() <= e["max_row"]
    # the variant operands are the per-variant streams [value_seed, K, complex]
    rp_s, ci_s = configs.c1_pattern(n=5000)
    rp_r, ci_r = powerlaw_pattern(n=5000, seed=e["seed"])
    assert np.array_equal(rp_s, rp_r) and np.array_equal(ci_s, ci_r)
    nnz, n = ci_s.size, rp_s.size - 1
    for K, cplx in ((2, False), (3, True)):
        rng = np.random.default_rng([e["value_seed"], K, int(cplx)])
        want = [mp_from_leads(rng.uniform(-1, 1, nnz), K, rng),
                mp_from_leads(rng.uniform(-1, 1, nnz), K, rng) if cplx else None,
                random_mp(n, K, rng), random_mp(n, K, rng) if cplx else None]
        got = configs.c1_operands(K, cplx, nnz, n)
        for g, w in zip(got, want):
            assert (g is None and w is None) or np.array_equal(g, w)


def test_c2_sizes():
    e = configs.load("c2")
    rp, ci, _ = diffusion3d_7pt(m=e["m"], sigma=2.5, az=0.01, seed=e["seed"])
    assert rp.size - 1 == e["n"] and ci.size == e["nnz"]


def test_c3_sizes():
    e = configs.load("c3")
    edges = configs.c3_edges().astype(np.int64)
    assert edges.size == e["systems"] and edges.min() >= e["edge_lo"] and edges.max() <= e["edge_hi"]
    # a 7-point grid of edge m has m^3 rows and 7 m^3 - 6 m^2 entries
    assert int((edges ** 3).sum()) == e["n"]
    assert int((7 * edges ** 3 - 6 * edges ** 2).sum()) == e["nnz"]
    rp, ci, a, sp = configs.c3_systems(0.01, systems=3)
    assert sp.size == 4 and sp[-1] == rp.size - 1 == int((edges[:3] ** 3).sum())
    assert configs.c3_rhs(10).shape == (2, 10, e["nrhs"])


def test_c4_law():
    e = configs.load("c4")
    assert e["train_edge_lo"] <= e["train_edge_hi"] and e["train_sigma_lo"] < e["train_sigma_hi"]
    assert e["eval_systems"] == 200 and e["eval_m"] == 64
