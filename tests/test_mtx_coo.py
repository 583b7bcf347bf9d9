"""COO -> CSR and Matrix Market I/O (CPU only).

* The oracle's COO -> CSR reproduces the CSR arrays the paper prints for its 5x5
  example (Sec. 3) from the COO arrays it prints; on shuffled random COO input it orders
  by row then column, keeps equal coordinates in input order, equals scipy's conversion
  when coordinates are unique, and converting (col, row) equals the stable transpose of
  the CSR of (row, col).  Coordinates outside the matrix are rejected.
* read_mtx / write_mtx: the 5x5 example round-trips through a file; symmetric,
  skew-symmetric and hermitian storage expand to the full matrix; pattern and integer
  fields; exact reading carries 0.1 to DD precision and recovers written DD values bit
  for bit; malformed files are rejected.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref
from paper_2412_17510_amd import mtx
from workloads import mp_from_leads

scipy_sparse = pytest.importorskip("scipy.sparse")


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "csr_5x5.json")) as f:
        return json.load(f)


def test_paper_5x5_coo_to_csr(golden_dir):
    g = _golden(golden_dir)
    rp, ci, a = ref.coo_to_csr(5, 5, g["coo_row"], g["coo_col"], np.array(g["coo_data"], float))
    assert rp.tolist() == g["csr_indptr"] and ci.tolist() == g["csr_indices"] and a.tolist() == g["csr_data"]
    # the same from a shuffled COO listing
    perm = np.random.default_rng(1).permutation(8)
    rp2, ci2, a2 = ref.coo_to_csr(5, 5, np.array(g["coo_row"])[perm], np.array(g["coo_col"])[perm],
                                  np.array(g["coo_data"], float)[perm])
    assert np.array_equal(rp2, rp) and np.array_equal(ci2, ci) and np.array_equal(a2, a)


@pytest.mark.parametrize("shape", [(300, 300), (120, 500), (500, 80)])
def test_random_coo_order_duplicates_and_transpose(shape):
    n, m = shape
    rng = np.random.default_rng(n * 7 + m)
    nnz = 3000
    row = rng.integers(0, n, nnz).astype(np.int32)
    col = rng.integers(0, m, nnz).astype(np.int32)
    dup = rng.choice(nnz, 200, replace=False)
    row[dup[100:]], col[dup[100:]] = row[dup[:100]], col[dup[:100]]   # planted duplicates
    v = rng.standard_normal((2, nnz))
    v[0, dup[100:]] = np.arange(100) + 1000.0                          # tags to check their order
    rp, ci, a = ref.coo_to_csr(n, m, row, col, v)
    assert rp[0] == 0 and rp[-1] == nnz and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = rows.astype(np.int64) * m + ci
    assert np.all(np.diff(key) >= 0)
    # stability: among equal coordinates the input order is kept
    order = np.lexsort((np.arange(nnz), col, row))
    assert np.array_equal(a, v[:, order]) and np.array_equal(ci, col[order])
    # unique coordinates: scipy's conversion
    keep = np.unique(row.astype(np.int64) * m + col, return_index=True)[1]
    rp_u, ci_u, a_u = ref.coo_to_csr(n, m, row[keep], col[keep], v[0, keep])
    S = scipy_sparse.coo_matrix((v[0, keep], (row[keep], col[keep])), shape=(n, m)).tocsr()
    S.sort_indices()
    assert np.array_equal(rp_u, S.indptr) and np.array_equal(ci_u, S.indices) and np.array_equal(a_u, S.data)
    # CSR of (col, row) = stable transpose of the CSR of (row, col)
    rpt, cit, at = ref.transpose(rp, ci, a, n_cols=m)
    rq, cq, aq = ref.coo_to_csr(m, n, col, row, v)
    assert np.array_equal(rq, rpt) and np.array_equal(cq, cit) and np.array_equal(aq, at)


def test_coo_rejects_outside_coordinates():
    with pytest.raises(ValueError):
        ref.coo_to_csr(4, 4, [0, 4], [0, 1], np.ones(2))
    with pytest.raises(ValueError):
        ref.coo_to_csr(4, 4, [0, 1], [0, -1], np.ones(2))
    rp, ci, a = ref.coo_to_csr(3, 3, np.zeros(0), np.zeros(0), np.zeros(0))
    assert rp.tolist() == [0, 0, 0, 0] and ci.size == 0


def test_mtx_round_trip_5x5(tmp_path, golden_dir):
    g = _golden(golden_dir)
    p = tmp_path / "a.mtx"
    mtx.write_mtx(p, 5, 5, g["coo_row"], g["coo_col"], np.array(g["coo_data"], float), comment="Eq. 1")
    text = p.read_text().splitlines()
    assert text[0] == "%%MatrixMarket matrix coordinate real general" and text[2] == "5 5 8"
    assert text[3] == "1 1 1.0" and text[6] == "2 5 -4.0"      # 1-based on file
    m = mtx.read_mtx(p, K=2)
    assert m["row"].tolist() == g["coo_row"] and m["col"].tolist() == g["coo_col"]
    assert m["re"][0].tolist() == g["coo_data"] and not m["re"][1].any() and m["im"] is None


def _dense(m):
    D = np.zeros((m["n_rows"], m["n_cols"]), dtype=complex)
    for k in range(m["row"].size):
        D[m["row"][k], m["col"][k]] += m["re"][0, k] + (1j * m["im"][0, k] if m["im"] is not None else 0)
    return D


def test_mtx_symmetric_storage(tmp_path):
    cases = {
        "real symmetric": ("%%MatrixMarket matrix coordinate real symmetric\n3 3 4\n1 1 2\n2 1 -1\n3 2 -1\n3 3 2\n",
                           np.array([[2, -1, 0], [-1, 0, -1], [0, -1, 2]])),
        "real skew-symmetric": ("%%MatrixMarket matrix coordinate real skew-symmetric\n3 3 2\n2 1 4\n3 1 -5\n",
                                np.array([[0, -4, 5], [4, 0, 0], [-5, 0, 0]])),
        "complex hermitian": ("%%MatrixMarket matrix coordinate complex hermitian\n2 2 3\n1 1 1 0\n2 1 2 3\n2 2 4 0\n",
                              np.array([[1, 2 - 3j], [2 + 3j, 4]])),
        "pattern symmetric": ("%%MatrixMarket matrix coordinate pattern symmetric\n%c\n3 3 2\n2 1\n3 3\n",
                              np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])),
        "integer general": ("%%MatrixMarket matrix coordinate integer general\n2 3 2\n1 3 7\n2 1 -2\n",
                            np.array([[0, 0, 7], [-2, 0, 0]])),
    }
    for name, (text, want) in cases.items():
        p = tmp_path / (name.replace(" ", "_") + ".mtx")
        p.write_text(text)
        m = mtx.read_mtx(p)
        assert np.array_equal(_dense(m), want), name


def test_mtx_exact_values(tmp_path):
    p = tmp_path / "e.mtx"
    p.write_text("%%MatrixMarket matrix coordinate real general\n1 3 3\n1 1 0.1\n1 2 0.5\n1 3 -1e-310\n")
    m = mtx.read_mtx(p, K=2, exact=True)
    tenth = Fraction(m["re"][0, 0]) + Fraction(m["re"][1, 0])
    assert abs(tenth - Fraction(1, 10)) <= Fraction(1, 10) * Fraction(1, 2 ** 105)
    assert m["re"][:, 1].tolist() == [0.5, 0.0]
    # written K-component values come back bit for bit through the exact decimal text
    rng = np.random.default_rng(3)
    vals = mp_from_leads(rng.uniform(-1, 1, 20), 2, rng)   # normalized DD values
    q = tmp_path / "dd.mtx"
    mtx.write_mtx(q, 4, 5, np.arange(20) // 5, np.arange(20) % 5, vals)
    back = mtx.read_mtx(q, K=2, exact=True)
    assert np.array_equal(back["re"], vals)


def test_mtx_rejects_malformed(tmp_path):
    bad = {
        "header": "%%MatrixMarket matrix array real general\n2 2\n1\n2\n3\n4\n",
        "count": "%%MatrixMarket matrix coordinate real general\n2 2 3\n1 1 1\n2 2 1\n",
        "range": "%%MatrixMarket matrix coordinate real general\n2 2 1\n3 1 1\n",
        "fields": "%%MatrixMarket matrix coordinate complex general\n2 2 1\n1 1 1\n",
        "skew diagonal": "%%MatrixMarket matrix coordinate real skew-symmetric\n2 2 1\n1 1 1\n",
    }
    for name, text in bad.items():
        p = tmp_path / ("bad_%s.mtx" % name.replace(" ", "_"))
        p.write_text(text)
        with pytest.raises(mtx.MtxError):
            mtx.read_mtx(p)
