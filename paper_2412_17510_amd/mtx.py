"""Matrix Market coordinate files: read into COO, write from COO, load as a device CSR.

The paper's test matrices come from the SuiteSparse collection, which ships them in
this format, and Sec. 3 stores a matrix in COO and converts it to CSR.  Reading and
writing are host I/O; the COO -> CSR conversion of `load_csr` runs on the GPU
(C ABI mp_coo_to_csr).

Supported: `%%MatrixMarket matrix coordinate {real|integer|complex|pattern}
{general|symmetric|skew-symmetric|hermitian}`.  Symmetric storage is expanded on
reading: every stored off-diagonal entry (i, j, v) adds (j, i, v) (skew: -v,
hermitian: conj(v)).  Coordinates are 1-based in the file and 0-based in memory.

Values.  By default each value is parsed to the nearest binary64 and becomes the
leading component of a K-component value with zero tails.  With exact=True the
decimal text is read as an exact rational and split into K binary64 components by
successive rounding (c0 = fl(v), c1 = fl(v - c0), ...), so a value that binary64 cannot
hold (0.1) is carried to K-component precision.  `write_mtx` writes one-component
values with the shortest round-trip decimal and K-component values as the exact
decimal of their sum, so exact reading recovers them.
"""
from fractions import Fraction

import numpy as np

FIELDS = ("real", "integer", "complex", "pattern")
SYMMETRIES = ("general", "symmetric", "skew-symmetric", "hermitian")


class MtxError(ValueError):
    pass


def _split(value, K):
    """K binary64 components of an exact rational by successive rounding."""
    out = np.zeros(K)
    rest = Fraction(value)
    for c in range(K):
        out[c] = float(rest)
        rest -= Fraction(out[c])
    return out


def _parse_header(line):
    parts = line.strip().split()
    if len(parts) != 5 or parts[0].lower() != "%%matrixmarket" or parts[1].lower() != "matrix":
        raise MtxError("not a Matrix Market matrix header: %r" % line.strip())
    fmt, field, sym = (p.lower() for p in parts[2:])
    if fmt != "coordinate":
        raise MtxError("only the coordinate format is supported (got %r)" % fmt)
    if field not in FIELDS:
        raise MtxError("unknown field %r" % field)
    if sym not in SYMMETRIES:
        raise MtxError("unknown symmetry %r" % sym)
    if field == "pattern" and sym in ("skew-symmetric", "hermitian"):
        raise MtxError("a pattern matrix cannot be %s" % sym)
    if sym == "hermitian" and field != "complex":
        raise MtxError("a hermitian matrix must be complex")
    return field, sym


def read_mtx(path, K=1, exact=False):
    """Read a coordinate Matrix Market file.

    Returns a dict with n_rows, n_cols, row, col (int32, 0-based, file order, with the
    mirrored entries of symmetric storage appended after the stored ones), re and im
    ((K, nnz) float64 component arrays; im is None unless the field is complex; a
    pattern matrix has value 1), field and symmetry."""
    with open(path, "r") as f:
        header = f.readline()
        field, sym = _parse_header(header)
        line = f.readline()
        while line and (line.startswith("%") or not line.strip()):
            line = f.readline()
        if not line:
            raise MtxError("missing size line")
        try:
            n_rows, n_cols, nnz = (int(t) for t in line.split())
        except ValueError:
            raise MtxError("bad size line: %r" % line.strip()) from None
        if n_rows < 0 or n_cols < 0 or nnz < 0:
            raise MtxError("negative size")
        if sym != "general" and n_rows != n_cols:
            raise MtxError("%s storage needs a square matrix" % sym)
        ncol = {"pattern": 2, "real": 3, "integer": 3, "complex": 4}[field]
        toks = [ln.split() for ln in f if ln.strip() and not ln.startswith("%")]
    if len(toks) != nnz:
        raise MtxError("expected %d entries, found %d" % (nnz, len(toks)))
    if any(len(t) != ncol for t in toks):
        raise MtxError("every entry of a %s matrix has %d fields" % (field, ncol))
    row = np.array([int(t[0]) for t in toks], dtype=np.int64) - 1
    col = np.array([int(t[1]) for t in toks], dtype=np.int64) - 1
    if nnz and (row.min() < 0 or row.max() >= n_rows or col.min() < 0 or col.max() >= n_cols):
        raise MtxError("coordinate outside the %d x %d matrix" % (n_rows, n_cols))

    def values(idx):
        if field == "pattern":
            v = np.zeros((K, nnz))
            v[0] = 1.0
            return v
        if exact:
            v = np.zeros((K, nnz))
            for k, t in enumerate(toks):
                v[:, k] = _split(Fraction(t[idx]), K)
            return v
        v = np.zeros((K, nnz))
        v[0] = np.array([float(t[idx]) for t in toks])
        return v

    re = values(2)
    im = values(3) if field == "complex" else None
    if sym != "general":
        off = row != col
        if sym == "skew-symmetric" and np.any(~off):
            raise MtxError("a skew-symmetric matrix stores no diagonal entries")
        mrow, mcol = col[off], row[off]
        mre = re[:, off] * (-1.0 if sym == "skew-symmetric" else 1.0)
        row = np.concatenate([row, mrow])
        col = np.concatenate([col, mcol])
        re = np.concatenate([re, mre], axis=1)
        if im is not None:
            sign = -1.0 if sym in ("skew-symmetric", "hermitian") else 1.0
            im = np.concatenate([im, im[:, off] * sign], axis=1)
    return {"n_rows": n_rows, "n_cols": n_cols, "row": row.astype(np.int32), "col": col.astype(np.int32),
            "re": re, "im": im, "field": field, "symmetry": sym}


def _exact_decimal(x):
    """Exact decimal text of a dyadic rational."""
    x = Fraction(x)
    if x == 0:
        return "0"
    sign = "-" if x < 0 else ""
    x = abs(x)
    num, den = x.numerator, x.denominator
    e = den.bit_length() - 1          # den = 2^e
    digits = str(num * 5 ** e)
    if e == 0:
        return sign + digits
    digits = digits.rjust(e + 1, "0")
    return sign + digits[:-e] + "." + digits[-e:].rstrip("0")


def _fmt(comps):
    comps = np.atleast_1d(comps)
    if comps.size == 1 or not np.any(comps[1:]):
        return repr(float(comps[0]))
    return _exact_decimal(sum((Fraction(float(c)) for c in comps), Fraction(0)))


def write_mtx(path, n_rows, n_cols, row, col, re=None, im=None, comment=None):
    """Write a general coordinate file (1-based).  re / im: (K, nnz) or (nnz,) values;
    re None writes a pattern matrix, im given writes a complex one."""
    row = np.asarray(row)
    col = np.asarray(col)
    nnz = row.size
    field = "pattern" if re is None else ("complex" if im is not None else "real")
    re2 = None if re is None else np.asarray(re, dtype=np.float64).reshape(-1, nnz)
    im2 = None if im is None else np.asarray(im, dtype=np.float64).reshape(-1, nnz)
    with open(path, "w") as f:
        f.write("%%%%MatrixMarket matrix coordinate %s general\n" % field)
        if comment:
            for ln in str(comment).splitlines():
                f.write("%% %s\n" % ln)
        f.write("%d %d %d\n" % (n_rows, n_cols, nnz))
        for k in range(nnz):
            parts = ["%d %d" % (row[k] + 1, col[k] + 1)]
            if re2 is not None:
                parts.append(_fmt(re2[:, k]))
            if im2 is not None:
                parts.append(_fmt(im2[:, k]))
            f.write(" ".join(parts) + "\n")


def load_csr(path, K=2, exact=False, stream=None):
    """Read a Matrix Market file and convert it to CSR on the GPU.  Returns
    (Csr, a_re, a_im or None) with (K, nnz) CUDA float64 values (row order, then
    column; equal coordinates kept in file order)."""
    import torch
    from . import _binding as mp
    m = read_mtx(path, K=K, exact=exact)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    return mp.mp_coo_to_csr(m["n_rows"], m["n_cols"], dev(m["row"]), dev(m["col"]), dev(m["re"]),
                            None if m["im"] is None else dev(m["im"]), stream=stream)
