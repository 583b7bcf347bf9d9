"""Seeded synthetic workloads shaped like the paper's inputs.

The paper measures on SuiteSparse matrices (Sec. 4) that are not available here;
these generators stand in for them with the shapes and value laws of the workload
configurations:

* ``laplace2d_5pt``   -- 2D 5-point operator on a 100x100 grid (n = 10,000,
  nnz = 49,600), diagonal 4+u, off-diagonals -1+0.01u, u ~ U(-1,1).
* ``powerlaw_csr``    -- n = 1e6, power-law row lengths (density ~ L^-2.1, mean 27,
  at most 4,096), each entry banded (|j-i| inside a 2,000-wide window) with
  probability 0.7 and uniform otherwise; values U(-1,1).
* ``diffusion3d_7pt`` -- cell-centred 7-point diffusion on an m^3 grid with
  lognormal cell coefficients (SPD), for the Krylov solvers.
* ``sqrt2_vector`` / ``sqrt_2p3i_vector`` -- the paper's test vectors
  v = sqrt(2)[1..n]^T and v = sqrt(2+3i)[1..n]^T (Sec. 4, Eq. 4), rounded to K
  binary64 components with exact integer arithmetic.

Multi-component values come from ``mp_from_leads``: a leading binary64 value h and
tails c_{k+1} = c_k * 2^-53 * v_k, v_k ~ U(-1,1), re-split without changing the
represented sum so that every component is at most half an ulp of the one above.

Layout (matches the C-ABI): a K-component array of length L is a (K, L) float64
array, component 0 leading.  CSR uses int32 row_ptr / col_idx, 0-based, columns
sorted within a row.

All draws use numpy's PCG64 from ``np.random.default_rng(seed)`` in a fixed order,
so every (function, arguments, seed) triple always yields the same bytes.
"""
from decimal import Decimal, getcontext
from fractions import Fraction
import math

import numpy as np

TWO_M53 = 2.0 ** -53


# --------------------------------------------------------------------------------------
# multi-component values
# --------------------------------------------------------------------------------------

def _resplit(hi, lo):
    """Exact re-split of hi + lo into (nearest binary64, remainder); the pair's sum is unchanged."""
    s = hi + lo
    bv = s - hi
    av = s - bv
    return s, (hi - av) + (lo - bv)


def is_nonoverlapping(comps):
    """True if every component c_{k+1} satisfies fl(c_k + c_{k+1}) == c_k (numpy (K, L) array)."""
    comps = np.asarray(comps)
    for k in range(comps.shape[0] - 1):
        if not np.all(comps[k] + comps[k + 1] == comps[k]):
            return False
    return True


def mp_from_leads(lead, K, rng):
    """(K, L) multi-component array with the given leading values and the tail law above."""
    lead = np.asarray(lead, dtype=np.float64)
    comps = [lead.copy()]
    c = lead
    for _ in range(1, K):
        v = rng.uniform(-1.0, 1.0, size=lead.shape)
        c = c * TWO_M53 * v
        comps.append(c)
    out = np.stack(comps) if K > 1 else lead[None, :].copy()
    # value-preserving sweeps until the components no longer overlap
    for _ in range(4 * K):
        if is_nonoverlapping(out):
            break
        for k in range(K - 1):
            out[k], out[k + 1] = _resplit(out[k], out[k + 1])
    assert is_nonoverlapping(out)
    return out


def random_mp(n, K, rng, low=-1.0, high=1.0):
    """Random K-component vector with U(low, high) leading values."""
    return mp_from_leads(rng.uniform(low, high, size=n), K, rng)


def _round_to_components(value, K):
    """Greedy K-component rounding of an exact (rational) value: c0 = fl(value), c1 = fl(value - c0), ..."""
    out = []
    rem = Fraction(value)
    for _ in range(K):
        c = float(rem)  # correctly rounded
        out.append(c)
        rem -= Fraction(c)
    return out


def sqrt2_vector(n, K, prec_bits=420):
    """v_j = sqrt(2) * j, j = 1..n, rounded to K components (Sec. 4, Eq. 4, real case)."""
    out = np.zeros((K, n))
    scale = 1 << prec_bits
    for j in range(1, n + 1):
        # floor(sqrt(2) j 2^P) / 2^P: within 2^-P of the true value, far below K*53 bits
        approx = Fraction(math.isqrt(2 * j * j * scale * scale), scale)
        out[:, j - 1] = _round_to_components(approx, K)
    return out


def _sqrt_2p3i(digits=140):
    getcontext().prec = digits
    mod = Decimal(13).sqrt()
    re = ((mod + 2) / 2).sqrt()
    im = ((mod - 2) / 2).sqrt()
    return Fraction(re), Fraction(im)


def sqrt_2p3i_vector(n, K):
    """v_j = sqrt(2+3i) * j (principal root), j = 1..n, as two (K, n) arrays (Sec. 4, Eq. 4)."""
    re, im = _sqrt_2p3i()
    vre = np.zeros((K, n))
    vim = np.zeros((K, n))
    for j in range(1, n + 1):
        vre[:, j - 1] = _round_to_components(re * j, K)
        vim[:, j - 1] = _round_to_components(im * j, K)
    return vre, vim


# --------------------------------------------------------------------------------------
# sparsity patterns
# --------------------------------------------------------------------------------------

def csr_from_dense(dense):
    """CSR arrays (row_ptr, col_idx, values) of a small dense numpy matrix, row-wise order."""
    dense = np.asarray(dense, dtype=np.float64)
    rows, cols = np.nonzero(dense)
    row_ptr = np.zeros(dense.shape[0] + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols.astype(np.int32), dense[rows, cols]


def paper_example_5x5():
    """The 5x5 example matrix of Sec. 3, Eq. 1 as a dense array."""
    return np.array([[1, 0, 2, 0, 0],
                     [0, 3, 0, 0, -4],
                     [0, 0, 5, 0, 0],
                     [6, 0, 0, -7, 0],
                     [0, 0, 0, 0, 8]], dtype=np.float64)


def laplace2d_5pt(nx=100, K=2, seed=0):
    """2D 5-point operator on an nx-by-nx grid (natural row-major order).

    Leading values: diagonal 4+u, off-diagonals -1+0.01u, u ~ U(-1,1) independent per
    entry (so the matrix is not symmetric); then K-component tails.  Draw order:
    the nnz u's (in CSR order), then the tails.  Returns (row_ptr, col_idx, a (K, nnz)).
    """
    rng = np.random.default_rng(seed)
    n = nx * nx
    ii, jj = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    rows, cols = [], []
    for di, dj in ((-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)):
        ok = (ii + di >= 0) & (ii + di < nx) & (jj + dj >= 0) & (jj + dj < nx)
        rows.append((ii * nx + jj)[ok])
        cols.append(((ii + di) * nx + (jj + dj))[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    u = rng.uniform(-1.0, 1.0, size=rows.size)
    lead = np.where(rows == cols, 4.0 + u, -1.0 + 0.01 * u)
    a = mp_from_leads(lead, K, rng)
    return row_ptr.astype(np.int32), cols.astype(np.int32), a


def random_csr(n_rows, n_cols, lengths, K, rng, cplx=False):
    """Random CSR with the given per-row lengths (<= n_cols), uniform distinct sorted columns.

    Returns (row_ptr, col_idx, a_re, a_im or None) with U(-1,1) leads and K-component tails.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    cols = [np.sort(rng.choice(n_cols, size=int(L), replace=False)) for L in lengths]
    col_idx = (np.concatenate(cols) if cols else np.zeros(0)).astype(np.int32)
    nnz = col_idx.size
    a_re = random_mp(nnz, K, rng)
    a_im = random_mp(nnz, K, rng) if cplx else None
    return row_ptr, col_idx, a_re, a_im


def powerlaw_xmin(mean=27.0, alpha=1.1, maxlen=4096):
    """x_min such that E[min(maxlen, floor(x_min U^(-1/alpha)))] == mean, U ~ U(0,1].

    E[L] = sum_{k=1}^{maxlen} P(L >= k) = sum_k min(1, (x_min/k)^alpha); bisection.
    """
    k = np.arange(1, maxlen + 1, dtype=np.float64)

    def expect(xm):
        return float(np.minimum(1.0, (xm / k) ** alpha).sum())

    lo, hi = 1.0, float(maxlen)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if expect(mid) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def powerlaw_pattern(n=1_000_000, mean=27.0, alpha=1.1, maxlen=4096, band=2000, p_band=0.7, seed=1, n_cols=None):
    """Power-law CSR pattern (row lengths with density ~ L^-(1+alpha), clipped at maxlen).

    Row length L_i = min(maxlen, n, floor(x_min * U^(-1/alpha))).  Each entry of row i is
    a band entry with probability p_band (column uniform in the window
    [i - band/2, i + band/2) clipped to [0, n)) or a uniform entry (column uniform in
    [0, n)).  Columns are distinct within a row: a row whose band draws exceed its
    window keeps the first |window| of them and turns the rest into uniform draws;
    duplicates are redrawn from their own law until none is left (rows that need more
    than half of their window are drawn as a random subset of the window directly).
    n_cols (default n): uniform entries are drawn from [0, n_cols) instead.
    Returns (row_ptr int32, col_idx int32).
    """
    nc = n if n_cols is None else int(n_cols)
    rng = np.random.default_rng(seed)
    xmin = powerlaw_xmin(mean, alpha, maxlen)
    u = 1.0 - rng.random(n)  # (0, 1]
    lengths = np.minimum(np.minimum(maxlen, n), np.floor(xmin * u ** (-1.0 / alpha))).astype(np.int64)
    nnz = int(lengths.sum())
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(lengths)
    row_of = np.repeat(np.arange(n, dtype=np.int64), lengths)
    half = band // 2
    w_lo = np.maximum(0, np.arange(n, dtype=np.int64) - half)
    w_hi = np.minimum(n, np.arange(n, dtype=np.int64) + half)
    w_size = w_hi - w_lo
    is_band = rng.random(nnz) < p_band
    # band capacity: keep the first |window| band flags of a row
    nb_incl = np.cumsum(is_band)
    nb_before_row = np.concatenate([[0], nb_incl])[row_ptr[:-1]]
    within = nb_incl - 1 - nb_before_row[row_of]
    is_band &= within < w_size[row_of]
    nb_row = np.bincount(row_of[is_band], minlength=n)
    dense_rows = np.nonzero(nb_row * 4 > w_size)[0]

    cols = np.empty(nnz, dtype=np.int64)
    r_u = rng.random(nnz)
    cols[is_band] = w_lo[row_of[is_band]] + np.floor(r_u[is_band] * w_size[row_of[is_band]]).astype(np.int64)
    cols[~is_band] = np.floor(r_u[~is_band] * nc).astype(np.int64)
    # rows needing more than a quarter of their window: a random subset of the window
    for i in dense_rows:
        sel = np.nonzero(is_band[row_ptr[i]:row_ptr[i + 1]])[0] + row_ptr[i]
        cols[sel] = w_lo[i] + rng.choice(w_size[i], size=sel.size, replace=False)
    # redraw duplicates from their own law; of an equal pair the uniform entry (else the
    # later band entry) is redrawn, so a full window never has to find a free slot.
    # After the first pass only the entries of rows that still hold duplicates are revisited.
    ent = np.arange(nnz, dtype=np.int64)
    for _ in range(200):
        key = row_of[ent] * nc + cols[ent]
        order = np.argsort(key * 2 + (~is_band[ent]), kind="stable")
        ks = key[order]
        dup_sorted = np.zeros(ent.size, dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        if not dup_sorted.any():
            break
        dup = ent[order[dup_sorted]]
        r = rng.random(dup.size)
        b = is_band[dup]
        cols[dup[b]] = w_lo[row_of[dup[b]]] + np.floor(r[b] * w_size[row_of[dup[b]]]).astype(np.int64)
        cols[dup[~b]] = np.floor(r[~b] * nc).astype(np.int64)
        rows_left = np.unique(row_of[dup])
        ent = np.concatenate([np.arange(row_ptr[i], row_ptr[i + 1]) for i in rows_left])
    else:
        raise RuntimeError("powerlaw_pattern: duplicate columns did not resolve")
    # sort columns within rows
    key = row_of * nc + cols
    cols = (np.sort(key) - row_of * nc).astype(np.int32)
    return row_ptr.astype(np.int32), cols


def powerlaw_csr(n=1_000_000, K=2, cplx=False, seed=1, **kw):
    """Power-law pattern plus U(-1,1) values with K-component tails (real, or independent re/im).

    Returns (row_ptr, col_idx, a_re, a_im or None, x_re, x_im or None).  The values use
    a separate stream seeded with (seed, K, cplx) so that every variant of one pattern
    is reproducible on its own.
    """
    row_ptr, col_idx = powerlaw_pattern(n=n, seed=seed, **kw)
    rng = np.random.default_rng([seed, K, int(cplx)])
    nnz = col_idx.size
    a_re = random_mp(nnz, K, rng)
    a_im = random_mp(nnz, K, rng) if cplx else None
    x_re = random_mp(n, K, rng)
    x_im = random_mp(n, K, rng) if cplx else None
    return row_ptr, col_idx, a_re, a_im, x_re, x_im


def diffusion3d_7pt(m=64, sigma=2.5, az=1.0, K=2, seed=2):
    """Cell-centred 7-point diffusion operator on an m^3 grid, Dirichlet-0 boundary.

    Cell coefficients kappa_c = exp(sigma * xi_c), xi ~ N(0,1) i.i.d.  The face between
    cells p and q along axis d has transmissibility f_d * 2 kappa_p kappa_q/(kappa_p +
    kappa_q) with axis factors f = (1, 1, az); a boundary face has f_d * 2 kappa_c.
    Off-diagonal entry (p, q) = -T_pq (the same binary64 lead and the same tails for
    (p, q) and (q, p), so A is exactly symmetric); the diagonal lead is fl(sum of the
    cell's face transmissibilities) with its own tails.  The diagonal exceeds the sum
    of the off-diagonal magnitudes by the boundary faces, so A is SPD.
    Returns (row_ptr, col_idx, a (K, nnz)).
    """
    rng = np.random.default_rng(seed)
    n = m ** 3
    kappa = np.exp(sigma * rng.standard_normal(n)).reshape(m, m, m)
    f = (1.0, 1.0, az)
    idx = np.arange(n).reshape(m, m, m)
    diag = np.zeros((m, m, m))
    rows, cols, vals = [], [], []
    for d in range(3):
        sl_a = [slice(None)] * 3
        sl_b = [slice(None)] * 3
        sl_a[d] = slice(0, m - 1)
        sl_b[d] = slice(1, m)
        ka, kb = kappa[tuple(sl_a)], kappa[tuple(sl_b)]
        t = f[d] * 2.0 * ka * kb / (ka + kb)
        diag[tuple(sl_a)] += t
        diag[tuple(sl_b)] += t
        pa, pb = idx[tuple(sl_a)].ravel(), idx[tuple(sl_b)].ravel()
        rows += [pa, pb]
        cols += [pb, pa]
        vals += [t.ravel(), t.ravel()]
        # boundary faces
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, 1)
        hi[d] = slice(m - 1, m)
        diag[tuple(lo)] += f[d] * 2.0 * kappa[tuple(lo)]
        diag[tuple(hi)] += f[d] * 2.0 * kappa[tuple(hi)]
    nface = rows[0].size + rows[2].size + rows[4].size
    # one tail draw per face, shared by the two symmetric entries
    face_leads = -np.concatenate([vals[0], vals[2], vals[4]])
    face_mp = mp_from_leads(face_leads, K, rng)
    diag_mp = mp_from_leads(diag.ravel(), K, rng)
    off0 = [0, rows[0].size, rows[0].size + rows[2].size]
    r_all, c_all, v_all = [], [], []
    for d in range(3):
        fm = face_mp[:, off0[d]:off0[d] + rows[2 * d].size]
        r_all += [rows[2 * d], rows[2 * d + 1]]
        c_all += [cols[2 * d], cols[2 * d + 1]]
        v_all += [fm, fm]
    r_all.append(np.arange(n))
    c_all.append(np.arange(n))
    v_all.append(diag_mp)
    r = np.concatenate(r_all)
    c = np.concatenate(c_all)
    v = np.concatenate(v_all, axis=1)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[:, order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    assert nface * 2 + n == c.size
    return row_ptr.astype(np.int32), c.astype(np.int32), np.ascontiguousarray(v)


def banded_nonsymmetric(n=1000, K=2, seed=3, diag=2.0, lower=-1.015, upper=-0.985, upper2=-0.0009):
    """Narrow-band non-symmetric matrix shaped like the paper's tub1000 (n = 1000, 3,996
    nonzeros): bands at offsets -1, 0, +1, +2 (4n - 4 entries), leads
    diag(1 + 0.01u), lower(1 + 0.01u), upper(1 + 0.01u), upper2(1 + 0.01u) with
    u ~ U(-1,1) per entry, then K-component tails.  Returns (row_ptr, col_idx, a)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for off, v in ((-1, lower), (0, diag), (1, upper), (2, upper2)):
        i = np.arange(max(0, -off), min(n, n - off))
        rows.append(i)
        cols.append(i + off)
        vals.append(np.full(i.size, v))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    lead = v * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=v.size))
    a = mp_from_leads(lead, K, rng)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), c.astype(np.int32), a


def batched_diffusion(edges, sigma=2.5, seed=3, K=2, az=1.0):
    """Block-diagonal CSR of independent 3D diffusion systems (one per grid edge in
    `edges`, system s generated by diffusion3d_7pt with seed (seed, s)).  Returns
    (row_ptr, col_idx, a (K, nnz), sys_ptr)."""
    rps, cis, avs, sys_ptr = [], [], [], [0]
    row_off = 0
    nnz_off = 0
    for s, m in enumerate(edges):
        rp, ci, a = diffusion3d_7pt(m=int(m), sigma=sigma, az=az, K=K, seed=int(seed) * 100003 + s)
        rps.append(rp[:-1].astype(np.int64) + nnz_off)
        cis.append(ci.astype(np.int64) + row_off)
        avs.append(a)
        row_off += rp.size - 1
        nnz_off += ci.size
        sys_ptr.append(row_off)
    row_ptr = np.concatenate(rps + [np.array([nnz_off])]).astype(np.int32)
    return row_ptr, np.concatenate(cis).astype(np.int32), np.concatenate(avs, axis=1), np.array(sys_ptr, np.int32)
