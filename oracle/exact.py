"""Exact arithmetic for pinning the oracle.  TEST INFRASTRUCTURE ONLY.

Every binary64 value is an integer times a power of two, so sums of products of
stored components can be formed exactly with Python integers on a common scale
2^E.  This module computes

* the exact product y_i = sum_j a_ij x_j of a CSR matrix and a vector whose entries
  are the exact sums of their stored components (the quantity the multi-component
  SpMV approximates, Sec. 3), and the matching sum of |a_ij||x_j|;
* exact values of multi-component numbers, for comparisons.

It uses no part of the method's arithmetic (no error-free transformations).
"""
from fractions import Fraction
import math

import numpy as np

E_SCALE = -2400  # products of binary64 values are multiples of 2^-2148


def fixed(v, E=E_SCALE):
    """Exact integer v * 2^-E of a finite binary64 v (E <= its lowest set bit)."""
    v = float(v)
    if v == 0.0:
        return 0
    m, e = math.frexp(v)
    M = int(m * (1 << 53))
    sh = e - 53 - E
    assert sh >= 0
    return M << sh


def fixed_mp(comps, E=E_SCALE):
    """Exact scaled integer of the sum of a multi-component value's components."""
    return sum(fixed(c, E) for c in comps)


def mp_value(comps):
    """Exact Fraction of a multi-component value (sum of its components)."""
    return sum((Fraction(float(c)) for c in comps), Fraction(0))


def _mant(v):
    """(M, e) with v = M * 2^e exactly, M an int."""
    if v == 0.0:
        return 0, 0
    m, e = math.frexp(v)
    return int(m * (1 << 53)), e - 53


def _prod_fixed(a, b, E):
    ma, ea = _mant(a)
    mb, eb = _mant(b)
    if ma == 0 or mb == 0:
        return 0
    sh = ea + eb - E
    assert sh >= 0
    return (ma * mb) << sh


def exact_row_products(row_ptr, col_idx, a, x, rows=None, E=E_SCALE):
    """Exact y_i and S_i = sum_j |a_ij||x_j| (as integers scaled by 2^-E) for the given rows.

    a: (K, nnz) components; x: (K, n) components.  Returns two Python lists.
    """
    a = np.asarray(a)
    x = np.asarray(x)
    Ka, Kx = a.shape[0], x.shape[0]
    rows = range(len(row_ptr) - 1) if rows is None else rows
    ys, ss = [], []
    for i in rows:
        y = 0
        s = 0
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            j = int(col_idx[k])
            av = [float(a[c, k]) for c in range(Ka)]
            xv = [float(x[c, j]) for c in range(Kx)]
            p = 0
            for ac in av:
                for xc in xv:
                    p += _prod_fixed(ac, xc, E)
            y += p
            s += abs(sum(fixed(c, E) for c in av)) * abs(sum(fixed(c, E) for c in xv)) >> (-E)
        ys.append(y)
        ss.append(s)
    return ys, ss


def within_bound(computed_fixed, exact_fixed, abs_fixed_sum, length, bits, E=E_SCALE):
    """|computed - exact| <= max(len,1) * 2^-bits * abs_sum, all exact.

    abs_fixed_sum is scaled by 2^-E (like the others); the test is done on integers.
    """
    lhs = abs(computed_fixed - exact_fixed) << bits
    rhs = max(int(length), 1) * abs_fixed_sum
    return lhs <= rhs


def error_ratio(computed_fixed, exact_fixed, abs_fixed_sum, length, bits):
    """|computed - exact| / (max(len,1) 2^-bits abs_sum) as a float (<= 1 means within bound)."""
    if abs_fixed_sum == 0:
        return 0.0 if computed_fixed == exact_fixed else math.inf
    return float(Fraction(abs(computed_fixed - exact_fixed) << bits, max(int(length), 1) * abs_fixed_sum))
