/*
 * exact_resid.c -- CPU ORACLE, exact residuals.  TEST INFRASTRUCTURE ONLY.
 *
 * Certifies a solve (Sec. 4.2: the solvers stop on ||b - A x|| <= rtol ||b||) without
 * trusting any rounded arithmetic: every stored binary64 component is an integer
 * times a power of two, so
 *
 *     r_i = sum_k b_i[k] - sum_j sum_k sum_l a_ij[k] x_j[l]
 *
 * (a, b and x taken as the exact sums of their stored components, Sec. 3) is an
 * integer multiple of 2^(lowest exponent in the row) and is formed exactly in a
 * long fixed-point accumulator (a Kulisch-style register of 32-bit digits held in
 * signed 64-bit cells, carries resolved once per row).  Each product of two
 * binary64 values is the product of their 53-bit integer significands (at most 106
 * bits, formed in unsigned 128-bit arithmetic) placed at the sum of their
 * exponents.  Nothing here uses the method's arithmetic (no error-free
 * transformations, no multi-component operations).
 *
 * From the exact r_i and b_i the routine returns
 *   r_near[i]  r_i rounded to the nearest binary64 (ties to even), optional;
 *   norms[0]   an upper bound on ||r||^2: each |r_i| rounded away from zero, squared
 *              and summed in binary64, times (1 + (n + 2) 2^-52);
 *   norms[1]   a lower bound on ||b||^2: each |b_i| rounded toward zero, squared,
 *              summed, times (1 - (n + 2) 2^-52);
 *   norms[2]   sum of r_near[i]^2 (for information);
 *   norms[3]   sum of the nearest binary64 of b_i, squared (for information).
 * The bound factors cover the rounding of each square and of each partial sum
 * (relative error at most 2^-53 per operation, n + 1 operations per total), so
 * norms[0] >= ||r||^2 and norms[1] <= ||b||^2 hold exactly unless a sum overflows
 * (then the routine returns -2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DIGIT_BITS 32
#define MAX_CELLS 160   /* 5120 bits: every binary64 product and sum fits */

typedef struct {
    int64_t cell[MAX_CELLS];
    int ncell;
    int base;           /* exponent of bit 0 of cell 0 */
} longacc;

/* v = m * 2^e with m a 53-bit (or smaller) integer; returns 0 for v == 0 */
static uint64_t decompose(double v, int *e)
{
    int ex;
    double f;
    if (v == 0.0) {
        *e = 0;
        return 0;
    }
    f = frexp(fabs(v), &ex);                /* v = f 2^ex, 0.5 <= f < 1 */
    *e = ex - 53;
    return (uint64_t)ldexp(f, 53);          /* exact: f has at most 53 significant bits */
}

/* add sign * m * 2^e (m < 2^107) into the accumulator */
static void acc_add(longacc *A, int negative, unsigned __int128 m, int e)
{
    int pos, c, o;
    if (m == 0) return;
    pos = e - A->base;
    c = pos / DIGIT_BITS;
    o = pos % DIGIT_BITS;
    /* m << o has at most 107 + 31 = 138 bits: five digits */
    {
        unsigned __int128 lo = m << o;                 /* low 128 bits */
        uint64_t hi = o ? (uint64_t)(m >> (128 - o)) : 0;   /* bits 128.. */
        int d;
        for (d = 0; d < 4; ++d) {
            int64_t dig = (int64_t)(uint32_t)(lo >> (DIGIT_BITS * d));
            A->cell[c + d] += negative ? -dig : dig;
        }
        A->cell[c + 4] += negative ? -(int64_t)hi : (int64_t)hi;
    }
}

/* resolve carries: afterwards cells 0..ncell-2 hold digits in [0, 2^32) and the top
 * cell the (signed) rest; returns the sign of the value (-1, 0, 1) */
static int acc_normalize(longacc *A)
{
    int i, nz = 0;
    for (i = 0; i + 1 < A->ncell; ++i) {
        int64_t v = A->cell[i];
        int64_t carry = v >> DIGIT_BITS;               /* arithmetic shift: floor division */
        A->cell[i] = v - carry * ((int64_t)1 << DIGIT_BITS);
        A->cell[i + 1] += carry;
    }
    if (A->cell[A->ncell - 1] < 0) return -1;
    for (i = 0; i < A->ncell; ++i) nz |= A->cell[i] != 0;
    return nz ? 1 : 0;
}

/* negate a normalized negative value into its (non-negative) magnitude */
static void acc_negate(longacc *A)
{
    int i;
    for (i = 0; i < A->ncell; ++i) A->cell[i] = -A->cell[i];
    acc_normalize(A);
}

/* a normalized non-negative accumulator rounded to binary64: mode 0 nearest (ties to
 * even), 1 away from zero, 2 toward zero */
static double acc_round(const longacc *A, int mode)
{
    int top = A->ncell - 1, bit, i, shift;
    uint64_t lead = 0;
    int sticky = 0;
    double r;
    while (top >= 0 && A->cell[top] == 0) --top;
    if (top < 0) return 0.0;
    /* the top cell may exceed 32 bits only if it is the last cell; cells are small
       enough that the value's highest set bit is found by scanning */
    {
        uint64_t t = (uint64_t)A->cell[top];
        bit = 63;
        while (!((t >> bit) & 1)) --bit;
        bit += top * DIGIT_BITS;                       /* absolute index of the highest bit */
    }
    /* take bits bit .. bit-63 into lead (64 bits), the rest into sticky */
    for (i = 0; i < 64; ++i) {
        int b = bit - i, c, o;
        uint64_t v;
        if (b < 0) break;
        c = b / DIGIT_BITS;
        o = b % DIGIT_BITS;
        v = ((uint64_t)A->cell[c] >> o) & 1;
        lead |= v << (63 - i);
    }
    for (i = 0; i <= bit - 64; ++i) {
        int c = i / DIGIT_BITS, o = i % DIGIT_BITS;
        if (((uint64_t)A->cell[c] >> o) & 1) { sticky = 1; break; }
    }
    /* lead holds the 64 leading bits: keep 53, decide with the other 11 and sticky */
    {
        uint64_t keep = lead >> 11, rest = lead & 0x7FF;
        int exact = (rest == 0 && !sticky);
        if (mode == 0) {
            if (rest > 0x400 || (rest == 0x400 && (sticky || (keep & 1)))) keep += 1;
        } else if (mode == 1) {
            if (!exact) keep += 1;
        }
        shift = bit - 52 + A->base;                    /* value = keep * 2^shift */
        r = ldexp((double)keep, shift);                /* keep <= 2^53: exact unless it overflows */
    }
    return r;
}

/* exponent range of the terms of row i: [emin, emax] of the lowest bits and highest
 * bits of every product and b component; returns 0 when every term is zero */
static int row_range(int Ka, int Kx, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                     const double *a, const double *b, const double *x, int64_t i, int *emin, int *emax)
{
    int any = 0, lo = 0, hi = 0, k, l, e1, e2;
    int64_t p;
    for (k = 0; k < Kx; ++k) {
        uint64_t m = decompose(b[k * n + i], &e1);
        if (m) {
            if (!any || e1 < lo) lo = e1;
            if (!any || e1 + 53 > hi) hi = e1 + 53;
            any = 1;
        }
    }
    for (p = rp[i]; p < rp[i + 1]; ++p) {
        int64_t j = ci[p];
        for (k = 0; k < Ka; ++k) {
            uint64_t ma = decompose(a[k * nnz + p], &e1);
            if (!ma) continue;
            for (l = 0; l < Kx; ++l) {
                uint64_t mx = decompose(x[l * n + j], &e2);
                if (!mx) continue;
                if (!any || e1 + e2 < lo) lo = e1 + e2;
                if (!any || e1 + e2 + 106 > hi) hi = e1 + e2 + 106;
                any = 1;
            }
        }
    }
    *emin = lo;
    *emax = hi;
    return any;
}

/*
 * Ka: components of the matrix values (1 = binary64 matrix, 2..4); Kx: components of
 * b and x (1..4).  a: Ka*nnz, b and x: Kx*n (planar).  Square n x n matrix.
 * Returns 0, -1 for bad arguments or a row whose terms span more than the
 * accumulator, -2 if a norm bound overflows.
 */
int oracle_exact_residual(int Ka, int Kx, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *a, const double *b, const double *x, double *r_near, double *norms)
{
    double rr_up = 0.0, bb_lo = 0.0, rr_n = 0.0, bb_n = 0.0;
    int64_t i;
    int bad = 0;
    if (Ka < 1 || Ka > 4 || Kx < 1 || Kx > 4 || n < 0 || !norms) return -1;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : rr_up, bb_lo, rr_n, bb_n) reduction(| : bad)
    for (i = 0; i < n; ++i) {
        longacc R, B;
        int emin, emax, k, l, e1, e2, s;
        int64_t p;
        double up, lo, near, bn;
        if (!row_range(Ka, Kx, n, nnz, row_ptr, col_idx, a, b, x, i, &emin, &emax)) {
            if (r_near) r_near[i] = 0.0;
            continue;
        }
        R.base = emin;
        R.ncell = (emax - emin + 64) / DIGIT_BITS + 3;   /* room for the carries of ~2^31 terms */
        if (R.ncell > MAX_CELLS) { bad = 1; continue; }
        memset(R.cell, 0, sizeof(int64_t) * (size_t)R.ncell);
        B = R;
        for (k = 0; k < Kx; ++k) {
            double v = b[k * n + i];
            uint64_t m = decompose(v, &e1);
            acc_add(&R, v < 0, m, e1);
            acc_add(&B, v < 0, m, e1);
        }
        for (p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col_idx[p];
            for (k = 0; k < Ka; ++k) {
                double av = a[k * nnz + p];
                uint64_t ma = decompose(av, &e1);
                if (!ma) continue;
                for (l = 0; l < Kx; ++l) {
                    double xv = x[l * n + j];
                    uint64_t mx = decompose(xv, &e2);
                    if (!mx) continue;
                    /* r -= a x: the product's sign flipped */
                    acc_add(&R, !((av < 0) != (xv < 0)), (unsigned __int128)ma * mx, e1 + e2);
                }
            }
        }
        s = acc_normalize(&R);
        if (s < 0) acc_negate(&R);
        up = acc_round(&R, 1);
        near = acc_round(&R, 0);
        if (r_near) r_near[i] = s < 0 ? -near : near;
        rr_up += up * up;
        rr_n += near * near;
        s = acc_normalize(&B);
        if (s < 0) acc_negate(&B);
        lo = acc_round(&B, 2);
        bn = acc_round(&B, 0);
        bb_lo += lo * lo;
        bb_n += bn * bn;
    }
    if (bad) return -1;
    {
        const double grow = ldexp((double)(n + 2), -52);
        norms[0] = rr_up * (1.0 + grow);
        norms[1] = bb_lo * (1.0 - grow);
        norms[2] = rr_n;
        norms[3] = bb_n;
        if (!isfinite(norms[0]) || !isfinite(norms[1])) return -2;
    }
    return 0;
}
