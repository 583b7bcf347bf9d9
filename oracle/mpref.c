/*
 * mpref.c -- CPU ORACLE.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, scalar, deliberately slow reference for multi-component (double-double,
 * triple-double, quad-double) CSR sparse matrix-vector products and the DD Krylov
 * solvers built on them.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no source with the GPU
 * library: every definition below is written from the paper (Kouya, "Performance
 * evaluation of accelerated real and complex multiple-precision sparse
 * matrix-vector multiplication", arXiv 2412.17510) and from the published
 * quad-double algorithms of Hida, Li and Bailey (ARITH-15, 2001) that the paper
 * builds its QD/TD arithmetic on.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no contraction: every "+" and "*" below is one IEEE binary64 operation with
 * round-to-nearest-even, and the only fused operation is none at all -- the
 * error of a product is obtained by Dekker's splitting, not by an FMA, so that
 * this oracle and the GPU's FMA-based TwoProd reach the same exact error term by
 * two different algorithms).
 *
 * Multi-component storage (Sec. 3): an array of L values with K components is one
 * block of K*L doubles, component c of element i at base[c*L + i] (component 0 is
 * the leading one).  Complex data are two such blocks (real, imaginary) over one
 * shared sparsity pattern (Sec. 3, Eq. 2).
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double c[4]; } mpv;   /* components beyond K are kept at +0 */

/* ------------------------------------------------------------------------- */
/* Error-free transformations (Sec. 2: QuickTwoSum, TwoSum, TwoProd).         */
/* ------------------------------------------------------------------------- */

/* Knuth's TwoSum: s = fl(a+b) and e with s + e == a + b exactly. */
static void two_sum(double a, double b, double *s, double *e)
{
    double sum = a + b;
    double b_virtual = sum - a;
    double a_virtual = sum - b_virtual;
    double b_round = b - b_virtual;
    double a_round = a - a_virtual;
    *s = sum;
    *e = a_round + b_round;
}

/* Dekker's QuickTwoSum (FastTwoSum): exact when |a| >= |b| or a == 0. */
static void quick_two_sum(double a, double b, double *s, double *e)
{
    double sum = a + b;
    *s = sum;
    *e = b - (sum - a);
}

/* Veltkamp/Dekker splitting of a binary64 into two 26-bit halves. */
static void split53(double a, double *hi, double *lo)
{
    double c = 134217729.0 * a;          /* 2^27 + 1 */
    double big = c - a;
    double h = c - big;
    *hi = h;
    *lo = a - h;
}

/* Dekker's TwoProduct: p = fl(a*b) and e with p + e == a*b exactly (no FMA). */
static void two_prod(double a, double b, double *p, double *e)
{
    double ah, al, bh, bl;
    double prod = a * b;
    split53(a, &ah, &al);
    split53(b, &bh, &bl);
    double err1 = prod - ah * bh;
    double err2 = err1 - al * bh;
    double err3 = err2 - ah * bl;
    *p = prod;
    *e = al * bl - err3;
}

/* ------------------------------------------------------------------------- */
/* Double-double (Algorithms 1 and 2, printed in full in Sec. 2).             */
/* ------------------------------------------------------------------------- */

/* Algorithm 1: TwoSum of the leading parts, plain sum of the trailing parts,
 * one plain add of the two error terms, QuickTwoSum renormalisation. */
static mpv dd_add(mpv x, mpv y)
{
    double s, e, w;
    mpv r = {{0.0, 0.0, 0.0, 0.0}};
    two_sum(x.c[0], y.c[0], &s, &e);
    w = x.c[1] + y.c[1];
    e = e + w;
    quick_two_sum(s, e, &r.c[0], &r.c[1]);
    return r;
}

/* Algorithm 2: exact product of the leading parts, two plain cross products,
 * their plain sum added to the product error, QuickTwoSum renormalisation. */
static mpv dd_mul(mpv x, mpv y)
{
    double p1, p2, w1, w2, w3;
    mpv r = {{0.0, 0.0, 0.0, 0.0}};
    two_prod(x.c[0], y.c[0], &p1, &p2);
    w1 = x.c[0] * y.c[1];
    w2 = x.c[1] * y.c[0];
    w3 = w1 + w2;
    p2 = p2 + w3;
    quick_two_sum(p1, p2, &r.c[0], &r.c[1]);
    return r;
}

/* Algorithm 3 (DD times binary64), with the trailing component multiplied by
 * y before it is added to the product error (the printed listing omits that
 * multiplication; without it the result is not a product). */
static mpv dd_mul_d(mpv x, double y)
{
    double p1, p2, w;
    mpv r = {{0.0, 0.0, 0.0, 0.0}};
    two_prod(x.c[0], y, &p1, &p2);
    w = x.c[1] * y;
    p2 = w + p2;
    quick_two_sum(p1, p2, &r.c[0], &r.c[1]);
    return r;
}

/* ------------------------------------------------------------------------- */
/* Quad-double (Sec. 2: "sloppy" addition and multiplication built from        */
/* ThreeSum, ThreeSum2 and a renormalisation, after Hida, Li and Bailey).      */
/* ------------------------------------------------------------------------- */

/* ThreeSum: (a, b, c) -> (s, e1, e2) with s + e1 + e2 == a + b + c exactly,
 * s the rounded sum, e1 and e2 the two levels of error below it. */
static void three_sum(double a, double b, double c, double *s, double *e1, double *e2)
{
    double t1, t2, t3;
    two_sum(a, b, &t1, &t2);
    two_sum(c, t1, s, &t3);
    two_sum(t2, t3, e1, e2);
}

/* ThreeSum2: like ThreeSum but the two error terms are merged by one plain add
 * (the third level is not needed by the caller). */
static void three_sum2(double a, double b, double c, double *s, double *e1)
{
    double t1, t2, t3;
    two_sum(a, b, &t1, &t2);
    two_sum(c, t1, s, &t3);
    *e1 = t2 + t3;
}

/* Renormalisation of five roughly ordered terms into four non-overlapping
 * components.  First sweep, bottom-up: a chain of QuickTwoSums from the
 * smallest term to the largest leaves t0 (the rounded total) and the errors
 * t1..t4.  Second sweep, top-down: (t0, t1) is already a QuickTwoSum pair, so a
 * non-zero t1 closes t0 as the first component and t1 becomes the carry s (else
 * s = t0); then for i = 2..4 form (s, e) = QuickTwoSum(s, t_i): a non-zero e
 * closes the current component (s is emitted and e becomes the new carry), a zero
 * e lets the carry absorb t_i.  Once three components are closed the fourth only
 * absorbs (its errors are dropped); the final carry is the last component.  Tests
 * against zero are exact comparisons with 0.0. */
static mpv renorm5(double c0, double c1, double c2, double c3, double c4)
{
    double s, t[5], e;
    mpv r = {{0.0, 0.0, 0.0, 0.0}};
    int k = 0, i;
    quick_two_sum(c3, c4, &s, &t[4]);
    quick_two_sum(c2, s, &s, &t[3]);
    quick_two_sum(c1, s, &s, &t[2]);
    quick_two_sum(c0, s, &t[0], &t[1]);
    s = t[0];
    if (t[1] != 0.0) {
        r.c[0] = t[0];
        k = 1;
        s = t[1];
    }
    for (i = 2; i <= 4; ++i) {
        double sn;
        quick_two_sum(s, t[i], &sn, &e);
        s = sn;
        if (e != 0.0 && k < 3) {
            r.c[k] = s;
            k = k + 1;
            s = e;
        }
    }
    r.c[k] = s;
    return r;
}

/* QD sloppy addition: componentwise TwoSum, then the error terms are merged
 * level by level (order eps, eps^2, eps^3) and the rest is summed plainly. */
static mpv qd_add(mpv x, mpv y)
{
    double s0, s1, s2, s3, e0, e1, e2, e3, t;
    two_sum(x.c[0], y.c[0], &s0, &e0);
    two_sum(x.c[1], y.c[1], &s1, &e1);
    two_sum(x.c[2], y.c[2], &s2, &e2);
    two_sum(x.c[3], y.c[3], &s3, &e3);
    /* order eps: s1 and the error of the leading sum */
    two_sum(s1, e0, &s1, &e0);
    /* order eps^2: s2, e0, e1 */
    three_sum(s2, e0, e1, &s2, &e0, &e1);
    /* order eps^3: s3, e0, e2 */
    three_sum2(s3, e0, e2, &s3, &e0);
    /* order eps^4: what is left */
    t = e0 + e1;
    t = t + e3;
    return renorm5(s0, s1, s2, s3, t);
}

/* QD sloppy multiplication: exact products for the partial products of order
 * 1, eps and eps^2, plain products for order eps^3 (order eps^4 and below is
 * not formed); each order is merged with the errors from the order above. */
static mpv qd_mul(mpv x, mpv y)
{
    double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
    double h1, m1, l1, u0, u1, u2, v0, v1, v2, s0, s1, s2, f0, f1, t;
    two_prod(x.c[0], y.c[0], &p0, &q0);               /* order 1   */
    two_prod(x.c[0], y.c[1], &p1, &q1);               /* order eps */
    two_prod(x.c[1], y.c[0], &p2, &q2);
    two_prod(x.c[0], y.c[2], &p3, &q3);               /* order eps^2 */
    two_prod(x.c[1], y.c[1], &p4, &q4);
    two_prod(x.c[2], y.c[0], &p5, &q5);
    /* order eps: p1, p2 and the error of the leading product */
    three_sum(p1, p2, q0, &h1, &m1, &l1);
    /* order eps^2: six terms -- m1, q1, q2 and p3, p4, p5 -- merged as two
     * ThreeSums whose outputs are added level by level */
    three_sum(m1, q1, q2, &u0, &u1, &u2);
    three_sum(p3, p4, p5, &v0, &v1, &v2);
    two_sum(u0, v0, &s0, &f0);
    two_sum(u1, v1, &s1, &f1);
    s2 = u2 + v2;
    two_sum(s1, f0, &s1, &f0);
    s2 = s2 + (f0 + f1);
    /* order eps^3: the four plain products and the errors from order eps^2 */
    t = x.c[0] * y.c[3];
    t = t + x.c[1] * y.c[2];
    t = t + x.c[2] * y.c[1];
    t = t + x.c[3] * y.c[0];
    t = t + l1;
    t = t + q3;
    t = t + q4;
    t = t + q5;
    s1 = s1 + t;
    return renorm5(p0, h1, s0, s1, s2);
}

/* Triple-double (Sec. 2): the QD operations applied with the fourth component
 * of both operands set to zero; the result keeps its first three components. */
static mpv td_trunc(mpv r) { r.c[3] = 0.0; return r; }
static mpv td_add(mpv x, mpv y) { x.c[3] = 0.0; y.c[3] = 0.0; return td_trunc(qd_add(x, y)); }
static mpv td_mul(mpv x, mpv y) { x.c[3] = 0.0; y.c[3] = 0.0; return td_trunc(qd_mul(x, y)); }

static mpv mp_add(int K, mpv x, mpv y)
{
    return K == 2 ? dd_add(x, y) : (K == 3 ? td_add(x, y) : qd_add(x, y));
}
static mpv mp_mul(int K, mpv x, mpv y)
{
    return K == 2 ? dd_mul(x, y) : (K == 3 ? td_mul(x, y) : qd_mul(x, y));
}
static mpv mp_neg(mpv x)
{
    mpv r;
    int c;
    for (c = 0; c < 4; ++c) r.c[c] = -x.c[c];
    return r;
}

static mpv load_mp(int K, const double *base, int64_t len, int64_t i)
{
    mpv v = {{0.0, 0.0, 0.0, 0.0}};
    int c;
    for (c = 0; c < K; ++c) v.c[c] = base[(int64_t)c * len + i];
    return v;
}
static void store_mp(int K, double *base, int64_t len, int64_t i, mpv v)
{
    int c;
    for (c = 0; c < K; ++c) base[(int64_t)c * len + i] = v.c[c];
}

/* ------------------------------------------------------------------------- */
/* Exported element-wise operations (for the tests of the arithmetic itself). */
/* op: 0 = add, 1 = mul, 2 = mul by binary64 (DD only, y holds n doubles).     */
/* ------------------------------------------------------------------------- */
int oracle_eft(int which, int64_t n, const double *a, const double *b, double *s, double *e)
{
    int64_t i;
    for (i = 0; i < n; ++i) {
        if (which == 0) two_sum(a[i], b[i], &s[i], &e[i]);
        else if (which == 1) quick_two_sum(a[i], b[i], &s[i], &e[i]);
        else if (which == 2) two_prod(a[i], b[i], &s[i], &e[i]);
        else return -1;
    }
    return 0;
}

int oracle_elementwise(int K, int op, int64_t n, const double *x, const double *y, double *r)
{
    int64_t i;
    if (K < 2 || K > 4) return -1;
    for (i = 0; i < n; ++i) {
        mpv a = load_mp(K, x, n, i), out;
        if (op == 2) {
            if (K != 2) return -1;
            out = dd_mul_d(a, y[i]);
        } else {
            mpv b = load_mp(K, y, n, i);
            out = op == 0 ? mp_add(K, a, b) : mp_mul(K, a, b);
        }
        store_mp(K, r, n, i, out);
    }
    return 0;
}

int oracle_renorm5(int64_t n, const double *c /* 5 x n */, double *r /* 4 x n */)
{
    int64_t i;
    for (i = 0; i < n; ++i) {
        mpv o = renorm5(c[i], c[n + i], c[2 * n + i], c[3 * n + i], c[4 * n + i]);
        store_mp(4, r, n, i, o);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* CSR SpMV (Sec. 3, Fig. 1; complex per Eq. 3).                               */
/*                                                                             */
/* Summation order of row i with len = row_ptr[i+1]-row_ptr[i] elements:       */
/*   W = 2^log2w[i] (canonical: the largest power of two <= min(len, 64));     */
/*   lane l < W owns elements row_ptr[i]+l, +W, +2W, ... in that order; its    */
/*   accumulator starts at its first product and then adds each product;       */
/*   the W accumulators are folded as acc[l] = add(acc[l], acc[l+off]) for     */
/*   off = W/2, ..., 1; y_i = acc[0].  An empty row gives +0 in every          */
/*   component.  Products are mul(a_k, x_col) -- the matrix operand first.     */
/* ------------------------------------------------------------------------- */

int oracle_canonical_log2w(int64_t len)
{
    int l = 0;
    if (len <= 0) return 0;
    while (l < 6 && ((int64_t)2 << l) <= len) ++l;
    return l;
}

/* One accumulator set: sum_k mul(A[k], X[col[k]]) in the lane/fold order. */
static mpv row_sum(int K, int64_t start, int64_t len, int W, const int32_t *col,
                   const double *A, int64_t nnz, const double *X, int64_t n, mpv *lanes)
{
    int l, off;
    for (l = 0; l < W; ++l) {
        int64_t k = start + l;
        lanes[l] = mp_mul(K, load_mp(K, A, nnz, k), load_mp(K, X, n, col[k]));
        for (k = k + W; k < start + len; k += W)
            lanes[l] = mp_add(K, lanes[l], mp_mul(K, load_mp(K, A, nnz, k), load_mp(K, X, n, col[k])));
    }
    for (off = W / 2; off >= 1; off /= 2)
        for (l = 0; l < off; ++l)
            lanes[l] = mp_add(K, lanes[l], lanes[l + off]);
    return lanes[0];
}

/*
 * y = A x.  K in {2,3,4}.  a_im/x_im/y_im NULL for a real product.
 * log2w: per-row lane-width exponent (NULL = canonical).  rows: optional list of
 * nsel row indices to compute (NULL = all n_rows rows; other rows of y untouched).
 * Returns 0, or -1 on a bad argument (W > len, W > 1024, K out of range).
 */
int oracle_spmv(int K, int64_t n_rows, int64_t n_cols, int64_t nnz,
                const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                const double *a_re, const double *a_im,
                const double *x_re, const double *x_im,
                double *y_re, double *y_im,
                int64_t nsel, const int64_t *rows, int nthreads)
{
    int64_t t, count = rows ? nsel : n_rows;
    int bad = 0;
    const int cplx = (a_im != NULL);
    if (K < 2 || K > 4) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        mpv *lanes = (mpv *)malloc(sizeof(mpv) * 1024);
#pragma omp for schedule(dynamic, 256)
        for (t = 0; t < count; ++t) {
            int64_t i = rows ? rows[t] : t;
            int64_t start = row_ptr[i], len = (int64_t)row_ptr[i + 1] - row_ptr[i];
            int lw = log2w ? log2w[i] : oracle_canonical_log2w(len);
            int W = 1 << lw;
            mpv zero = {{0.0, 0.0, 0.0, 0.0}};
            if (len == 0) {
                store_mp(K, y_re, n_rows, i, zero);
                if (cplx) store_mp(K, y_im, n_rows, i, zero);
                continue;
            }
            if (lw > 10 || W > len) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            if (!cplx) {
                store_mp(K, y_re, n_rows, i, row_sum(K, start, len, W, col_idx, a_re, nnz, x_re, n_cols, lanes));
            } else {
                /* Eq. 3 with four accumulator sets, combined at the end of the row */
                mpv rr = row_sum(K, start, len, W, col_idx, a_re, nnz, x_re, n_cols, lanes);
                mpv ii = row_sum(K, start, len, W, col_idx, a_im, nnz, x_im, n_cols, lanes);
                mpv ri = row_sum(K, start, len, W, col_idx, a_re, nnz, x_im, n_cols, lanes);
                mpv ir = row_sum(K, start, len, W, col_idx, a_im, nnz, x_re, n_cols, lanes);
                store_mp(K, y_re, n_rows, i, mp_add(K, rr, mp_neg(ii)));
                store_mp(K, y_im, n_rows, i, mp_add(K, ri, ir));
            }
        }
        free(lanes);
    }
    return bad ? -1 : 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
