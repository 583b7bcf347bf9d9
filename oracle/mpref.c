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
/* Algorithm 4 (QD times binary64), with the garbled steps read after Hida, Li and
 * Bailey's product of a quad-double by a double: the three leading partial products
 * exactly (TwoProd), the fourth plainly (the listing adds x[3] and y where the
 * product is meant); the order-eps terms merged by a TwoSum (the listing prints
 * TwoProd, but errors of sums are summed); the order-eps^2 terms by ThreeSum; the
 * first order-eps^2 error, the second product error and the fourth product by
 * ThreeSum2 (the listing's operand list repeats an already consumed term); the two
 * remaining errors by one plain add; then the 5 -> 4 renormalisation. */
static mpv qd_mul_d(mpv x, double y)
{
    double p0, q0, p1, q1, p2, q2, p3, s1, s2;
    two_prod(x.c[0], y, &p0, &q0);
    two_prod(x.c[1], y, &p1, &q1);
    two_prod(x.c[2], y, &p2, &q2);
    p3 = x.c[3] * y;
    two_sum(q0, p1, &s1, &s2);
    three_sum(s2, q1, p2, &s2, &q1, &p2);
    three_sum2(q1, q2, p3, &q1, &q2);
    return renorm5(p0, s1, s2, q1, q2 + p2);
}

static mpv td_trunc(mpv r) { r.c[3] = 0.0; return r; }

/* Algorithm 5 (TD times binary64): the QD product of the zero-padded value, first
 * three components kept -- TD operations are the QD ones with x[3] = 0 (Sec. 2). */
static mpv td_mul_d(mpv x, double y) { x.c[3] = 0.0; return td_trunc(qd_mul_d(x, y)); }

/* K-component value times a binary64 value (Algs 3-5) */
static mpv mp_mul_d(int K, mpv x, double y)
{
    return K == 2 ? dd_mul_d(x, y) : (K == 3 ? td_mul_d(x, y) : qd_mul_d(x, y));
}
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
/* op: 0 = add, 1 = mul, 2 = mul by binary64 (Algs 3-5; y holds n doubles).     */
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
            out = mp_mul_d(K, a, y[i]);
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

/* One accumulator set with a binary64 matrix: sum_k mul_d(X[col[k]], A[k]) in the
 * lane/fold order of row_sum. */
static mpv row_sum_d(int K, int64_t start, int64_t len, int W, const int32_t *col, const double *A,
                     const double *X, int64_t n, mpv *lanes)
{
    int l, off;
    for (l = 0; l < W; ++l) {
        int64_t k = start + l;
        lanes[l] = mp_mul_d(K, load_mp(K, X, n, col[k]), A[k]);
        for (k = k + W; k < start + len; k += W)
            lanes[l] = mp_add(K, lanes[l], mp_mul_d(K, load_mp(K, X, n, col[k]), A[k]));
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
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel num_threads(nt)
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

/* ------------------------------------------------------------------------- */
/* DD vector kernels and scalars for the Krylov solvers (Sec. 4.2).           */
/* ------------------------------------------------------------------------- */

#define DOT_LANES 256
#define DOT_CHUNK 4096

/* DD comparison a <= b on (leading, trailing) pairs of non-overlapping values. */
static int dd_le(mpv a, mpv b)
{
    return (a.c[0] < b.c[0]) || (a.c[0] == b.c[0] && a.c[1] <= b.c[1]);
}

/* DD division a / b (Dekker's long division): q1 = a0/b0, the remainder
 * a - q1*b formed with TwoProd/TwoSum and the trailing parts, q2 = remainder/b0,
 * result QuickTwoSum(q1, q2). */
static mpv dd_div(mpv a, mpv b)
{
    double q1, p, e, w, s, f, q2;
    mpv r = {{0.0, 0.0, 0.0, 0.0}};
    q1 = a.c[0] / b.c[0];
    two_prod(q1, b.c[0], &p, &e);
    w = q1 * b.c[1];
    e = e + w;
    two_sum(a.c[0], -p, &s, &f);
    f = f - e;
    f = f + a.c[1];
    q2 = (s + f) / b.c[0];
    quick_two_sum(q1, q2, &r.c[0], &r.c[1]);
    return r;
}

/* Dot product order (K-component operations; the same tree for every K): the vector
 * is cut into chunks of 4096 elements; inside a
 * chunk, lane l < 256 accumulates elements l, l+256, ... (the SpMV row order with
 * W = 256), the lanes holding elements are folded acc[l] += acc[l+off], off =
 * 128..1, a lane without elements being skipped; the chunk sums are then combined
 * by a pairwise tree, P[i] = add(P[2i], P[2i+1]) level by level, an unpaired last
 * element passing up unchanged.  n = 0 gives 0. */
static mpv dot_tree(int K, int64_t n, const double *x, const double *y)
{
    int64_t nch = (n + DOT_CHUNK - 1) / DOT_CHUNK, c, m;
    mpv zero = {{0.0, 0.0, 0.0, 0.0}};
    mpv *P, out;
    if (n == 0) return zero;
    P = (mpv *)malloc(sizeof(mpv) * (size_t)nch);
    /* chunks are independent (each thread sums whole chunks in the order above) */
#pragma omp parallel for schedule(static) if (nch >= 8)
    for (c = 0; c < nch; ++c) {
        int64_t base = c * DOT_CHUNK, cnt = n - base < DOT_CHUNK ? n - base : DOT_CHUNK;
        int l, off, used = cnt < DOT_LANES ? (int)cnt : DOT_LANES;
        mpv lanes[DOT_LANES];
        for (l = 0; l < used; ++l) {
            int64_t k = base + l;
            lanes[l] = mp_mul(K, load_mp(K, x, n, k), load_mp(K, y, n, k));
            for (k = k + DOT_LANES; k < base + cnt; k += DOT_LANES)
                lanes[l] = mp_add(K, lanes[l], mp_mul(K, load_mp(K, x, n, k), load_mp(K, y, n, k)));
        }
        for (off = DOT_LANES / 2; off >= 1; off /= 2)
            for (l = 0; l < off; ++l)
                if (l + off < used) lanes[l] = mp_add(K, lanes[l], lanes[l + off]);
        P[c] = lanes[0];
    }
    for (m = nch; m > 1; m = (m + 1) / 2) {
        int64_t i;
        for (i = 0; i < m / 2; ++i) P[i] = mp_add(K, P[2 * i], P[2 * i + 1]);
        if (m % 2) P[m / 2] = P[m - 1];
    }
    out = P[0];
    free(P);
    return out;
}

static mpv dd_dot_vec(int64_t n, const double *x, const double *y) { return dot_tree(2, n, x, y); }

int oracle_dd_dot(int64_t n, const double *x, const double *y, double *out2)
{
    mpv d = dd_dot_vec(n, x, y);
    out2[0] = d.c[0];
    out2[1] = d.c[1];
    return 0;
}

int oracle_dd_div(const double *a2, const double *b2, double *out2)
{
    mpv a = {{a2[0], a2[1], 0.0, 0.0}}, b = {{b2[0], b2[1], 0.0, 0.0}}, r = dd_div(a, b);
    out2[0] = r.c[0];
    out2[1] = r.c[1];
    return 0;
}

/* Krylov result record (matches the solver info of the GPU library). */
typedef struct {
    int32_t status;      /* 0 converged, -5 not converged, -6 breakdown */
    int32_t iters;
    int32_t restarts;    /* true-residual confirmations that failed */
    int32_t reserved;
    double rr_true[2];   /* DD ||b - A x||^2 at exit */
    double bb[2];        /* DD ||b||^2 */
} oracle_solve_info;

typedef struct {
    int64_t n, nnz;
    const int32_t *row_ptr, *col_idx;
    const uint8_t *log2w;
    const double *a;
} dd_mat;

static void dd_spmv(const dd_mat *M, const double *x, double *y)
{
    oracle_spmv(2, M->n, M->n, M->nnz, M->row_ptr, M->col_idx, M->log2w, M->a, NULL, x, NULL, y, NULL,
                0, NULL, 0);
}

static mpv ld2(const double *v, int64_t n, int64_t i) { return load_mp(2, v, n, i); }
static void st2(double *v, int64_t n, int64_t i, mpv x) { store_mp(2, v, n, i, x); }

/* r = b - A x  (q is scratch) */
static void dd_residual(const dd_mat *M, const double *b, const double *x, double *q, double *r)
{
    int64_t i, n = M->n;
    dd_spmv(M, x, q);
#pragma omp parallel for schedule(static) if (n >= 32768)
    for (i = 0; i < n; ++i) st2(r, n, i, dd_add(ld2(b, n, i), mp_neg(ld2(q, n, i))));
}

/* z = M^-1 r: Jacobi (z_i = DDmulD(r_i, minv_i), Alg. 3) or copy when minv is NULL */
static void dd_precond(int64_t n, const double *minv, const double *r, double *z)
{
    int64_t i;
#pragma omp parallel for schedule(static) if (n >= 32768)
    for (i = 0; i < n; ++i) st2(z, n, i, minv ? dd_mul_d(ld2(r, n, i), minv[i]) : ld2(r, n, i));
}

/* Jacobi inverse diagonal: fl(1 / leading component of a_ii) (1 where the row has no
 * diagonal entry). */
int oracle_jacobi_minv(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *a_hi,
                       double *minv)
{
    int64_t i, k;
    for (i = 0; i < n; ++i) {
        minv[i] = 1.0;
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col_idx[k] == i) minv[i] = 1.0 / a_hi[k];
    }
    return 0;
}

/*
 * Preconditioned CG in DD (Hestenes-Stiefel form; x0 given, stop on the recurrence
 * residual ||r_k||^2 <= rtol^2 ||b||^2, confirmed with the true residual b - A x;
 * a failed confirmation restarts from the true residual).
 *   minv: Jacobi inverse diagonal (NULL = no preconditioner).  hist (optional,
 *   2*(max_iter+1) doubles): DD ||r_k||^2 of the recurrence at iteration k.
 */
int oracle_cg(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
              const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
              oracle_solve_info *info, double *hist)
{
    dd_mat M = {n, nnz, row_ptr, col_idx, log2w, a};
    double *r = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    mpv rho, rr, bb, tol2, pq, alpha, beta, rho_new;
    int64_t i;
    int32_t k = 0;
    int status = -5;
    memset(info, 0, sizeof(*info));
    bb = dd_dot_vec(n, b, b);
    tol2 = dd_mul_d(bb, rtol * rtol);
    dd_residual(&M, b, x, q, r);
    dd_precond(n, minv, r, z);
    memcpy(p, z, sizeof(double) * 2 * (size_t)n);
    rho = dd_dot_vec(n, r, z);
    rr = dd_dot_vec(n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (dd_le(rr, tol2)) {
            /* confirm with the true residual */
            dd_residual(&M, b, x, q, r);
            rr = dd_dot_vec(n, r, r);
            if (dd_le(rr, tol2)) { status = 0; break; }
            info->restarts++;
            dd_precond(n, minv, r, z);
            memcpy(p, z, sizeof(double) * 2 * (size_t)n);
            rho = dd_dot_vec(n, r, z);
        }
        if (k >= max_iter) break;
        dd_spmv(&M, p, q);
        pq = dd_dot_vec(n, p, q);
        if (!(pq.c[0] > 0.0) || !isfinite(pq.c[0])) { status = -6; break; }
        alpha = dd_div(rho, pq);
#pragma omp parallel for schedule(static) if (n >= 32768)
        for (i = 0; i < n; ++i) {
            st2(x, n, i, dd_add(ld2(x, n, i), dd_mul(alpha, ld2(p, n, i))));
            st2(r, n, i, dd_add(ld2(r, n, i), mp_neg(dd_mul(alpha, ld2(q, n, i)))));
        }
        dd_precond(n, minv, r, z);
        rho_new = dd_dot_vec(n, r, z);
        rr = dd_dot_vec(n, r, r);
        k++;
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0]) || !isfinite(rho_new.c[0])) { status = -6; break; }
        beta = dd_div(rho_new, rho);
        rho = rho_new;
#pragma omp parallel for schedule(static) if (n >= 32768)
        for (i = 0; i < n; ++i) st2(p, n, i, dd_add(ld2(z, n, i), dd_mul(beta, ld2(p, n, i))));
    }
    /* exit record: the true residual of the returned x */
    dd_residual(&M, b, x, q, r);
    rr = dd_dot_vec(n, r, r);
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(z); free(p); free(q);
    return status;
}

/*
 * BiCGSTAB (van der Vorst) in DD with right preconditioning by minv (NULL = none);
 * shadow residual = the initial residual.  Same stopping rule and restart-on-failed-
 * confirmation as oracle_cg; the convergence test is made on ||s||^2 after the
 * half step and on ||r||^2 after the full step.
 */
int oracle_bicgstab(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                    const double *a, const double *b, double *x, const double *minv, double rtol,
                    int32_t max_iter, oracle_solve_info *info, double *hist)
{
    dd_mat M = {n, nnz, row_ptr, col_idx, log2w, a};
    size_t bytes = sizeof(double) * 2 * (size_t)n;
    double *r = (double *)malloc(bytes), *rh = (double *)malloc(bytes), *p = (double *)malloc(bytes);
    double *v = (double *)malloc(bytes), *ph = (double *)malloc(bytes), *s = (double *)malloc(bytes);
    double *sh = (double *)malloc(bytes), *t = (double *)malloc(bytes), *q = (double *)malloc(bytes);
    mpv one = {{1.0, 0.0, 0.0, 0.0}}, zero = {{0.0, 0.0, 0.0, 0.0}};
    mpv rho_old = one, alpha = one, omega = one, rho, beta, rv, ts, tt, rr, ss, bb, tol2;
    int64_t i;
    int32_t k = 0;
    int status = -5, fresh = 1;
    memset(info, 0, sizeof(*info));
    bb = dd_dot_vec(n, b, b);
    tol2 = dd_mul_d(bb, rtol * rtol);
    dd_residual(&M, b, x, q, r);
    memcpy(rh, r, bytes);
    memset(v, 0, bytes);
    memset(p, 0, bytes);
    rr = dd_dot_vec(n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (dd_le(rr, tol2)) {
            dd_residual(&M, b, x, q, r);
            rr = dd_dot_vec(n, r, r);
            if (dd_le(rr, tol2)) { status = 0; break; }
            info->restarts++;
            memcpy(rh, r, bytes);
            fresh = 1;
        }
        if (k >= max_iter) break;
        rho = dd_dot_vec(n, rh, r);
        if (rho.c[0] == 0.0 || !isfinite(rho.c[0])) { status = -6; break; }
        if (fresh) {
            memcpy(p, r, bytes);
            fresh = 0;
        } else {
            beta = dd_mul(dd_div(rho, rho_old), dd_div(alpha, omega));
            for (i = 0; i < n; ++i) {
                mpv pv = dd_add(ld2(p, n, i), mp_neg(dd_mul(omega, ld2(v, n, i))));
                st2(p, n, i, dd_add(ld2(r, n, i), dd_mul(beta, pv)));
            }
        }
        dd_precond(n, minv, p, ph);
        dd_spmv(&M, ph, v);
        rv = dd_dot_vec(n, rh, v);
        if (rv.c[0] == 0.0 || !isfinite(rv.c[0])) { status = -6; break; }
        alpha = dd_div(rho, rv);
        for (i = 0; i < n; ++i) st2(s, n, i, dd_add(ld2(r, n, i), mp_neg(dd_mul(alpha, ld2(v, n, i)))));
        ss = dd_dot_vec(n, s, s);
        k++;
        if (dd_le(ss, tol2)) {
            for (i = 0; i < n; ++i) st2(x, n, i, dd_add(ld2(x, n, i), dd_mul(alpha, ld2(ph, n, i))));
            memcpy(r, s, bytes);
            rr = ss;
            if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
            rho_old = rho;
            omega = one;
            fresh = 1;
            continue;
        }
        dd_precond(n, minv, s, sh);
        dd_spmv(&M, sh, t);
        ts = dd_dot_vec(n, t, s);
        tt = dd_dot_vec(n, t, t);
        if (tt.c[0] == 0.0 || !isfinite(tt.c[0])) { status = -6; break; }
        omega = dd_div(ts, tt);
        for (i = 0; i < n; ++i) {
            mpv xv = dd_add(ld2(x, n, i), dd_mul(alpha, ld2(ph, n, i)));
            st2(x, n, i, dd_add(xv, dd_mul(omega, ld2(sh, n, i))));
            st2(r, n, i, dd_add(ld2(s, n, i), mp_neg(dd_mul(omega, ld2(t, n, i)))));
        }
        rr = dd_dot_vec(n, r, r);
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0])) { status = -6; break; }
        if (omega.c[0] == 0.0) { status = -6; break; }
        rho_old = rho;
    }
    (void)zero;
    dd_residual(&M, b, x, q, r);
    rr = dd_dot_vec(n, r, r);
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(q);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Mixed-precision iterative refinement (DD residual and update, binary64 or  */
/* binary32 inner Jacobi-PCG on the leading component of A).                   */
/* ------------------------------------------------------------------------- */

/* Inner plain-precision PCG, written once per type.  The preconditioner is z = M r
 * with M given by its values on A's pattern (mv, applied as an SpMV), else
 * z_i = r_i minv_i (Jacobi), else z = r.  SpMV order: each row summed
 * sequentially in element order (first product, then one add per element).  Dot
 * products: the DD dot tree's shape (chunks of 4096, W = 256 lanes, halving fold,
 * pairwise chunk tree) in the inner type.  d starts at 0; stop when ||r||^2 <=
 * inner_rtol^2 ||r0||^2, or at max_iter, or on breakdown (pq <= 0, non-finite). */
#define DEFINE_INNER(T, SUF)                                                                        \
    static T dot_##SUF(int64_t n, const T *x, const T *y)                                          \
    {                                                                                              \
        int64_t nch = (n + DOT_CHUNK - 1) / DOT_CHUNK, c, m;                                       \
        T *P, out;                                                                                 \
        if (n == 0) return (T)0;                                                                   \
        P = (T *)malloc(sizeof(T) * (size_t)nch);                                                  \
        _Pragma("omp parallel for schedule(static) if (nch >= 8)")                                 \
        for (c = 0; c < nch; ++c) {                                                                \
            int64_t base = c * DOT_CHUNK, cnt = n - base < DOT_CHUNK ? n - base : DOT_CHUNK;      \
            int l, off, used = cnt < DOT_LANES ? (int)cnt : DOT_LANES;                             \
            T lanes[DOT_LANES];                                                                    \
            for (l = 0; l < used; ++l) {                                                           \
                int64_t k = base + l;                                                              \
                T prod = x[k] * y[k];                                                              \
                lanes[l] = prod;                                                                   \
                for (k = k + DOT_LANES; k < base + cnt; k += DOT_LANES) {                          \
                    prod = x[k] * y[k];                                                            \
                    lanes[l] = lanes[l] + prod;                                                    \
                }                                                                                  \
            }                                                                                      \
            for (off = DOT_LANES / 2; off >= 1; off /= 2)                                          \
                for (l = 0; l < off; ++l)                                                          \
                    if (l + off < used) lanes[l] = lanes[l] + lanes[l + off];                      \
            P[c] = lanes[0];                                                                       \
        }                                                                                          \
        for (m = nch; m > 1; m = (m + 1) / 2) {                                                    \
            int64_t i;                                                                             \
            for (i = 0; i < m / 2; ++i) P[i] = P[2 * i] + P[2 * i + 1];                            \
            if (m % 2) P[m / 2] = P[m - 1];                                                        \
        }                                                                                          \
        out = P[0];                                                                                \
        free(P);                                                                                   \
        return out;                                                                                \
    }                                                                                              \
    static void spmv_##SUF(int64_t n, const int32_t *rp, const int32_t *ci, const T *a, const T *x, T *y) \
    {                                                                                              \
        int64_t i;                                                                                 \
        _Pragma("omp parallel for schedule(static)")                                               \
        for (i = 0; i < n; ++i) {                                                                  \
            int64_t k;                                                                             \
            T s = (T)0;                                                                            \
            for (k = rp[i]; k < rp[i + 1]; ++k) {                                                  \
                T prod = a[k] * x[ci[k]];                                                          \
                s = (k == rp[i]) ? prod : s + prod;                                                \
            }                                                                                      \
            y[i] = s;                                                                              \
        }                                                                                          \
    }                                                                                              \
    /* returns iterations; *status: 0 converged, -5 limit, -6 breakdown */                        \
    static int inner_pcg_##SUF(int64_t n, const int32_t *rp, const int32_t *ci, const T *a,       \
                               const T *minv, const T *mv, const T *r0, T *d, double inner_rtol,   \
                               int max_iter, int *status)                                          \
    {                                                                                              \
        size_t bytes = sizeof(T) * (size_t)n;                                                      \
        T *r = (T *)malloc(bytes), *z = (T *)malloc(bytes), *p = (T *)malloc(bytes),               \
          *q = (T *)malloc(bytes);                                                                 \
        T rho, rr, rr0, tol, pq, alpha, beta, rho_new;                                             \
        int64_t i;                                                                                 \
        int k = 0;                                                                                 \
        *status = -5;                                                                              \
        for (i = 0; i < n; ++i) {                                                                  \
            d[i] = (T)0;                                                                           \
            r[i] = r0[i];                                                                          \
            z[i] = minv ? r[i] * minv[i] : r[i];                                                   \
        }                                                                                          \
        if (mv) spmv_##SUF(n, rp, ci, mv, r, z);                                                   \
        for (i = 0; i < n; ++i) p[i] = z[i];                                                       \
        rho = dot_##SUF(n, r, z);                                                                  \
        rr0 = dot_##SUF(n, r, r);                                                                  \
        tol = (T)(inner_rtol * inner_rtol) * rr0;                                                  \
        if (rr0 <= tol) *status = 0;                                                               \
        while (*status == -5 && k < max_iter) {                                                    \
            spmv_##SUF(n, rp, ci, a, p, q);                                                        \
            pq = dot_##SUF(n, p, q);                                                               \
            if (!(pq > (T)0) || !isfinite((double)pq)) { *status = -6; break; }                   \
            alpha = rho / pq;                                                                      \
            _Pragma("omp parallel for schedule(static) if (n >= 32768)")                           \
            for (i = 0; i < n; ++i) {                                                              \
                T ap = alpha * p[i], aq = alpha * q[i];                                            \
                d[i] = d[i] + ap;                                                                  \
                r[i] = r[i] - aq;                                                                  \
                z[i] = minv ? r[i] * minv[i] : r[i];                                               \
            }                                                                                      \
            if (mv) spmv_##SUF(n, rp, ci, mv, r, z);                                               \
            rho_new = dot_##SUF(n, r, z);                                                          \
            rr = dot_##SUF(n, r, r);                                                               \
            k++;                                                                                   \
            if (!isfinite((double)rr) || !isfinite((double)rho_new)) { *status = -6; break; }      \
            beta = rho_new / rho;                                                                  \
            rho = rho_new;                                                                         \
            if (rr <= tol) { *status = 0; break; }                                                 \
            _Pragma("omp parallel for schedule(static) if (n >= 32768)")                           \
            for (i = 0; i < n; ++i) {                                                              \
                T bp = beta * p[i];                                                                \
                p[i] = z[i] + bp;                                                                  \
            }                                                                                      \
        }                                                                                          \
        free(r); free(z); free(p); free(q);                                                        \
        return k;                                                                                  \
    }

DEFINE_INNER(double, f64)
DEFINE_INNER(float, f32)

typedef struct {
    int32_t status;
    int32_t iters;        /* inner iterations (+ fallback DD CG iterations) */
    int32_t outer_iters;
    int32_t fell_back;
    double rr_true[2];
    double bb[2];
} oracle_ir_info;

/*
 * Iterative refinement: r = b - A x in DD (DD SpMV in the given order + DD subtract),
 * stop when ||r||^2 <= rtol^2 ||b||^2 (DD); otherwise e = exponent of max|hi(r)|
 * (frexp), inner right-hand side hi(r) * 2^-e rounded to the inner type, inner PCG
 * on hi(A) (binary64) or fl32(hi(A)) (binary32) with Jacobi fl(1/hi(a_ii)) (rounded
 * to binary32 for the binary32 inner), then x_i = DDadd(x_i, (d_i * 2^e, 0)).
 * With mvals (a learned approximate inverse on A's pattern, rounded to binary32 for
 * the binary32 inner) the inner PCG uses z = M r instead of the Jacobi step.
 * Stall: two consecutive outer steps that each fail to reduce ||r||^2 below a quarter
 * of the previous value switch to DD Jacobi-CG from the current x (max_iter
 * iterations); so does reaching max_outer.
 */
int oracle_ir(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
              const double *a, const double *b, double *x, int inner_fp32, int jacobi, const double *mvals,
              double rtol, double inner_rtol, int32_t inner_max_iter, int32_t max_outer, int32_t max_iter,
              oracle_ir_info *info)
{
    dd_mat M = {n, nnz, row_ptr, col_idx, log2w, a};
    size_t vb = sizeof(double) * 2 * (size_t)n;
    double *r = (double *)malloc(vb), *q = (double *)malloc(vb);
    double *minv = (double *)malloc(sizeof(double) * (size_t)n);
    double *r64 = (double *)malloc(sizeof(double) * (size_t)n), *d64 = (double *)malloc(sizeof(double) * (size_t)n);
    float *a32 = NULL, *m32 = NULL, *r32 = NULL, *d32 = NULL, *mv32 = NULL;
    mpv bb, tol2, rr;
    double prev = 0.0, prev2 = 0.0;
    int64_t i, k;
    int outer = 0, stalled = 0, status = -5;
    memset(info, 0, sizeof(*info));
    oracle_jacobi_minv(n, row_ptr, col_idx, a, minv);
    if (inner_fp32) {
        a32 = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
        m32 = (float *)malloc(sizeof(float) * (size_t)n);
        r32 = (float *)malloc(sizeof(float) * (size_t)n);
        d32 = (float *)malloc(sizeof(float) * (size_t)n);
        for (k = 0; k < nnz; ++k) a32[k] = (float)a[k];
        for (i = 0; i < n; ++i) m32[i] = (float)minv[i];
        if (mvals) {
            mv32 = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
            for (k = 0; k < nnz; ++k) mv32[k] = (float)mvals[k];
        }
    }
    bb = dd_dot_vec(n, b, b);
    tol2 = dd_mul_d(bb, rtol * rtol);
    for (;;) {
        double mx = 0.0;
        int e, st, it;
        dd_residual(&M, b, x, q, r);
        rr = dd_dot_vec(n, r, r);
        if (dd_le(rr, tol2)) { status = 0; break; }
        if (!isfinite(rr.c[0])) { status = -6; break; }
        if (outer >= 2 && rr.c[0] > 0.25 * prev && prev > 0.25 * prev2) { stalled = 1; break; }
        if (outer >= max_outer) { stalled = 1; break; }
        prev2 = prev;
        prev = rr.c[0];
        for (i = 0; i < n; ++i) if (fabs(r[i]) > mx) mx = fabs(r[i]);
        (void)frexp(mx, &e);
        if (inner_fp32) {
            for (i = 0; i < n; ++i) r32[i] = (float)ldexp(r[i], -e);
            it = inner_pcg_f32(n, row_ptr, col_idx, a32, (jacobi && !mvals) ? m32 : NULL, mv32, r32, d32, inner_rtol,
                               inner_max_iter, &st);
            for (i = 0; i < n; ++i) d64[i] = (double)d32[i];
        } else {
            for (i = 0; i < n; ++i) r64[i] = ldexp(r[i], -e);
            it = inner_pcg_f64(n, row_ptr, col_idx, a, (jacobi && !mvals) ? minv : NULL, mvals, r64, d64, inner_rtol,
                               inner_max_iter, &st);
        }
        info->iters += it;
        for (i = 0; i < n; ++i) {
            mpv dv = {{ldexp(d64[i], e), 0.0, 0.0, 0.0}};
            st2(x, n, i, dd_add(ld2(x, n, i), dv));
        }
        outer++;
    }
    info->outer_iters = outer;
    if (stalled) {
        oracle_solve_info ci;
        info->fell_back = 1;
        /* a learned inner preconditioner falls back to plain Jacobi DD CG */
        status = oracle_cg(n, nnz, row_ptr, col_idx, log2w, a, b, x, (jacobi || mvals) ? minv : NULL, rtol, max_iter,
                           &ci, NULL);
        info->iters += ci.iters;
    }
    dd_residual(&M, b, x, q, r);
    rr = dd_dot_vec(n, r, r);
    info->status = status;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(q); free(minv); free(r64); free(d64);
    free(a32); free(m32); free(r32); free(d32); free(mv32);
    return status;
}

/*
 * y = A x with a binary64 matrix (one value per element) and a K-component x
 * (the paper's SpMV of binary64 SuiteSparse matrices, Sec. 2 with Algs 3-5): each
 * product is mul_d(x_col, a_k); the summation order is oracle_spmv's.  Real only.
 */
int oracle_spmv_dmat(int K, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr,
                     const int32_t *col_idx, const uint8_t *log2w, const double *a, const double *x, double *y,
                     int64_t nsel, const int64_t *rows, int nthreads)
{
    int64_t t, count = rows ? nsel : n_rows;
    int bad = 0;
    if (K < 2 || K > 4) return -1;
    (void)nnz;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel num_threads(nt)
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
                store_mp(K, y, n_rows, i, zero);
                continue;
            }
            if (lw > 10 || W > len) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            store_mp(K, y, n_rows, i, row_sum_d(K, start, len, W, col_idx, a, x, n_cols, lanes));
        }
        free(lanes);
    }
    return bad ? -1 : 0;
}

/*
 * Complex y = A x with a binary64 complex matrix (a_re, a_im: one value per element)
 * and a K-component complex x: Eq. 3 with four accumulator sets in the summation
 * order of oracle_spmv, each product mul_d(x_col, a_k) (Algs 3-5); y_re = rr - ii,
 * y_im = ri + ir at the end of the row.
 */
int oracle_spmv_dmat_complex(int K, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, const uint8_t *log2w, const double *a_re, const double *a_im,
                             const double *x_re, const double *x_im, double *y_re, double *y_im, int64_t nsel,
                             const int64_t *rows, int nthreads)
{
    int64_t t, count = rows ? nsel : n_rows;
    int bad = 0;
    if (K < 2 || K > 4) return -1;
    (void)nnz;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel num_threads(nt)
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
                store_mp(K, y_im, n_rows, i, zero);
                continue;
            }
            if (lw > 10 || W > len) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            {
                mpv rr = row_sum_d(K, start, len, W, col_idx, a_re, x_re, n_cols, lanes);
                mpv ii = row_sum_d(K, start, len, W, col_idx, a_im, x_im, n_cols, lanes);
                mpv ri = row_sum_d(K, start, len, W, col_idx, a_re, x_im, n_cols, lanes);
                mpv ir = row_sum_d(K, start, len, W, col_idx, a_im, x_re, n_cols, lanes);
                store_mp(K, y_re, n_rows, i, mp_add(K, rr, mp_neg(ii)));
                store_mp(K, y_im, n_rows, i, mp_add(K, ri, ir));
            }
        }
        free(lanes);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Transpose (for A^T v, Sec. 3): a stable counting sort by column, so row j   */
/* of A^T holds column j of A in increasing row order.  a: ncomp planar value  */
/* arrays of nnz (permuted together with the pattern).                         */
/* ------------------------------------------------------------------------- */
int oracle_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz, int ncomp, const int32_t *row_ptr,
                     const int32_t *col_idx, const double *a, int32_t *row_ptr_t, int32_t *col_idx_t, double *a_t)
{
    int64_t i, k, j;
    int c;
    int64_t *next = (int64_t *)calloc((size_t)n_cols + 1, sizeof(int64_t));
    if (!next) return -1;
    for (k = 0; k < nnz; ++k) next[col_idx[k] + 1]++;
    for (j = 0; j < n_cols; ++j) next[j + 1] += next[j];
    for (j = 0; j <= n_cols; ++j) row_ptr_t[j] = (int32_t)next[j];
    for (i = 0; i < n_rows; ++i)
        for (k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t dst = next[col_idx[k]]++;
            col_idx_t[dst] = (int32_t)i;
            for (c = 0; c < ncomp; ++c) a_t[(int64_t)c * nnz + dst] = a[(int64_t)c * nnz + k];
        }
    free(next);
    return 0;
}




/* ------------------------------------------------------------------------- */
/* COO -> CSR (the storage conversion of Sec. 3): elements ordered by row, and */
/* within a row by column; elements with the same (row, column) keep their    */
/* input order (two stable counting sorts: by column, then by row).  Returns  */
/* -2 when a coordinate is outside the matrix.  v: ncomp planar arrays of nnz. */
/* ------------------------------------------------------------------------- */
int oracle_coo_to_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row, const int32_t *col, int ncomp,
                      const double *v, int32_t *row_ptr, int32_t *col_idx, double *a)
{
    int64_t k, j;
    int c;
    int64_t *cnt, *by_col;
    for (k = 0; k < nnz; ++k)
        if (row[k] < 0 || row[k] >= n_rows || col[k] < 0 || col[k] >= n_cols) return -2;
    cnt = (int64_t *)calloc((size_t)(n_cols > n_rows ? n_cols : n_rows) + 1, sizeof(int64_t));
    by_col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!cnt || !by_col) { free(cnt); free(by_col); return -1; }
    /* pass 1: stable order by column */
    for (k = 0; k < nnz; ++k) cnt[col[k] + 1]++;
    for (j = 0; j < n_cols; ++j) cnt[j + 1] += cnt[j];
    for (k = 0; k < nnz; ++k) by_col[cnt[col[k]]++] = k;
    /* pass 2: stable order by row of the column-ordered sequence */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)(n_cols > n_rows ? n_cols : n_rows) + 1));
    for (k = 0; k < nnz; ++k) cnt[row[k] + 1]++;
    for (j = 0; j < n_rows; ++j) cnt[j + 1] += cnt[j];
    for (j = 0; j <= n_rows; ++j) row_ptr[j] = (int32_t)cnt[j];
    for (k = 0; k < nnz; ++k) {
        int64_t src = by_col[k], dst = cnt[row[src]]++;
        col_idx[dst] = col[src];
        for (c = 0; c < ncomp; ++c) a[(int64_t)c * nnz + dst] = v[(int64_t)c * nnz + src];
    }
    free(cnt);
    free(by_col);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* K-component Krylov layer (TD and QD solvers; K = 2 reproduces the DD one).  */
/* ------------------------------------------------------------------------- */

/* a <= b by lexicographic comparison of the components (both normalised): the first
 * component that differs decides, and a comparison that is not an equality (greater,
 * or a NaN) is false; for K = 2 this is dd_le. */
static int mp_le(int K, mpv a, mpv b)
{
    int c;
    for (c = 0; c < K; ++c) {
        if (a.c[c] < b.c[c]) return 1;
        if (!(a.c[c] == b.c[c])) return 0;
    }
    return 1;
}

/* K-component division a / b.  DD: Dekker's division (dd_div).  TD / QD: long
 * division after Hida, Li and Bailey's quad-double division, written with the
 * K-component operations: q0 = a0 / b0; three times r = r - b * q_i (a K-component
 * times binary64 product and a K-component addition, starting from r = a) and
 * q_{i+1} = r0 / b0; the quotient is the renormalisation of (q0, q1, q2, q3) (Renorm
 * 5 -> 4 with a zero fifth term), truncated to three components for TD. */
static mpv mp_div(int K, mpv a, mpv b)
{
    double q[4];
    mpv r, out;
    int i;
    if (K == 2) return dd_div(a, b);
    r = a;
    for (i = 0; i < 4; ++i) {
        q[i] = r.c[0] / b.c[0];
        if (i < 3) r = mp_add(K, r, mp_neg(mp_mul_d(K, b, q[i])));
    }
    out = renorm5(q[0], q[1], q[2], q[3], 0.0);
    return K == 3 ? td_trunc(out) : out;
}

/* The dot product tree of dd_dot_vec (one function for every K). */
static mpv mp_dot_vec(int K, int64_t n, const double *x, const double *y) { return dot_tree(K, n, x, y); }

int oracle_mp_div(int K, const double *a, const double *b, double *out)
{
    mpv x = {{0.0, 0.0, 0.0, 0.0}}, y = {{0.0, 0.0, 0.0, 0.0}}, r;
    int c;
    for (c = 0; c < K; ++c) { x.c[c] = a[c]; y.c[c] = b[c]; }
    r = mp_div(K, x, y);
    for (c = 0; c < K; ++c) out[c] = r.c[c];
    return 0;
}

int oracle_mp_dot(int K, int64_t n, const double *x, const double *y, double *out)
{
    mpv d = mp_dot_vec(K, n, x, y);
    int c;
    for (c = 0; c < K; ++c) out[c] = d.c[c];
    return 0;
}

typedef struct {
    int K;
    int64_t n, nnz;
    const int32_t *row_ptr, *col_idx;
    const uint8_t *log2w;
    const double *a;
} mp_mat;

static void mpm_spmv(const mp_mat *M, const double *x, double *y)
{
    oracle_spmv(M->K, M->n, M->n, M->nnz, M->row_ptr, M->col_idx, M->log2w, M->a, NULL, x, NULL, y, NULL,
                0, NULL, 0);
}

static mpv ldk(const mp_mat *M, const double *v, int64_t i) { return load_mp(M->K, v, M->n, i); }
static void stk(const mp_mat *M, double *v, int64_t i, mpv x) { store_mp(M->K, v, M->n, i, x); }

static void mpm_residual(const mp_mat *M, const double *b, const double *x, double *q, double *r)
{
    int64_t i;
    mpm_spmv(M, x, q);
#pragma omp parallel for schedule(static) if (M->n >= 32768)
    for (i = 0; i < M->n; ++i) stk(M, r, i, mp_add(M->K, ldk(M, b, i), mp_neg(ldk(M, q, i))));
}

static void mpm_precond(const mp_mat *M, const double *minv, const double *r, double *z)
{
    int64_t i;
#pragma omp parallel for schedule(static) if (M->n >= 32768)
    for (i = 0; i < M->n; ++i) stk(M, z, i, minv ? mp_mul_d(M->K, ldk(M, r, i), minv[i]) : ldk(M, r, i));
}

static void mpm_info(const mp_mat *M, oracle_solve_info *info, int status, int32_t k, mpv rr, mpv bb)
{
    (void)M;
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
}

/*
 * Preconditioned CG in K-component arithmetic: the steps, stopping rule, confirmation
 * and restarts of oracle_cg with mp_add / mp_mul / mp_mul_d / mp_div / mp_dot_vec /
 * mp_le for K components (vectors K * n, planar).  For K = 2 it is oracle_cg.  The
 * info record carries the two leading components of rr_true and bb.
 */
int oracle_cg_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                oracle_solve_info *info, double *hist)
{
    mp_mat M = {K, n, nnz, row_ptr, col_idx, log2w, a};
    size_t vb = sizeof(double) * (size_t)K * (size_t)n;
    double *r = (double *)malloc(vb), *z = (double *)malloc(vb), *p = (double *)malloc(vb), *q = (double *)malloc(vb);
    mpv rho, rr, bb, tol2, pq, alpha, beta, rho_new;
    int64_t i;
    int32_t k = 0;
    int status = -5;
    memset(info, 0, sizeof(*info));
    bb = mp_dot_vec(K, n, b, b);
    tol2 = mp_mul_d(K, bb, rtol * rtol);
    mpm_residual(&M, b, x, q, r);
    mpm_precond(&M, minv, r, z);
    memcpy(p, z, vb);
    rho = mp_dot_vec(K, n, r, z);
    rr = mp_dot_vec(K, n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (mp_le(K, rr, tol2)) {
            mpm_residual(&M, b, x, q, r);
            rr = mp_dot_vec(K, n, r, r);
            if (mp_le(K, rr, tol2)) { status = 0; break; }
            info->restarts++;
            mpm_precond(&M, minv, r, z);
            memcpy(p, z, vb);
            rho = mp_dot_vec(K, n, r, z);
        }
        if (k >= max_iter) break;
        mpm_spmv(&M, p, q);
        pq = mp_dot_vec(K, n, p, q);
        if (!(pq.c[0] > 0.0) || !isfinite(pq.c[0])) { status = -6; break; }
        alpha = mp_div(K, rho, pq);
#pragma omp parallel for schedule(static) if (n >= 32768)
        for (i = 0; i < n; ++i) {
            stk(&M, x, i, mp_add(K, ldk(&M, x, i), mp_mul(K, alpha, ldk(&M, p, i))));
            stk(&M, r, i, mp_add(K, ldk(&M, r, i), mp_neg(mp_mul(K, alpha, ldk(&M, q, i)))));
        }
        mpm_precond(&M, minv, r, z);
        rho_new = mp_dot_vec(K, n, r, z);
        rr = mp_dot_vec(K, n, r, r);
        k++;
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0]) || !isfinite(rho_new.c[0])) { status = -6; break; }
        beta = mp_div(K, rho_new, rho);
        rho = rho_new;
#pragma omp parallel for schedule(static) if (n >= 32768)
        for (i = 0; i < n; ++i) stk(&M, p, i, mp_add(K, ldk(&M, z, i), mp_mul(K, beta, ldk(&M, p, i))));
    }
    mpm_residual(&M, b, x, q, r);
    rr = mp_dot_vec(K, n, r, r);
    mpm_info(&M, info, status, k, rr, bb);
    free(r); free(z); free(p); free(q);
    return status;
}

/*
 * BiCGSTAB in K-component arithmetic: the steps of oracle_bicgstab (right Jacobi
 * preconditioning, shadow r0, half-step test on (s, s), restarts) with K-component
 * operations.  For K = 2 it is oracle_bicgstab.
 */
int oracle_bicgstab_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      const uint8_t *log2w, const double *a, const double *b, double *x, const double *minv,
                      double rtol, int32_t max_iter, oracle_solve_info *info, double *hist)
{
    mp_mat M = {K, n, nnz, row_ptr, col_idx, log2w, a};
    size_t vb = sizeof(double) * (size_t)K * (size_t)n;
    double *r = (double *)malloc(vb), *rh = (double *)malloc(vb), *p = (double *)malloc(vb);
    double *v = (double *)malloc(vb), *ph = (double *)malloc(vb), *s = (double *)malloc(vb);
    double *sh = (double *)malloc(vb), *t = (double *)malloc(vb), *q = (double *)malloc(vb);
    mpv one = {{1.0, 0.0, 0.0, 0.0}};
    mpv rho_old = one, alpha = one, omega = one, rho, beta, rv, ts, tt, rr, ss, bb, tol2;
    int64_t i;
    int32_t k = 0;
    int status = -5, fresh = 1;
    memset(info, 0, sizeof(*info));
    bb = mp_dot_vec(K, n, b, b);
    tol2 = mp_mul_d(K, bb, rtol * rtol);
    mpm_residual(&M, b, x, q, r);
    memcpy(rh, r, vb);
    memset(v, 0, vb);
    memset(p, 0, vb);
    rr = mp_dot_vec(K, n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (mp_le(K, rr, tol2)) {
            mpm_residual(&M, b, x, q, r);
            rr = mp_dot_vec(K, n, r, r);
            if (mp_le(K, rr, tol2)) { status = 0; break; }
            info->restarts++;
            memcpy(rh, r, vb);
            fresh = 1;
        }
        if (k >= max_iter) break;
        rho = mp_dot_vec(K, n, rh, r);
        if (rho.c[0] == 0.0 || !isfinite(rho.c[0])) { status = -6; break; }
        if (fresh) {
            memcpy(p, r, vb);
            fresh = 0;
        } else {
            beta = mp_mul(K, mp_div(K, rho, rho_old), mp_div(K, alpha, omega));
            for (i = 0; i < n; ++i) {
                mpv pv = mp_add(K, ldk(&M, p, i), mp_neg(mp_mul(K, omega, ldk(&M, v, i))));
                stk(&M, p, i, mp_add(K, ldk(&M, r, i), mp_mul(K, beta, pv)));
            }
        }
        mpm_precond(&M, minv, p, ph);
        mpm_spmv(&M, ph, v);
        rv = mp_dot_vec(K, n, rh, v);
        if (rv.c[0] == 0.0 || !isfinite(rv.c[0])) { status = -6; break; }
        alpha = mp_div(K, rho, rv);
        for (i = 0; i < n; ++i) stk(&M, s, i, mp_add(K, ldk(&M, r, i), mp_neg(mp_mul(K, alpha, ldk(&M, v, i)))));
        ss = mp_dot_vec(K, n, s, s);
        k++;
        if (mp_le(K, ss, tol2)) {
            for (i = 0; i < n; ++i) stk(&M, x, i, mp_add(K, ldk(&M, x, i), mp_mul(K, alpha, ldk(&M, ph, i))));
            memcpy(r, s, vb);
            rr = ss;
            if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
            rho_old = rho;
            omega = one;
            fresh = 1;
            continue;
        }
        mpm_precond(&M, minv, s, sh);
        mpm_spmv(&M, sh, t);
        ts = mp_dot_vec(K, n, t, s);
        tt = mp_dot_vec(K, n, t, t);
        if (tt.c[0] == 0.0 || !isfinite(tt.c[0])) { status = -6; break; }
        omega = mp_div(K, ts, tt);
        for (i = 0; i < n; ++i) {
            mpv xv = mp_add(K, ldk(&M, x, i), mp_mul(K, alpha, ldk(&M, ph, i)));
            stk(&M, x, i, mp_add(K, xv, mp_mul(K, omega, ldk(&M, sh, i))));
            stk(&M, r, i, mp_add(K, ldk(&M, s, i), mp_neg(mp_mul(K, omega, ldk(&M, t, i)))));
        }
        rr = mp_dot_vec(K, n, r, r);
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0])) { status = -6; break; }
        if (omega.c[0] == 0.0) { status = -6; break; }
        rho_old = rho;
    }
    mpm_residual(&M, b, x, q, r);
    rr = mp_dot_vec(K, n, r, r);
    mpm_info(&M, info, status, k, rr, bb);
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(q);
    return status;
}

int oracle_mp_le(int K, const double *a, const double *b)
{
    mpv x = {{0.0, 0.0, 0.0, 0.0}}, y = {{0.0, 0.0, 0.0, 0.0}};
    int c;
    for (c = 0; c < K; ++c) { x.c[c] = a[c]; y.c[c] = b[c]; }
    return mp_le(K, x, y);
}

/*
 * Preconditioned BiCG in K-component arithmetic (DD: K = 2) (Fletcher's biconjugate gradients, Sec. 4.2's list of
 * Krylov methods), Jacobi preconditioning (symmetric, so the shadow system uses the
 * same M).  A^T is given explicitly (row_ptr_t, col_idx_t, a_t: the stable transpose,
 * log2w_t its lane widths).  r~ = r at the start; per step q = A p, q~ = A^T p~,
 * sigma = (p~, q), alpha = rho / sigma, x += alpha p, r -= alpha q, r~ -= alpha q~,
 * z = M r, z~ = M r~, rho' = (r~, z), beta = rho' / rho, p = z + beta p,
 * p~ = z~ + beta p~.  Stop test, confirmation and restart as oracle_cg (a restart
 * also resets r~ to the true residual).  Breakdown: sigma = 0 or non-finite, rho' = 0
 * while not converged, or a non-finite rho' or ||r||^2.
 */
int oracle_bicg_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                const double *a, const int32_t *row_ptr_t, const int32_t *col_idx_t, const uint8_t *log2w_t,
                const double *a_t, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                oracle_solve_info *info, double *hist)
{
    mp_mat M = {K, n, nnz, row_ptr, col_idx, log2w, a};
    mp_mat Mt = {K, n, nnz, row_ptr_t, col_idx_t, log2w_t, a_t};
    size_t vb = sizeof(double) * (size_t)K * (size_t)n;
    double *r = (double *)malloc(vb), *z = (double *)malloc(vb), *p = (double *)malloc(vb), *q = (double *)malloc(vb);
    double *rt = (double *)malloc(vb), *zt = (double *)malloc(vb), *pt = (double *)malloc(vb);
    double *qt = (double *)malloc(vb);
    mpv rho, rr, bb, tol2, sigma, alpha, beta, rho_new;
    int64_t i;
    int32_t k = 0;
    int status = -5;
    memset(info, 0, sizeof(*info));
    bb = mp_dot_vec(K, n, b, b);
    tol2 = mp_mul_d(K, bb, rtol * rtol);
    mpm_residual(&M, b, x, q, r);
    memcpy(rt, r, vb);
    mpm_precond(&M, minv, r, z);
    memcpy(zt, z, vb);
    memcpy(p, z, vb);
    memcpy(pt, z, vb);
    rho = mp_dot_vec(K, n, rt, z);
    rr = mp_dot_vec(K, n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (mp_le(K, rr, tol2)) {
            mpm_residual(&M, b, x, q, r);
            rr = mp_dot_vec(K, n, r, r);
            if (mp_le(K, rr, tol2)) { status = 0; break; }
            info->restarts++;
            memcpy(rt, r, vb);
            mpm_precond(&M, minv, r, z);
            memcpy(zt, z, vb);
            memcpy(p, z, vb);
            memcpy(pt, z, vb);
            rho = mp_dot_vec(K, n, rt, z);
        }
        if (k >= max_iter) break;
        mpm_spmv(&M, p, q);
        mpm_spmv(&Mt, pt, qt);
        sigma = mp_dot_vec(K, n, pt, q);
        if (sigma.c[0] == 0.0 || !isfinite(sigma.c[0])) { status = -6; break; }
        alpha = mp_div(K, rho, sigma);
        for (i = 0; i < n; ++i) {
            stk(&M, x, i, mp_add(K, ldk(&M, x, i), mp_mul(K, alpha, ldk(&M, p, i))));
            stk(&M, r, i, mp_add(K, ldk(&M, r, i), mp_neg(mp_mul(K, alpha, ldk(&M, q, i)))));
            stk(&M, rt, i, mp_add(K, ldk(&M, rt, i), mp_neg(mp_mul(K, alpha, ldk(&M, qt, i)))));
        }
        mpm_precond(&M, minv, r, z);
        mpm_precond(&M, minv, rt, zt);
        rho_new = mp_dot_vec(K, n, rt, z);
        rr = mp_dot_vec(K, n, r, r);
        k++;
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0]) || !isfinite(rho_new.c[0])) { status = -6; break; }
        if (rho_new.c[0] == 0.0 && !mp_le(K, rr, tol2)) { status = -6; break; }
        beta = mp_div(K, rho_new, rho);
        rho = rho_new;
        for (i = 0; i < n; ++i) {
            stk(&M, p, i, mp_add(K, ldk(&M, z, i), mp_mul(K, beta, ldk(&M, p, i))));
            stk(&M, pt, i, mp_add(K, ldk(&M, zt, i), mp_mul(K, beta, ldk(&M, pt, i))));
        }
    }
    mpm_residual(&M, b, x, q, r);
    rr = mp_dot_vec(K, n, r, r);
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(z); free(p); free(q); free(rt); free(zt); free(pt); free(qt);
    return status;
}

int oracle_bicg(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                const double *a, const int32_t *row_ptr_t, const int32_t *col_idx_t, const uint8_t *log2w_t,
                const double *a_t, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                oracle_solve_info *info, double *hist)
{
    return oracle_bicg_k(2, n, nnz, row_ptr, col_idx, log2w, a, row_ptr_t, col_idx_t, log2w_t, a_t, b, x, minv, rtol,
                         max_iter, info, hist);
}

/*
 * CGS in K-component arithmetic (DD: K = 2) (Sonneveld's conjugate gradient squared, Sec. 4.2's list), with right
 * Jacobi preconditioning as oracle_bicgstab (solve A M y = b, x = M y, so r stays
 * the true recurrence residual of A x = b).  Shadow r~ = r at the start and after
 * each restart.  Step: rho = (r~, r) (breakdown when 0 or not finite); the first
 * step after a (re)start takes u = p = r, later steps beta = rho / rho_old,
 * u = r + beta q, p = u + beta (q + beta p); p^ = M p, v = A p^, sigma = (r~, v)
 * (breakdown when 0 or not finite), alpha = rho / sigma, q = u - alpha v,
 * u^ = M (u + q), x += alpha u^, r -= alpha A u^.  Stop test, confirmation and
 * restarts as oracle_cg.
 */
int oracle_cgs_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
               const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
               oracle_solve_info *info, double *hist)
{
    mp_mat M = {K, n, nnz, row_ptr, col_idx, log2w, a};
    size_t vb = sizeof(double) * (size_t)K * (size_t)n;
    double *r = (double *)malloc(vb), *rh = (double *)malloc(vb), *u = (double *)malloc(vb), *p = (double *)malloc(vb);
    double *q = (double *)malloc(vb), *v = (double *)malloc(vb), *uh = (double *)malloc(vb), *t = (double *)malloc(vb);
    double *ph = (double *)malloc(vb);
    mpv rho, rho_old = {{1.0, 0.0, 0.0, 0.0}}, beta, sigma, alpha, rr, bb, tol2;
    int64_t i;
    int32_t k = 0;
    int status = -5, fresh = 1;
    memset(info, 0, sizeof(*info));
    bb = mp_dot_vec(K, n, b, b);
    tol2 = mp_mul_d(K, bb, rtol * rtol);
    mpm_residual(&M, b, x, t, r);
    memcpy(rh, r, vb);
    memset(q, 0, vb);
    memset(p, 0, vb);
    rr = mp_dot_vec(K, n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (mp_le(K, rr, tol2)) {
            mpm_residual(&M, b, x, t, r);
            rr = mp_dot_vec(K, n, r, r);
            if (mp_le(K, rr, tol2)) { status = 0; break; }
            info->restarts++;
            memcpy(rh, r, vb);
            fresh = 1;
        }
        if (k >= max_iter) break;
        rho = mp_dot_vec(K, n, rh, r);
        if (rho.c[0] == 0.0 || !isfinite(rho.c[0])) { status = -6; break; }
        if (fresh) {
            memcpy(u, r, vb);
            memcpy(p, r, vb);
            fresh = 0;
        } else {
            beta = mp_div(K, rho, rho_old);
            for (i = 0; i < n; ++i) {
                mpv ui = mp_add(K, ldk(&M, r, i), mp_mul(K, beta, ldk(&M, q, i)));
                mpv w = mp_add(K, ldk(&M, q, i), mp_mul(K, beta, ldk(&M, p, i)));
                stk(&M, u, i, ui);
                stk(&M, p, i, mp_add(K, ui, mp_mul(K, beta, w)));
            }
        }
        mpm_precond(&M, minv, p, ph);
        mpm_spmv(&M, ph, v);
        sigma = mp_dot_vec(K, n, rh, v);
        if (sigma.c[0] == 0.0 || !isfinite(sigma.c[0])) { status = -6; break; }
        alpha = mp_div(K, rho, sigma);
        for (i = 0; i < n; ++i) {
            mpv qi = mp_add(K, ldk(&M, u, i), mp_neg(mp_mul(K, alpha, ldk(&M, v, i))));
            mpv s = mp_add(K, ldk(&M, u, i), qi);
            stk(&M, q, i, qi);
            stk(&M, uh, i, minv ? mp_mul_d(K, s, minv[i]) : s);
        }
        for (i = 0; i < n; ++i) stk(&M, x, i, mp_add(K, ldk(&M, x, i), mp_mul(K, alpha, ldk(&M, uh, i))));
        mpm_spmv(&M, uh, t);
        for (i = 0; i < n; ++i) stk(&M, r, i, mp_add(K, ldk(&M, r, i), mp_neg(mp_mul(K, alpha, ldk(&M, t, i)))));
        rr = mp_dot_vec(K, n, r, r);
        k++;
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0])) { status = -6; break; }
        rho_old = rho;
    }
    mpm_residual(&M, b, x, t, r);
    rr = mp_dot_vec(K, n, r, r);
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(rh); free(u); free(p); free(q); free(v); free(uh); free(t); free(ph);
    return status;
}

int oracle_cgs(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
               const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
               oracle_solve_info *info, double *hist)
{
    return oracle_cgs_k(2, n, nnz, row_ptr, col_idx, log2w, a, b, x, minv, rtol, max_iter, info, hist);
}

/*
 * GPBiCG in K-component arithmetic (DD: K = 2) (Zhang's generalized product-type BiCG, Sec. 4.2's list), with right
 * Jacobi preconditioning as oracle_bicgstab: every product with A is a product with
 * A M, and x collects M times the y-space corrections.  Shadow r~ = r at the start and
 * after each restart.  One step:
 *   rho = (r~, r) (breakdown when 0 or not finite);
 *   first step after a (re)start: p = r; later steps: beta = (alpha'/zeta')(rho/rho'),
 *     p = r + beta (p - u), w = c' + beta q'  (primes: the previous step's values);
 *   q = A M p; sigma = (r~, q) (breakdown when 0 or not finite); alpha = rho / sigma;
 *   t = r - alpha q; later steps y = t' - t - alpha w;
 *   half step: when (t, t) meets the tolerance, x += M (alpha p), r = t, and the
 *     next step starts fresh (as BiCGSTAB's s test);
 *   c = A M t;
 *   first step: zeta = (c, t) / (c, c), eta = 0 (breakdown when (c, c) is 0);
 *   later steps, with d = (c,c)(y,y) - (y,c)^2 (breakdown when 0):
 *     zeta = ((y,y)(c,t) - (y,t)(y,c)) / d,  eta = ((c,c)(y,t) - (y,c)(c,t)) / d;
 *   breakdown when zeta is 0 or zeta / eta are not finite;
 *   u = zeta q + eta (t' - r + beta u)       [first step: u = zeta q]
 *   z = zeta r + eta z - alpha u             [first step: z = zeta r - alpha u]
 *   x += M (alpha p + z)
 *   r = t - eta y - zeta c                   [first step: r = t - zeta c]
 *   t' = t.
 * Stop test, confirmation and restarts as oracle_cg; a step is counted when t is formed.
 */
int oracle_gpbicg_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                  const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                  oracle_solve_info *info, double *hist)
{
    mp_mat M = {K, n, nnz, row_ptr, col_idx, log2w, a};
    size_t vb = sizeof(double) * (size_t)K * (size_t)n;
    double *r = (double *)malloc(vb), *rh = (double *)malloc(vb), *p = (double *)malloc(vb);
    double *q = (double *)malloc(vb), *t = (double *)malloc(vb), *c = (double *)malloc(vb);
    double *y = (double *)malloc(vb), *u = (double *)malloc(vb), *z = (double *)malloc(vb);
    double *w = (double *)malloc(vb), *tp = (double *)malloc(vb), *tmp = (double *)malloc(vb);
    mpv zero = {{0.0, 0.0, 0.0, 0.0}};
    mpv rho, rho_old = zero, beta = zero, sigma, alpha = zero, zeta = zero, eta = zero;
    mpv rr, tt, cc, ct, yy, yc, yt, den, bb, tol2;
    int64_t i;
    int32_t k = 0;
    int status = -5, fresh = 1;
    memset(info, 0, sizeof(*info));
    bb = mp_dot_vec(K, n, b, b);
    tol2 = mp_mul_d(K, bb, rtol * rtol);
    mpm_residual(&M, b, x, tmp, r);
    memcpy(rh, r, vb);
    rr = mp_dot_vec(K, n, r, r);
    if (hist) { hist[0] = rr.c[0]; hist[1] = rr.c[1]; }
    for (;;) {
        if (mp_le(K, rr, tol2)) {
            mpm_residual(&M, b, x, tmp, r);
            rr = mp_dot_vec(K, n, r, r);
            if (mp_le(K, rr, tol2)) { status = 0; break; }
            info->restarts++;
            memcpy(rh, r, vb);
            fresh = 1;
        }
        if (k >= max_iter) break;
        rho = mp_dot_vec(K, n, rh, r);
        if (rho.c[0] == 0.0 || !isfinite(rho.c[0])) { status = -6; break; }
        if (fresh) {
            memcpy(p, r, vb);
        } else {
            beta = mp_mul(K, mp_div(K, alpha, zeta), mp_div(K, rho, rho_old));
            for (i = 0; i < n; ++i) {
                mpv pu = mp_add(K, ldk(&M, p, i), mp_neg(ldk(&M, u, i)));
                stk(&M, p, i, mp_add(K, ldk(&M, r, i), mp_mul(K, beta, pu)));
                stk(&M, w, i, mp_add(K, ldk(&M, c, i), mp_mul(K, beta, ldk(&M, q, i))));
            }
        }
        mpm_precond(&M, minv, p, tmp);
        mpm_spmv(&M, tmp, q);
        sigma = mp_dot_vec(K, n, rh, q);
        if (sigma.c[0] == 0.0 || !isfinite(sigma.c[0])) { status = -6; break; }
        alpha = mp_div(K, rho, sigma);
        for (i = 0; i < n; ++i) {
            mpv ti = mp_add(K, ldk(&M, r, i), mp_neg(mp_mul(K, alpha, ldk(&M, q, i))));
            stk(&M, t, i, ti);
            if (!fresh) {
                mpv d = mp_add(K, ldk(&M, tp, i), mp_neg(ti));
                stk(&M, y, i, mp_add(K, d, mp_neg(mp_mul(K, alpha, ldk(&M, w, i)))));
            }
        }
        tt = mp_dot_vec(K, n, t, t);
        k++;
        if (mp_le(K, tt, tol2)) {
            for (i = 0; i < n; ++i) {
                mpv d = mp_mul(K, alpha, ldk(&M, p, i));
                stk(&M, x, i, mp_add(K, ldk(&M, x, i), minv ? mp_mul_d(K, d, minv[i]) : d));
            }
            memcpy(r, t, vb);
            rr = tt;
            if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
            rho_old = rho;
            fresh = 1;
            continue;
        }
        mpm_precond(&M, minv, t, tmp);
        mpm_spmv(&M, tmp, c);
        cc = mp_dot_vec(K, n, c, c);
        ct = mp_dot_vec(K, n, c, t);
        if (fresh) {
            if (cc.c[0] == 0.0 || !isfinite(cc.c[0])) { status = -6; break; }
            zeta = mp_div(K, ct, cc);
            eta = zero;
        } else {
            yy = mp_dot_vec(K, n, y, y);
            yc = mp_dot_vec(K, n, y, c);
            yt = mp_dot_vec(K, n, y, t);
            den = mp_add(K, mp_mul(K, cc, yy), mp_neg(mp_mul(K, yc, yc)));
            if (den.c[0] == 0.0 || !isfinite(den.c[0])) { status = -6; break; }
            zeta = mp_div(K, mp_add(K, mp_mul(K, yy, ct), mp_neg(mp_mul(K, yt, yc))), den);
            eta = mp_div(K, mp_add(K, mp_mul(K, cc, yt), mp_neg(mp_mul(K, yc, ct))), den);
        }
        if (zeta.c[0] == 0.0 || !isfinite(zeta.c[0]) || !isfinite(eta.c[0])) { status = -6; break; }
        for (i = 0; i < n; ++i) {
            mpv ri = ldk(&M, r, i), ti = ldk(&M, t, i), ui, zi, d;
            if (fresh) {
                ui = mp_mul(K, zeta, ldk(&M, q, i));
                zi = mp_add(K, mp_mul(K, zeta, ri), mp_neg(mp_mul(K, alpha, ui)));
            } else {
                mpv g = mp_add(K, mp_add(K, ldk(&M, tp, i), mp_neg(ri)), mp_mul(K, beta, ldk(&M, u, i)));
                ui = mp_add(K, mp_mul(K, zeta, ldk(&M, q, i)), mp_mul(K, eta, g));
                mpv zr = mp_add(K, mp_mul(K, zeta, ri), mp_mul(K, eta, ldk(&M, z, i)));
                zi = mp_add(K, zr, mp_neg(mp_mul(K, alpha, ui)));
            }
            stk(&M, u, i, ui);
            stk(&M, z, i, zi);
            d = mp_add(K, mp_mul(K, alpha, ldk(&M, p, i)), zi);
            stk(&M, x, i, mp_add(K, ldk(&M, x, i), minv ? mp_mul_d(K, d, minv[i]) : d));
            if (fresh)
                ri = mp_add(K, ti, mp_neg(mp_mul(K, zeta, ldk(&M, c, i))));
            else {
                mpv ty = mp_add(K, ti, mp_neg(mp_mul(K, eta, ldk(&M, y, i))));
                ri = mp_add(K, ty, mp_neg(mp_mul(K, zeta, ldk(&M, c, i))));
            }
            stk(&M, r, i, ri);
            stk(&M, tp, i, ti);
        }
        rr = mp_dot_vec(K, n, r, r);
        if (hist) { hist[2 * k] = rr.c[0]; hist[2 * k + 1] = rr.c[1]; }
        if (!isfinite(rr.c[0])) { status = -6; break; }
        rho_old = rho;
        fresh = 0;
    }
    mpm_residual(&M, b, x, tmp, r);
    rr = mp_dot_vec(K, n, r, r);
    info->status = status;
    info->iters = k;
    info->rr_true[0] = rr.c[0]; info->rr_true[1] = rr.c[1];
    info->bb[0] = bb.c[0]; info->bb[1] = bb.c[1];
    free(r); free(rh); free(p); free(q); free(t); free(c); free(y); free(u); free(z); free(w); free(tp); free(tmp);
    return status;
}

int oracle_gpbicg(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                  const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                  oracle_solve_info *info, double *hist)
{
    return oracle_gpbicg_k(2, n, nnz, row_ptr, col_idx, log2w, a, b, x, minv, rtol, max_iter, info, hist);
}
