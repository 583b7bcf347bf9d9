/*
 * sanitize_driver.c -- CPU ORACLE, TEST INFRASTRUCTURE ONLY.
 *
 * A stand-alone program that runs the oracle's entry points on small matrices so that
 * the oracle can be built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py): every SpMV variant (real, complex, binary64 matrix;
 * K = 2, 3, 4; canonical, explicit and row-subset calls), the transpose, COO -> CSR, the
 * DD and K-component Krylov solvers, refinement and the exact residual.  A sanitizer
 * finding aborts the program; a returned status other than the one expected makes it
 * exit with 1.  Inputs come from a fixed linear congruential sequence (no method
 * arithmetic here).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t status, iters, restarts, reserved;
    double rr_true[2], bb[2];
} oracle_solve_info;

typedef struct {
    int32_t status, iters, outer_iters, fell_back;
    double rr_true[2], bb[2];
} oracle_ir_info;

typedef int (*solver_k)(int, int64_t, int64_t, const int32_t *, const int32_t *, const uint8_t *, const double *,
                        const double *, double *, const double *, double, int32_t, oracle_solve_info *, double *);

int oracle_spmv(int K, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                const uint8_t *log2w, const double *a_re, const double *a_im, const double *x_re, const double *x_im,
                double *y_re, double *y_im, int64_t nsel, const int64_t *rows, int nthreads);
int oracle_spmv_dmat(int K, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr,
                     const int32_t *col_idx, const uint8_t *log2w, const double *a, const double *x, double *y,
                     int64_t nsel, const int64_t *rows, int nthreads);
int oracle_spmv_dmat_complex(int K, int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, const uint8_t *log2w, const double *a_re, const double *a_im,
                             const double *x_re, const double *x_im, double *y_re, double *y_im, int64_t nsel,
                             const int64_t *rows, int nthreads);
int oracle_transpose(int64_t n_rows, int64_t n_cols, int64_t nnz, int ncomp, const int32_t *row_ptr,
                     const int32_t *col_idx, const double *a, int32_t *row_ptr_t, int32_t *col_idx_t, double *a_t);
int oracle_coo_to_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t *row, const int32_t *col, int ncomp,
                      const double *v, int32_t *row_ptr, int32_t *col_idx, double *a);
int oracle_cg(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
              const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
              oracle_solve_info *info, double *hist);
int oracle_bicgstab(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                    const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                    oracle_solve_info *info, double *hist);
int oracle_cg_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                oracle_solve_info *info, double *hist);
int oracle_bicgstab_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      const uint8_t *log2w, const double *a, const double *b, double *x, const double *minv,
                      double rtol, int32_t max_iter, oracle_solve_info *info, double *hist);
int oracle_cgs_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
                 const double *a, const double *b, double *x, const double *minv, double rtol, int32_t max_iter,
                 oracle_solve_info *info, double *hist);
int oracle_gpbicg_k(int K, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                    const uint8_t *log2w, const double *a, const double *b, double *x, const double *minv, double rtol,
                    int32_t max_iter, oracle_solve_info *info, double *hist);
int oracle_ir(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *log2w,
              const double *a, const double *b, double *x, int inner_fp32, int jacobi, const double *mvals,
              double rtol, double inner_rtol, int32_t inner_max_iter, int32_t max_outer, int32_t max_iter,
              oracle_ir_info *info);
int oracle_exact_residual(int Ka, int Kx, int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *a, const double *b, const double *x, double *r_near, double *norms);
int oracle_mp_dot(int K, int64_t n, const double *x, const double *y, double *out);

static uint64_t lcg_state = 88172645463325252ull;

/* uniform in [-1, 1) from the top 53 bits of a 64-bit LCG */
static double urand(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 4503599627370496.0) - 1.0;
}

static void fill(double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i) v[i] = urand();
}

static int failures = 0;

static void expect(const char *what, int got, int want)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

/* ragged matrix: rows of 0..12 elements with sorted distinct columns */
static int64_t ragged(int64_t n, int32_t *rp, int32_t *ci)
{
    int64_t nnz = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int len = (int)((urand() + 1.0) * 6.5);
        int32_t c = (int32_t)((urand() + 1.0) * 2.0);
        for (int k = 0; k < len && c < n; ++k) {
            ci[nnz++] = c;
            c += 1 + (int32_t)((urand() + 1.0) * 3.0);
        }
        rp[i + 1] = (int32_t)nnz;
    }
    return nnz;
}

/* SPD tridiagonal matrix 4, -1 with planar K-component values (components beyond the
 * first zero) */
static int64_t tridiag(int64_t n, int K, int32_t *rp, int32_t *ci, double *a, int64_t cap)
{
    int64_t nnz = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i - 1; j <= i + 1; ++j) {
            if (j < 0 || j >= n) continue;
            ci[nnz] = (int32_t)j;
            for (int c = 0; c < K; ++c) a[c * cap + nnz] = c == 0 ? (i == j ? 4.0 : -1.0) : 0.0;
            ++nnz;
        }
        rp[i + 1] = (int32_t)nnz;
    }
    return nnz;
}

int main(void)
{
    enum { N = 300, CAP = 300 * 13 };
    int32_t *rp = malloc(sizeof(int32_t) * (N + 1)), *ci = malloc(sizeof(int32_t) * CAP);
    double *are = malloc(sizeof(double) * 4 * CAP), *aim = malloc(sizeof(double) * 4 * CAP);
    double *xre = malloc(sizeof(double) * 4 * N), *xim = malloc(sizeof(double) * 4 * N);
    double *yre = malloc(sizeof(double) * 4 * N), *yim = malloc(sizeof(double) * 4 * N);
    uint8_t *lw = malloc(N);
    int64_t rows[3] = {0, 7, N - 1};
    const int64_t nnz = ragged(N, rp, ci);
    fill(are, 4 * CAP);
    fill(aim, 4 * CAP);
    fill(xre, 4 * N);
    fill(xim, 4 * N);
    for (int64_t i = 0; i < N; ++i) lw[i] = 0;
    for (int K = 2; K <= 4; ++K) {
        /* planar components of nnz values: component c at a[c * nnz + k] */
        expect("spmv real", oracle_spmv(K, N, N, nnz, rp, ci, NULL, are, NULL, xre, NULL, yre, NULL, 0, NULL, 2), 0);
        expect("spmv complex", oracle_spmv(K, N, N, nnz, rp, ci, NULL, are, aim, xre, xim, yre, yim, 0, NULL, 2), 0);
        expect("spmv rows", oracle_spmv(K, N, N, nnz, rp, ci, lw, are, NULL, xre, NULL, yre, NULL, 3, rows, 1), 0);
        expect("spmv dmat", oracle_spmv_dmat(K, N, N, nnz, rp, ci, NULL, are, xre, yre, 0, NULL, 2), 0);
        expect("spmv dmat complex",
               oracle_spmv_dmat_complex(K, N, N, nnz, rp, ci, NULL, are, aim, xre, xim, yre, yim, 0, NULL, 2), 0);
        double d[4];
        expect("dot", oracle_mp_dot(K, N, xre, xim, d), 0);
    }
    /* a lane width wider than a (non-empty) row is refused */
    int64_t wr = 0;
    while (rp[wr + 1] == rp[wr]) ++wr;
    lw[wr] = 10;
    expect("spmv bad width", oracle_spmv(2, N, N, nnz, rp, ci, lw, are, NULL, xre, NULL, yre, NULL, 0, NULL, 1), -1);
    lw[wr] = 0;

    int32_t *rpt = malloc(sizeof(int32_t) * (N + 1)), *cit = malloc(sizeof(int32_t) * CAP);
    double *at = malloc(sizeof(double) * 2 * CAP);
    expect("transpose", oracle_transpose(N, N, nnz, 2, rp, ci, are, rpt, cit, at), 0);

    int32_t *cr = malloc(sizeof(int32_t) * CAP), *cc = malloc(sizeof(int32_t) * CAP);
    for (int64_t i = 0; i < N; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            cr[k] = (int32_t)(N - 1 - i);
            cc[k] = ci[k];
        }
    expect("coo to csr", oracle_coo_to_csr(N, N, nnz, cr, cc, 2, are, rpt, cit, at), 0);
    cr[0] = N;   /* a row outside the matrix */
    expect("coo out of range", oracle_coo_to_csr(N, N, nnz, cr, cc, 2, are, rpt, cit, at), -2);

    /* solvers on the tridiagonal SPD system, b random */
    double *b = malloc(sizeof(double) * 4 * N), *x = malloc(sizeof(double) * 4 * N);
    double *minv = malloc(sizeof(double) * N), *hist = malloc(sizeof(double) * 2 * 4001);
    double norms[4];
    oracle_solve_info info;
    oracle_ir_info iri;
    for (int64_t i = 0; i < N; ++i) minv[i] = 0.25;
    for (int K = 2; K <= 4; ++K) {
        const int64_t tn = tridiag(N, K, rp, ci, are, CAP);
        /* the solvers read the matrix as K planar arrays of tn values */
        double *ak = malloc(sizeof(double) * K * tn);
        for (int c = 0; c < K; ++c) memcpy(ak + c * tn, are + c * CAP, sizeof(double) * tn);
        fill(b, (size_t)K * N);
        for (int c = 1; c < K; ++c)
            for (int64_t i = 0; i < N; ++i) b[c * N + i] = 0.0;
        const solver_k solvers[4] = {oracle_cg_k, oracle_bicgstab_k, oracle_cgs_k, oracle_gpbicg_k};
        const char *names[4] = {"cg_k", "bicgstab_k", "cgs_k", "gpbicg_k"};
        for (int s = 0; s < 4; ++s) {
            memset(x, 0, sizeof(double) * K * N);
            expect(names[s], solvers[s](K, N, tn, rp, ci, NULL, ak, b, x, minv, 1e-25, 4000, &info, hist), 0);
            expect(names[s], info.status, 0);
        }
        expect("exact residual", oracle_exact_residual(K, K, N, tn, rp, ci, ak, b, x, NULL, norms), 0);
        if (K == 2) {
            memset(x, 0, sizeof(double) * 2 * N);
            expect("cg", oracle_cg(N, tn, rp, ci, NULL, ak, b, x, minv, 1e-28, 4000, &info, hist), 0);
            memset(x, 0, sizeof(double) * 2 * N);
            expect("bicgstab", oracle_bicgstab(N, tn, rp, ci, NULL, ak, b, x, NULL, 1e-28, 4000, &info, hist), 0);
            for (int fp32 = 0; fp32 <= 1; ++fp32) {
                memset(x, 0, sizeof(double) * 2 * N);
                expect("ir", oracle_ir(N, tn, rp, ci, NULL, ak, b, x, fp32, 1, NULL, 1e-28, fp32 ? 1e-5 : 1e-8, 2000,
                                       50, 4000, &iri),
                       0);
                expect("ir status", iri.status, 0);
            }
            /* an iteration limit is reported, not an error of the call */
            memset(x, 0, sizeof(double) * 2 * N);
            oracle_cg(N, tn, rp, ci, NULL, ak, b, x, minv, 1e-28, 3, &info, hist);
            expect("cg limit", info.status, -5);
        }
        free(ak);
    }
    free(rp); free(ci); free(are); free(aim); free(xre); free(xim); free(yre); free(yim); free(lw);
    free(rpt); free(cit); free(at); free(cr); free(cc); free(b); free(x); free(minv); free(hist);
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
