/*
 * mpsparse.h -- C ABI of the MI355X (gfx950) multi-component-precision sparse library.
 *
 * What it computes: CSR sparse matrix-vector products y = A x in double-double (DD,
 * K = 2 binary64 components), triple-double (TD, K = 3) and quad-double (QD, K = 4)
 * arithmetic, real and complex (Kouya, arXiv 2412.17510, Sec. 2 and Sec. 3), and the
 * DD Krylov solvers that call them (Sec. 4.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer (memory of the current HIP
 *   device), unless the comment says "host".  The caller owns all of them; the library
 *   never frees caller memory.  Plans (mp_plan) are library-owned: create and destroy
 *   them with the calls below.
 * Multi-component layout (Sec. 3: one binary64 array per component).  An array of
 *   length L with K components is ONE block of K*L doubles; component c (0 = leading)
 *   of element i is at base[c*L + i].  Components are non-overlapping with the leading
 *   one first (each at most half an ulp of the one above).
 * Complex data (Sec. 3, Eq. 2): separate real and imaginary multi-component blocks
 *   over one shared sparsity pattern.
 * CSR (Sec. 3): row_ptr int32[n_rows+1], col_idx int32[nnz], 0-based, row_ptr[0] = 0,
 *   non-decreasing, columns in [0, n_cols).  Values follow the col_idx order.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   SpMV calls only enqueue work and return.  Calls documented as synchronising wait
 *   for their stream before returning.
 * Errors.  Every call returns an mp_status; nothing aborts and no C++ exception
 *   crosses the ABI.  Host-side O(1) checks run on every call (null pointers, sizes,
 *   K, aliasing of outputs with inputs); a failed HIP call returns MP_ERR_HIP.  The
 *   message of the last failure of the calling thread is in mp_last_error().
 *   O(nnz) structural checks of a CSR matrix are done only by mp_csr_validate.
 *
 * Summation order (the reading of Sec. 3, Fig. 1 this library fixes).  For row i with
 *   len elements and lane width W = 2^log2w[i] (W <= len, W <= 1024): lane l < W
 *   accumulates the products of elements l, l+W, l+2W, ... in that order, starting
 *   from its first product; the W lane sums are folded as acc[l] = add(acc[l],
 *   acc[l+off]) for off = W/2, ..., 1; y_i = acc[0].  Products are mul(a, x) with the
 *   matrix operand first.  An empty row gives +0.  The canonical order uses the
 *   largest power of two W <= min(len, 64).  Two calls with the same lane widths give
 *   bitwise identical results, whatever kernel mapping a plan uses.
 */
#ifndef MPSPARSE_H
#define MPSPARSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MP_OK = 0,
    MP_ERR_INVALID_ARG = -1,   /* null pointer, bad size, bad K, malformed CSR (validate) */
    MP_ERR_ALIAS = -2,         /* an output overlaps an input */
    MP_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
    MP_ERR_NO_MEMORY = -4,     /* library allocation failed / workspace too small */
    MP_ERR_NOT_CONVERGED = -5, /* solver hit max_iter; best iterate written back */
    MP_ERR_BREAKDOWN = -6,     /* solver breakdown (zero or non-finite scalar) */
    MP_ERR_UNSUPPORTED = -7    /* option combination not provided */
} mp_status;

/* A CSR sparsity pattern (device pointers; see the conventions above). */
typedef struct {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
} mp_csr;

/* Opaque execution plan of one pattern for one variant (K components, real or
 * complex): the per-row lane widths (the summation order) and the work decomposition
 * one SpMV launch walks -- contiguous row tiles of at most tile_nnz elements whose
 * products are staged in LDS, single-row tiles for longer rows, and (row_groups)
 * wavefronts that each sum up to 64 / W rows of one lane width W in registers.  Owned by the
 * library and read-only after creation: SpMV calls that share a plan may run
 * concurrently on several streams (each with its own workspace). */
typedef struct mp_plan mp_plan;

/* Plan options.  Lane widths: log2w(len) = clamp(floor(log2(len)) - shift, 0,
 * max_log2w) for len >= 1 (empty rows get 0); shift = 0, max_log2w = 6 is the
 * canonical order.  tile_nnz: elements staged per workgroup tile, one of 256, 512,
 * 1024, 2048 and at most what the variant's LDS budget allows (DD real 2048, TD/QD
 * real 1024, DD/TD complex 512, QD complex 256); 0 = the largest allowed, capped at
 * 1024. */
typedef struct {
    int32_t shift;      /* 0..12: aim at >= 2^shift elements per lane */
    int32_t max_log2w;  /* 0..10: widest lane group (1024 lanes) */
    int32_t tile_nnz;   /* 0 or 256..2048 (power of two) */
    int32_t row_groups; /* 0: every row in tiles; rows with W <= 64 summed in wavefront lane
                           groups (same order): 1 those with at most 16 elements per lane,
                           2 all of them */
} mp_plan_opts;

/* Last error message of the calling thread ("" if none).  Static storage. */
const char *mp_last_error(void);

/* Library version string. */
const char *mp_version(void);

/* O(nnz) structural check of a CSR pattern on the device (row_ptr[0] == 0,
 * non-decreasing, row_ptr[n_rows] == nnz, col_idx in range).  Synchronises `stream`.
 * Returns MP_OK or MP_ERR_INVALID_ARG (with the first problem in mp_last_error()). */
mp_status mp_csr_validate(const mp_csr *A, void *stream);

/* Build a plan for pattern A and variant (ncomp in {2,3,4}, is_complex in {0,1}) with
 * the given options (NULL = canonical order, default tile size).  Reads row_ptr back
 * to the host once and uploads the tile list.  Synchronises `stream`. */
mp_status mp_plan_create(const mp_csr *A, int32_t ncomp, int32_t is_complex, const mp_plan_opts *opts,
                         void *stream, mp_plan **out);

/* Build a plan whose lane widths are given explicitly: host array log2w[n_rows],
 * each entry <= 10 and with 2^log2w[i] <= len_i for non-empty rows (0 for empty rows).
 * tile_nnz as in mp_plan_opts.  Synchronises `stream`. */
mp_status mp_plan_create_explicit(const mp_csr *A, int32_t ncomp, int32_t is_complex, const uint8_t *log2w_host,
                                  int32_t tile_nnz, void *stream, mp_plan **out);

/* Autotuned plan (Sec. 4.1 observes that SpMV speed depends on the matrix size and
 * structure): times the K-component kernel (complex if is_complex) on the caller's
 * operands (only read; y is overwritten) for a fixed list of tile sizes, then of width
 * policies, then of those policies (W <= 64) with row groups of both kinds; re-times
 * the three fastest twice more and keeps the lowest total.  The winning options are
 * returned in *chosen (may be NULL).  Synchronises `stream`. */
mp_status mp_plan_autotune(const mp_csr *A, int32_t ncomp, int32_t is_complex,
                           const double *a_re, const double *a_im, const double *x_re, const double *x_im,
                           double *y_re, double *y_im, int32_t reps, void *stream,
                           mp_plan **out, mp_plan_opts *chosen);

mp_status mp_plan_destroy(mp_plan *plan);

/* Copy the plan's per-row lane-width exponents to host array log2w_host[n_rows]
 * (the summation order of every row, for reproducing a result elsewhere). */
mp_status mp_plan_row_log2w(const mp_plan *plan, uint8_t *log2w_host);

/* Plan facts (host ints; any pointer may be NULL): rows, tiles, staged elements per
 * tile, variant. */
mp_status mp_plan_info(const mp_plan *plan, int32_t *n_rows, int32_t *n_tiles, int32_t *tile_nnz,
                       int32_t *ncomp, int32_t *is_complex);

/* Bytes of device workspace a planned SpMV with this plan needs (host size_t out):
 * an interleaved copy of x (its K components -- complex: then the K imaginary ones --
 * side by side per column, so one gather fetches every component), which the call
 * writes before its tile kernel reads it.  0 for a NULL plan. */
mp_status mpspmv_workspace_bytes(const mp_plan *plan, size_t *bytes);

/*
 * Real SpMV y = A x (Sec. 3, Fig. 1) in DD (Algs 1-2), TD and QD (Sec. 2).
 *   a: K*nnz values, x: K*n_cols, y: K*n_rows (multi-component layout above).
 *   plan: NULL = canonical order with a kernel that needs no plan (eight rows per
 *   wavefront: rows with W <= 8 on groups of eight lanes, wider rows on the whole
 *   wavefront); otherwise the plan's order and tiles (the plan must have been made for
 *   this variant and for a pattern with the same n_rows and nnz).
 *   ws: device workspace of ws_bytes >= mpspmv_workspace_bytes(plan) bytes, 256-byte
 *   aligned (ignored when that is 0, e.g. plan NULL); overwritten by the call and in
 *   use until it completes on `stream`, so concurrent calls need separate workspaces.
 *   y must not overlap a or x, nor ws an operand (MP_ERR_ALIAS); a workspace that is
 *   too small gives MP_ERR_NO_MEMORY.  Enqueues on `stream` and returns.
 */
mp_status mpspmv_csr_dd(const mp_csr *A, const double *a, const double *x, double *y,
                        const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_td(const mp_csr *A, const double *a, const double *x, double *y,
                        const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_qd(const mp_csr *A, const double *a, const double *x, double *y,
                        const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);

/*
 * mpspmv_csr_dd without workspace, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, order, results and errors as mpspmv_csr_dd, but the interleaved
 * copy of x is staged in a fixed 16 MiB device array of the library (one per GPU,
 * held from module load until the process ends), so n_cols <= 1,048,576 when plan is
 * non-NULL (larger: MP_ERR_NO_MEMORY before anything is launched).  Calls no
 * allocating routine.  Calls that overlap on one GPU share that array and race:
 * order them on one stream or with events.  Enqueues on `stream` and returns.
 */
mp_status mpspmv_csr_dd_noalloc(const mp_csr *A, const double *a, const double *x, double *y,
                                const mp_plan *plan, void *stream);

/*
 * Complex SpMV (Sec. 3, Eq. 3): with A = A_re + i A_im and x = x_re + i x_im,
 *   y_re = A_re x_re - A_im x_im and y_im = A_re x_im + A_im x_re, formed as four
 *   accumulator sets in one pass over the pattern (each in the order above) and
 *   combined at the end of the row: y_re = add(rr, -ii), y_im = add(ri, ir).
 *   Same layouts, workspace and rules as the real calls; y_re / y_im must not overlap
 *   any input or each other.
 */
mp_status mpspmv_csr_dd_complex(const mp_csr *A, const double *a_re, const double *a_im,
                                const double *x_re, const double *x_im, double *y_re, double *y_im,
                                const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_td_complex(const mp_csr *A, const double *a_re, const double *a_im,
                                const double *x_re, const double *x_im, double *y_re, double *y_im,
                                const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_qd_complex(const mp_csr *A, const double *a_re, const double *a_im,
                                const double *x_re, const double *x_im, double *y_re, double *y_im,
                                const mp_plan *plan, void *ws, size_t ws_bytes, void *stream);

/*
 * y = A x with a binary64 matrix and a K-component vector (Sec. 2: the SuiteSparse
 * matrices are binary64, multiplied by DD/QD/TD vectors with the mixed products of
 * Algs 3, 4 and 5).  a: nnz binary64 values (ONE component, element order of A);
 * x, y: K-component planar arrays as in mpspmv_csr_dd.  Each product is
 * mul_d(x_col, a_k) -- DD: TwoProd of the leading part plus the trailing part times
 * a, QuickTwoSum (Alg. 3); QD: Alg. 4 read after Hida, Li and Bailey; TD: the QD
 * product of the zero-padded value, three components kept (Alg. 5 per Sec. 2) --
 * and the row sums follow the plan's order exactly as in mpspmv_csr_dd, so a plan
 * made for (K, real) serves both.  For DD the result equals mpspmv_csr_dd on the
 * same matrix stored with zero trailing components.  Workspace, errors and aliasing
 * rules as mpspmv_csr_dd (a is nnz doubles).
 */
mp_status mpspmv_csr_dd_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                          void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_td_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                          void *ws, size_t ws_bytes, void *stream);
mp_status mpspmv_csr_qd_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * Complex y = A x with a binary64 complex matrix and a K-component complex vector
 * (Eq. 3 with the mixed products of Algs 3-5; the paper's complex SuiteSparse matrices
 * are binary64 too).  a_re, a_im: nnz binary64 values each (element order of A);
 * x_re, x_im, y_re, y_im: K-component planar arrays as in mpspmv_csr_dd_complex.
 * Four accumulator sets in the plan's order, each product the x part times the matrix
 * part: rr = sum mul_d(x_re, a_re), ii = sum mul_d(x_im, a_im), ri = sum mul_d(x_im,
 * a_re), ir = sum mul_d(x_re, a_im); y_re = rr + (-ii), y_im = ri + ir at the end of
 * the row.  A plan made for (K, complex) serves both this call and
 * mpspmv_csr_{dd,td,qd}_complex.  Workspace, errors and aliasing rules as
 * mpspmv_csr_dd_complex (a_re, a_im are nnz doubles each).
 */
mp_status mpspmv_csr_dd_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                  const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws,
                                  size_t ws_bytes, void *stream);
mp_status mpspmv_csr_td_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                  const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws,
                                  size_t ws_bytes, void *stream);
mp_status mpspmv_csr_qd_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                  const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws,
                                  size_t ws_bytes, void *stream);

/*
 * A^T in CSR, for A^T v (Sec. 3's SpTMV, which the paper computes by splitting A
 * across threads and combining the partial results in a critical section, and
 * suggests transposing first).  Row j of A^T lists column j of A in increasing row
 * order (a stable sort of the elements by column), the values permuted with the
 * pattern, so A^T v = an ordinary SpMV of A^T (with a plan of A^T) and is
 * deterministic.  ncomp: value components per array (1 for a binary64 matrix, 2..4
 * for DD/TD/QD); a_im/at_im both NULL (real) or both given.  Outputs (device,
 * caller-owned): row_ptr_t int32[n_cols+1], col_idx_t int32[nnz], at_re (and at_im)
 * double[ncomp*nnz] planar like a.  Allocates temporary device memory (about 16
 * bytes per element plus the sort workspace) and synchronises `stream`.  nnz must be
 * below 2^31.  MP_ERR_ALIAS if an output overlaps an input or another output.
 */
mp_status mp_csr_transpose(const mp_csr *A, int32_t ncomp, const double *a_re, const double *a_im,
                           int32_t *row_ptr_t, int32_t *col_idx_t, double *at_re, double *at_im, void *stream);

/*
 * COO -> CSR on the device (Sec. 3 describes both storage formats and the CSR
 * arrays a COO matrix maps to).  row, col: nnz 0-based coordinates (device int32);
 * v_re (and v_im for complex data, else NULL): ncomp planar value arrays of nnz
 * doubles (ncomp 1..4: a binary64 matrix or K components).  Outputs (device,
 * caller-allocated, not overlapping the inputs or each other): row_ptr int32[n_rows+1],
 * col_idx int32[nnz], a_re / a_im (ncomp*nnz doubles, a_im NULL iff v_im is NULL).
 * Elements are ordered by row, then column (a stable sort: elements with equal
 * coordinates stay in input order and are kept as separate elements, which the SpMV
 * then adds in that order).  Allocates temporaries and synchronises `stream`.
 * MP_ERR_INVALID_ARG for a coordinate outside the matrix (nothing written), negative
 * sizes, NULL pointers or ncomp out of range; MP_ERR_ALIAS for overlapping buffers;
 * MP_ERR_UNSUPPORTED for nnz >= 2^31.
 */
mp_status mp_coo_to_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row, const int32_t *col,
                        int32_t ncomp, const double *v_re, const double *v_im, int32_t *row_ptr, int32_t *col_idx,
                        double *a_re, double *a_im, void *stream);

/* ---------------------------------------------------------------------------
 * Krylov solvers in double-double (Sec. 4.2: CG for symmetric positive-definite A,
 * BiCGSTAB for non-symmetric A; x0 given, stop on the residual norm).
 *
 * The solve runs on the device: one SpMV (in the plan's order, or the canonical
 * order when plan is NULL) and fused DD vector kernels per step; every dot product
 * uses one fixed reduction tree (chunks of 4096 elements summed in the W = 256 lane
 * order, chunk sums combined pairwise), so iterates are reproducible bit for bit.
 * The iteration stops when the recurrence residual satisfies ||r||^2 <= rtol^2
 * ||b||^2 (DD comparison) and the true residual b - A x confirms it; a failed
 * confirmation restarts the recurrence from the true residual.  Scalars (alpha,
 * beta, omega) are DD, divisions use Dekker's DD long division.  The host reads the
 * device state back every `check_every` iterations (the only device-to-host
 * traffic of a solve).
 * ------------------------------------------------------------------------- */

enum { MP_PRECOND_NONE = 0, MP_PRECOND_JACOBI = 1, MP_PRECOND_LEARNED = 2 };
enum { MP_INNER_FP64 = 0, MP_INNER_FP32 = 1 };

typedef struct {
    int32_t precond;        /* MP_PRECOND_NONE or MP_PRECOND_JACOBI (z_i = r_i * fl(1/hi(a_ii)), Alg. 3);
                               MP_PRECOND_LEARNED for mpkrylov_ir_learned only */
    int32_t max_iter;       /* Krylov iterations (for refinement: per inner solve) */
    double rtol;            /* target ||b - A x||_2 <= rtol ||b||_2 */
    int32_t check_every;    /* iterations between host reads of the device state (0 = 32) */
    int32_t inner;          /* refinement only: MP_INNER_FP64 or MP_INNER_FP32 */
    double inner_rtol;      /* refinement only: residual reduction asked of each inner solve */
    int32_t inner_max_iter; /* refinement only (0 = max_iter) */
    int32_t max_outer;      /* refinement only: refinement steps */
} mp_solve_opts;

typedef struct {
    int32_t status;      /* MP_OK, MP_ERR_NOT_CONVERGED or MP_ERR_BREAKDOWN */
    int32_t iters;       /* Krylov iterations (refinement: total inner iterations) */
    int32_t outer_iters; /* refinement steps (0 for the plain solvers) */
    int32_t restarts;    /* failed true-residual confirmations */
    double rr_true[2];   /* DD ||b - A x||^2 of the returned x */
    double bb[2];        /* DD ||b||^2 */
    double relres;       /* sqrt(rr_true / bb) in binary64 */
    double seconds;      /* wall time of the call */
    int32_t fell_back;   /* refinement only: 1 if it switched to DD Jacobi-CG (stall or max_outer) */
    int32_t reserved;
} mp_solve_info;

/* z = x - y for n DD values (x, y, z: 2*n planar), each element by Alg. 1's addition
 * of x_i and the negation of y_i (exact sign flips of both components), so the result
 * keeps both components (e.g. the error x* - x_k of an iterate).  z may be x or y
 * itself but must not overlap them otherwise (MP_ERR_ALIAS).  Enqueues and returns. */
mp_status mpvec_dd_sub(int64_t n, const double *x, const double *y, double *z, void *stream);

/* Bytes of device workspace a solver needs for A and opts (host size_t out).  It
 * includes the staging buffer of the planned SpMV, so a solve only reads its plan and
 * solves that share a plan may run concurrently with separate workspaces. */
mp_status mpkrylov_workspace_bytes(const mp_csr *A, const mp_solve_opts *opts, size_t *bytes);

/*
 * DD preconditioned CG.  a: 2*nnz DD values of an SPD matrix (n_rows == n_cols);
 * b: 2*n right-hand side; x: 2*n, in = x0, out = solution (the best iterate on
 * non-convergence).  ws: device workspace of ws_bytes >= mpkrylov_workspace_bytes.
 * plan: NULL or a DD real plan of A.  info: host struct, filled on return.
 * Synchronises `stream`.  Returns MP_OK, MP_ERR_NOT_CONVERGED or MP_ERR_BREAKDOWN
 * (pAp <= 0 or a non-finite scalar), or an argument / HIP error.
 */
mp_status mpkrylov_cg(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                      const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);

/*
 * DD BiCGSTAB (van der Vorst) with right Jacobi preconditioning (or none), shadow
 * residual r0.  Arguments as mpkrylov_cg; A need not be symmetric.  Breakdown when
 * (r0, r), (r0, v) or (t, t) vanishes or omega = 0.
 */
mp_status mpkrylov_bicgstab(const mp_csr *A, const double *a, const double *b, double *x,
                            const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                            mp_solve_info *info, void *stream);

/*
 * DD CGS (Sonneveld's conjugate gradient squared; Sec. 4.2's list of product-type
 * Krylov methods) with right Jacobi preconditioning (opts.precond; solves A M y = b,
 * x = M y, so r is the residual of A x = b).  Shadow r~ = r at the start and after a
 * restart.  Step: rho = (r~, r) (breakdown if 0 or not finite); the first step after
 * a (re)start takes u = p = r, later ones beta = rho / rho_old, u = r + beta q,
 * p = u + beta (q + beta p); p^ = M p, v = A p^, sigma = (r~, v) (breakdown if 0 or
 * not finite), alpha = rho / sigma, q = u - alpha v, u^ = M (u + q), x += alpha u^,
 * r -= alpha A u^.  Two SpMVs per step.  Stop test, confirmation, restarts and
 * arguments as mpkrylov_cg (A need not be symmetric).
 */
mp_status mpkrylov_cgs(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                       const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);

/*
 * CG and BiCGSTAB in triple-double (_td, K = 3) and quad-double (_qd, K = 4): Sec. 4.2
 * runs the Krylov methods in every precision.  The steps, stopping rule, confirmation,
 * restarts and breakdown rules are those of mpkrylov_cg / mpkrylov_bicgstab with
 * K-component operations: add and mul (TD = the QD operation on zero-padded values,
 * three components kept), K-component times binary64 (Jacobi, Algs 4-5), division by
 * long division (q0 = a0/b0, three times r = r - b*q_i and q_{i+1} = r0/b0, the
 * quotient the 5 -> 4 renormalisation of q0..q3, truncated to three components for
 * TD), stop tests by lexicographic comparison of the components, and the dot
 * product tree of the DD solvers.  a: K*nnz values (component-planar); b, x: K*n;
 * plan: NULL or a K-component real plan of A; ws: device workspace of at least
 * mpkrylov_mp_workspace_bytes(A, K) bytes, 256-byte aligned; n <= 4,194,304.  info
 * carries the two leading components of rr_true and bb (relres from the leading
 * ones).  Synchronises `stream`.  Returns MP_OK, MP_ERR_NOT_CONVERGED,
 * MP_ERR_BREAKDOWN or an argument / HIP error (as mpkrylov_cg).
 */
mp_status mpkrylov_mp_workspace_bytes(const mp_csr *A, int32_t ncomp, size_t *bytes);
mp_status mpkrylov_cg_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                         const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_cg_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                         const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_bicgstab_td(const mp_csr *A, const double *a, const double *b, double *x,
                               const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                               mp_solve_info *info, void *stream);
mp_status mpkrylov_bicgstab_qd(const mp_csr *A, const double *a, const double *b, double *x,
                               const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                               mp_solve_info *info, void *stream);

/* CGS, GPBiCG and BiCG in TD / QD: the steps of mpkrylov_cgs, mpkrylov_gpbicg and
 * mpkrylov_bicg with the K-component operations above (BiCG: At, at the K-component
 * transpose, e.g. from mp_csr_transpose with ncomp = K, plan_t NULL or a K-component
 * plan of At).  Arguments, workspace and results as mpkrylov_cg_td / _qd. */
mp_status mpkrylov_cgs_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                          const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_cgs_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                          const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_gpbicg_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                             const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_gpbicg_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                             const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_bicg_td(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                           double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                           size_t ws_bytes, mp_solve_info *info, void *stream);
mp_status mpkrylov_bicg_qd(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                           double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                           size_t ws_bytes, mp_solve_info *info, void *stream);

/*
 * DD GPBiCG (Zhang's generalized product-type method based on BiCG; Sec. 4.2's list)
 * with right Jacobi preconditioning (opts.precond; every product with A is one with
 * A M and x collects M times the corrections, so r is the residual of A x = b).
 * Shadow r~ = r at the start and after a restart.  Step: rho = (r~, r) (breakdown if
 * 0 or not finite); the first step after a (re)start takes p = r, later ones
 * beta = (alpha'/zeta')(rho/rho'), p = r + beta (p - u), w = c' + beta q' (primes:
 * previous step); q = A M p, sigma = (r~, q) (breakdown if 0 or not finite),
 * alpha = rho / sigma, t = r - alpha q, later steps y = t' - t - alpha w.  If
 * (t, t) meets the tolerance: x += M (alpha p), r = t, confirm, and the next step is
 * fresh.  Else c = A M t; first step zeta = (c,t)/(c,c), eta = 0; later steps
 * d = (c,c)(y,y) - (y,c)^2, zeta = ((y,y)(c,t) - (y,t)(y,c))/d,
 * eta = ((c,c)(y,t) - (y,c)(c,t))/d (breakdown if (c,c) or d is 0, zeta is 0, or zeta
 * or eta is not finite); u = zeta q + eta (t' - r + beta u), z = zeta r + eta z -
 * alpha u (first step: u = zeta q, z = zeta r - alpha u), x += M (alpha p + z),
 * r = t - eta y - zeta c (first step: t - zeta c), t' = t.  Two SpMVs per step; a
 * step is counted when t is formed.  Stop test, confirmation, restarts and arguments
 * as mpkrylov_cg (A need not be symmetric).
 */
mp_status mpkrylov_gpbicg(const mp_csr *A, const double *a, const double *b, double *x,
                          const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                          mp_solve_info *info, void *stream);

/*
 * DD BiCG (Fletcher's biconjugate gradients; Sec. 4.2 lists BiCG among the product-
 * type Krylov methods, and its SpTMV is what slows it down there).  A^T is passed
 * explicitly (At, at: e.g. from mp_csr_transpose, 2*nnz DD values) with an optional
 * DD real plan of At (plan_t), so both products are ordinary planned SpMVs.  Jacobi
 * (opts.precond) is symmetric, so the shadow system uses the same M.  r~ = r at the
 * start and after every restart.  Step: q = A p, q~ = A^T p~, sigma = (p~, q),
 * alpha = rho / sigma, x += alpha p, r -= alpha q, r~ -= alpha q~, z = M r,
 * z~ = M r~, rho' = (r~, z), beta = rho' / rho, p = z + beta p, p~ = z~ + beta p~.
 * Stop test, true-residual confirmation and restarts as mpkrylov_cg.  Breakdown:
 * sigma = 0, rho' = 0 before convergence, or a non-finite scalar.  On an exactly
 * symmetric A (pattern and values) with At its stable transpose the iterates equal
 * mpkrylov_cg's bit for bit.  Other arguments as mpkrylov_cg.
 */
mp_status mpkrylov_bicg(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                        double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                        size_t ws_bytes, mp_solve_info *info, void *stream);

/*
 * Mixed-precision iterative refinement (layer on the paper's method; the paper lists
 * mixed-precision Krylov methods as future work, Sec. 5).  Outer loop in DD: r = b - A x
 * with the DD SpMV (plan order) and a DD subtraction; stop when ||r||^2 <= rtol^2
 * ||b||^2.  Otherwise the inner right-hand side is hi(r) scaled by 2^-e (e = exponent of
 * max |hi(r)|, an exact scaling) and rounded to the inner precision; the inner solve is
 * Jacobi-PCG (opts.precond) on hi(A) in binary64 (MP_INNER_FP64) or on fl32(hi(A)) in
 * binary32 (MP_INNER_FP32), to a residual reduction of opts.inner_rtol or
 * opts.inner_max_iter iterations, each row of its SpMV summed sequentially and its dot
 * products in the DD solver's tree shape; then x_i = DDadd(x_i, (d_i 2^e, 0)).  If two
 * consecutive refinement steps each reduce ||r||^2 by less than 4x, or max_outer steps
 * pass, the solve continues as DD Jacobi-CG from the current x (opts.max_iter
 * iterations) and info.fell_back = 1.  Arguments as mpkrylov_cg; A must be SPD for the
 * inner CG.  Workspace: mpkrylov_workspace_bytes with the same opts (binary32 adds a
 * copy of hi(A)).
 */
mp_status mpkrylov_ir(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                      const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream);

/*
 * Refinement as mpkrylov_ir, with the inner PCG preconditioned by a given sparse
 * approximate inverse M instead of Jacobi: z = M r, M given by its binary64 values on
 * A's pattern (m_values: device double[nnz], same element order as a; read only;
 * rounded to binary32 for MP_INNER_FP32), each row of z = M r summed sequentially in
 * element order.  M must be symmetric positive definite for the inner CG (the
 * network of mp_mpnn_forward guarantees it).  opts.precond must be
 * MP_PRECOND_LEARNED; the stall / max_outer fallback is plain DD Jacobi-CG.  With M =
 * D^-1 stored on the pattern (zero off-diagonal values) the iterates equal
 * mpkrylov_ir's with MP_PRECOND_JACOBI.  Workspace: mpkrylov_workspace_bytes with the
 * same opts (binary32 adds copies of hi(A) and M).  MP_ERR_ALIAS if m_values overlaps
 * x or the workspace.
 */
mp_status mpkrylov_ir_learned(const mp_csr *A, const double *a, const double *m_values, const double *b, double *x,
                              const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                              mp_solve_info *info, void *stream);

/* ---------------------------------------------------------------------------
 * Batched systems (layer on the paper's method): nsys independent square systems
 * stored as the diagonal blocks of ONE block-diagonal CSR matrix A (system s owns rows
 * and columns [sys_ptr[s], sys_ptr[s+1]); no entry outside its block), each with nrhs
 * right-hand sides (nrhs in {1, 2, 4, 8}).  Multi-RHS arrays are DD, component-major,
 * right-hand sides fastest: V[c*N*nrhs + row*nrhs + r] (N = n_rows, c in {0, 1}).
 * Every row of the batched SpMM is summed sequentially in element order (the SpMV
 * order with W = 1), so results equal separate mpspmv_csr_dd calls with a plan whose
 * lane widths are all 1, and the batched CG equals separate mpkrylov_cg calls (one per
 * system and right-hand side) with such a plan, bit for bit.
 * ------------------------------------------------------------------------- */

/* Opaque batch schedule: the system table, the per-system chunks of the dot products
 * and the SpMM thread mapping (threads per row).  Owned by the library. */
typedef struct mp_batch_plan mp_batch_plan;

/* Build a batch plan.  sys_ptr_host: host int32[nsys+1], sys_ptr[0] = 0, strictly
 * increasing, sys_ptr[nsys] = n_rows.  threads_per_row: power of two <= nrhs (each
 * thread computes nrhs/threads_per_row right-hand sides of one row).  Checks on the
 * device that A is block-diagonal (MP_ERR_INVALID_ARG otherwise).  Synchronises. */
mp_status mp_batch_plan_create(const mp_csr *A, const int32_t *sys_ptr_host, int32_t nsys, int32_t nrhs,
                               int32_t threads_per_row, void *stream, mp_batch_plan **out);

/* Autotune the batch schedule on the caller's operands (X read, Y overwritten): the
 * persistent SpMM of the CG step is timed for every threads-per-row choice (each
 * thread computes nrhs/threads_per_row right-hand sides of one row) and every tile of
 * (256 / threads_per_row) * {1, 2, 4} rows, and the dot-chunk kernels for the two item
 * orders (chunks in row order, or the chunks of the largest systems first); the
 * fastest choices are kept in the plan.  *threads_per_row (host, may be NULL) receives
 * the chosen mapping.  Allocates temporaries and synchronises. */
mp_status mp_batch_plan_autotune(mp_batch_plan *plan, const mp_csr *A, const double *a, const double *X, double *Y,
                                 int32_t reps, void *stream, int32_t *threads_per_row);

/* The plan's schedule (host ints, any may be NULL): threads per row, rows per SpMM
 * tile of the CG step, and the chunk order (0 row order, 1 largest systems first). */
mp_status mp_batch_plan_schedule(const mp_batch_plan *plan, int32_t *threads_per_row, int32_t *rows_per_tile,
                                 int32_t *chunk_order);

/* Set the schedule explicitly (instead of autotuning): threads_per_row a power of two
 * <= nrhs, SpMM tiles of (256 / threads_per_row) * rows_mult rows with rows_mult in
 * {1, 2, 4}, chunk_order 0 or 1.  Results do not depend on the schedule. */
mp_status mp_batch_plan_set_schedule(mp_batch_plan *plan, int32_t threads_per_row, int32_t rows_mult,
                                     int32_t chunk_order);

mp_status mp_batch_plan_destroy(mp_batch_plan *plan);

/* Y = A X for every right-hand side (DD).  a: 2*nnz; X, Y: 2*N*nrhs.  plan may be NULL
 * (one thread per row).  Enqueues and returns. */
mp_status mpspmm_csr_dd_batched(const mp_csr *A, const double *a, const double *X, double *Y, int32_t nrhs,
                                const mp_batch_plan *plan, void *stream);

/* Device workspace bytes of mpkrylov_cg_batched for a plan (host size_t out). */
mp_status mpkrylov_batched_workspace_bytes(const mp_batch_plan *plan, size_t *bytes);

/*
 * DD Jacobi-PCG (opts.precond) for every (system, right-hand side) pair at once.
 * B: right-hand sides, X: in = starting vectors, out = solutions (2*N*nrhs each).
 * Each pair keeps its own DD scalars, stop test (rtol), true-residual confirmation,
 * restarts and iteration limit, exactly as mpkrylov_cg.  One step is four persistent
 * kernels over all pairs (the SpMM over row tiles; the (p, q) chunk sums; alpha and the
 * update of x and r with the (r, z), (r, r) chunk sums; beta, the stop tests and p),
 * each sized to the device's resident occupancy, its workgroups taking tiles or dot
 * chunks in the plan's order from one work queue per XCD (a vector-memory atomic
 * counter each; a workgroup that finds its queue empty takes from the others; no
 * workgroup ever waits for another).  Every item of a system forms that system's
 * scalars itself from the chunk sums (the per-system trees).  With use_graph = 1 a
 * chunk of opts.check_every steps is captured once into a hipGraph and replayed (on a
 * private stream ordered after `stream`) until every pair has finished.  info: host
 * array of nsys*nrhs records, pair (s, r) at index s*nrhs + r.  Synchronises `stream`.
 * Returns MP_OK when every pair converged, else the worst pair status.
 */
mp_status mpkrylov_cg_batched(const mp_csr *A, const double *a, const double *B, double *X, int32_t nrhs,
                              const mp_solve_opts *opts, const mp_batch_plan *plan, int32_t use_graph, void *ws,
                              size_t ws_bytes, mp_solve_info *info, void *stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (layer on the paper's method, for the refinement's inner
 * solve): a message-passing network over the graph of a Stieltjes matrix (SPD with
 * non-positive off-diagonal entries, like every diffusion matrix; symmetric pattern,
 * sorted columns) predicts M = S (I + Delta + G o W) S on A's pattern (S = D^-1/2,
 * W = the scaled negated off-diagonal part, g_ij in [0, 1) symmetric, Delta >= 0
 * diagonal): a damped first-order Neumann approximation of A^-1 = S (I - W)^-1 S.  M
 * is SPD (W >= 0 has spectral radius below 1, so does G o W <= W), and zero weights
 * give exactly M = D^-1.  Network, with w_ij = -hi(a_ij)/sqrt(hi(a_ii) hi(a_jj)) and
 * node features f_i = [sum_j w_ij, sum_j w_ij^2, deg_i/8, 1]:
 *   h0 = relu(f W0 + b0); three layers h = relu(h Ws + (sum_j w_ij h_j) Wn + b);
 *   u_i = h_i.wu + bu; v_ij = sum_k qv_k h_ik h_jk + bv; g_ij = tanh(v_ij)^2;
 *   M_ij = g_ij w_ij sqrt(m_i m_j) (i != j), M_ii = (1 + log(1 + u_i^2)) m_i, m = 1/a_ii.
 * Hidden width 64; 25218 parameters, float32 master copy in this order: W0 (4x64,
 * row-major), b0, then per layer Ws (64x64), Wn (64x64), b; then wu, bu, qv, bv.
 * Weights and dense-layer inputs are rounded to bfloat16 (nearest-even) when used,
 * products accumulate in float32; M is assembled in binary64.  Training minimises
 * L = (M r - e)^T A (M r - e) / e^T A e over pairs (r, e = A^-1 r); the backward pass
 * takes the bfloat16 roundings as the identity.  Every reduction has a fixed order,
 * so forward values and gradients are deterministic.
 * ------------------------------------------------------------------------- */

typedef struct mp_mpnn mp_mpnn;     /* parameters, gradients, Adam moments (device) */
typedef struct mp_graph mp_graph;   /* one matrix's graph, features and activations */

/* Number of parameters (host int32 out). */
mp_status mp_mpnn_param_count(int32_t *count);

/* Create a network with all parameters, gradients and moments zero.  hidden must be 64
 * (MP_ERR_UNSUPPORTED otherwise). */
mp_status mp_mpnn_create(int32_t hidden, mp_mpnn **out);
mp_status mp_mpnn_destroy(mp_mpnn *net);

/* Copy parameters from / to a host float[param_count]; set also zeroes the Adam
 * moments.  Gradients: host float[param_count].  These synchronise the device. */
mp_status mp_mpnn_set_params(mp_mpnn *net, const float *host_params);
mp_status mp_mpnn_get_params(const mp_mpnn *net, float *host_params);
mp_status mp_mpnn_get_grads(const mp_mpnn *net, float *host_grads);

/* Zero the gradient accumulator (enqueued on stream). */
mp_status mp_mpnn_zero_grads(mp_mpnn *net, void *stream);

/*
 * Build the graph of A: a = DD values (device, 2*nnz; only hi is read).  The graph
 * keeps pointers to A's row_ptr/col_idx and to a: they must stay valid and unchanged
 * while it exists.  MP_ERR_INVALID_ARG unless every row has a positive diagonal, every
 * off-diagonal entry is <= 0 and has its transpose (columns sorted).  Synchronises.
 */
mp_status mp_graph_create(const mp_csr *A, const double *a, void *stream, mp_graph **out);
mp_status mp_graph_destroy(mp_graph *g);

/* Forward pass: m_values (device double[nnz], A's element order) = M.  Enqueues. */
mp_status mp_mpnn_forward(const mp_mpnn *net, mp_graph *g, double *m_values, void *stream);

/*
 * Forward pass, loss and backward pass for npairs pairs (device, r and e each
 * npairs*n binary64 values, pair p at offset p*n; 1 <= npairs <= n): the
 * gradients of the npairs losses are ADDED to the network's accumulator.
 * loss_host: NULL or host double[npairs] (then the call synchronises).  A = hi of the
 * graph's values.  Calls on one graph must not overlap (activations are per graph).
 */
mp_status mp_mpnn_loss_grad(mp_mpnn *net, mp_graph *g, const double *r, const double *e, int32_t npairs,
                            double *loss_host, void *stream);

/* One Adam step (bias-corrected, step >= 1) on the accumulated gradients times
 * grad_scale.  Enqueues. */
mp_status mp_mpnn_adam_step(mp_mpnn *net, float lr, float beta1, float beta2, float eps, float grad_scale,
                            int32_t step, void *stream);

/* ------------------------------------------------------------------------- */
/* Measured ceilings                                                          */
/* ------------------------------------------------------------------------- */

/*
 * Throughput of the arithmetic the kernels are made of, measured on the current
 * device, so that roofline fractions can be stated against what the device delivers
 * as well as against its specification.  kind 0: binary64 FMA instructions per second
 * (per lane; eight independent chains per thread, 16 workgroups of 256 threads per
 * compute unit).  kind K = 2, 3, 4: K-component "mul then add" steps per second, the
 * inner step of the SpMV (Sec. 2 operations: Algs 1-2 for DD, the quad-double
 * sequences for QD, TD as QD on zero-padded values), two independent accumulators per
 * thread; each step also carries one binary64 multiply that keeps the product in the
 * loop.  *per_second is a host double.  Allocates and frees 8 MiB of device memory and
 * synchronises the stream.  MP_ERR_INVALID_ARG for another kind or a NULL output.
 */
mp_status mp_measure_rate(int32_t kind, double *per_second, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MPSPARSE_H */
