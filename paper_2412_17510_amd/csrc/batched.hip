// batched.hip -- many independent DD systems with several right-hand sides.
//
// The systems are the diagonal blocks of one block-diagonal CSR matrix: system s owns
// rows and columns [sys_ptr[s], sys_ptr[s+1]).  Multi-RHS vectors are component-major
// with the right-hand sides fastest: V[c][row][r] at V[c*N*R + row*R + r].
//
// SpMM y_r = A x_r for every r: one thread per (row, group of R/TPR right-hand sides);
// each row is summed sequentially in element order (the SpMV order with W = 1), so
// the result equals R separate single-vector SpMVs with a W = 1 plan bit for bit.
// The matrix entry of an element is loaded once and used for all of the thread's
// right-hand sides; x_j's R values are contiguous (one 16-64 B run per component).
//
// Batched CG: the DD Jacobi-PCG of krylov.hip run for every (system, rhs) pair at
// once.  Dot products of a pair follow the single-system tree over that system's rows
// (chunks of 4096 rows from the system's first row; W = 256 lane order; pairwise
// chunk tree), every pair has its own DD scalars and state, and a pair whose state is
// not "running" is left untouched by the update kernels -- so each pair's iterates
// equal those of a separate mpkrylov_cg call with a W = 1 plan, bit for bit.  One
// step is six kernels over all pairs; a chunk of steps is captured once into a
// hipGraph and replayed, the host reading the pair states between replays to
// confirm converged pairs with their true residuals (and restart those that fail).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "mp_arith.hpp"

namespace mpk {

constexpr int kBLanes = 256;
constexpr int kBChunk = 4096;
constexpr int kBMaxRhs = 8;
constexpr int kBMaxSysChunks = 2048;

}  // namespace mpk

struct mp_batch_plan {
    int32_t n_rows = 0;
    int64_t nnz = 0;
    int32_t nsys = 0;
    int32_t nrhs = 0;
    int32_t tpr = 1;          // SpMM threads per row
    int32_t n_chunks = 0;     // dot chunks (<= 4096 rows of one system)
    int32_t max_sys_chunks = 0;
    int32_t *d_sys_ptr = nullptr;
    int32_t *d_sys_chunk = nullptr;   // nsys + 1: first chunk of each system
    int32_t *d_chunk_row = nullptr;   // n_chunks: first row of each chunk
    int32_t *d_chunk_sys = nullptr;   // n_chunks: system of each chunk
    std::vector<int32_t> sys_ptr;
};

namespace mpk {

enum : int32_t { B_RUN = 0, B_RECURRENCE_MET = 1, B_BROKE_DOWN = 2, B_ITER_LIMIT = 3, B_CONFIRMED = 4, B_RESTART = 5 };

struct BState {
    dd_t rho, rr, bb, tol2, pq, alpha, beta, rr_true;
    int32_t done;
    int32_t iters;
    int32_t restarts;
    int32_t pad;
};

__device__ __forceinline__ dd_t bz()
{
    dd_t r;
    r.c[0] = 0.0;
    r.c[1] = 0.0;
    return r;
}

// V[c][row][r]
__device__ __forceinline__ dd_t bld(const double *__restrict__ v, int64_t NR, int64_t row, int R, int r)
{
    dd_t x;
    x.c[0] = v[row * R + r];
    x.c[1] = v[NR + row * R + r];
    return x;
}

__device__ __forceinline__ void bst(double *__restrict__ v, int64_t NR, int64_t row, int R, int r, const dd_t &x)
{
    v[row * R + r] = x.c[0];
    v[NR + row * R + r] = x.c[1];
}

__device__ __forceinline__ int bxcd_block(int b, int nblocks)
{
    const int xcd = b & 7;
    const int idx = b >> 3;
    const int per = nblocks >> 3;
    const int rem = nblocks & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// ---------------------------------------------------------------------------
// SpMM
// ---------------------------------------------------------------------------

template <int R, int TPR>
__global__ __launch_bounds__(256) void k_bspmm(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                               const double *__restrict__ a, int64_t nnz, const double *__restrict__ X,
                                               double *__restrict__ Y)
{
    constexpr int RPT = R / TPR;
    const int64_t g = (int64_t)bxcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t row = g / TPR;
    if (row >= n) return;
    const int r0 = (int)(g % TPR) * RPT;
    const int64_t NR = (int64_t)n * R;
    const int32_t b = rp[row], e = rp[row + 1];
    dd_t acc[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) acc[q] = bz();
    // elements in groups of kG: matrix operands first, then the x gathers, then the
    // products in element order.  Eight covers a 7-point stencil row in one round of
    // loads (measured 10 % faster than groups of four on the batched diffusion systems).
    constexpr int kG = 8;
    for (int32_t k0 = b; k0 < e; k0 += kG) {
        int64_t jv[kG];
        dd_t av[kG];
        // branch-free (a slot past the row's end re-reads its first element), so all
        // gathers of the group are in flight together
#pragma unroll
        for (int u = 0; u < kG; ++u) {
            const int32_t k = k0 + u < e ? k0 + u : b;
            jv[u] = __builtin_nontemporal_load(ci + k);
            av[u].c[0] = __builtin_nontemporal_load(a + k);
            av[u].c[1] = __builtin_nontemporal_load(a + nnz + k);
        }
        dd_t xv[kG][RPT];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) xv[u][q] = bld(X, NR, jv[u], R, r0 + q);
        }
#pragma unroll
        for (int u = 0; u < kG; ++u)
            if (k0 + u < e) {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const dd_t p = dd_mul(av[u], xv[u][q]);
                    acc[q] = (k0 + u == b) ? p : dd_add(acc[q], p);
                }
            }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) bst(Y, NR, row, R, r0 + q, acc[q]);
}

// ---------------------------------------------------------------------------
// reductions over the rows of one system
// ---------------------------------------------------------------------------

// Chunk workgroups: kBLanes lanes x tpl(R) threads per lane.  Thread t serves lane
// t / tpl and right-hand sides r = t % tpl + tpl*i (i < R / tpl), so the threads of a
// wavefront read the R adjacent values of consecutive rows together (coalesced), while
// every (lane, right-hand side) still accumulates its rows in order.
template <int R>
struct BMap {
    static constexpr int TPL = R < 4 ? R : 4;   // threads per lane
    static constexpr int RPT = R / TPL;         // right-hand sides per thread
    static constexpr int THREADS = kBLanes * TPL;
    __device__ static int lane() { return threadIdx.x / TPL; }
    __device__ static int rhs(int i) { return threadIdx.x % TPL + TPL * i; }
};

// fold the lane sums (lanes [0, used) hold values): lds[l][r] += lds[l + off][r] for
// off = 128 .. 1; out[r] = lds[0][r]
template <int R>
__device__ __forceinline__ void bfold(const dd_t (&acc)[BMap<R>::RPT], int used, dd_t (*lds)[R], dd_t *out)
{
    using M = BMap<R>;
    const int l = M::lane();
#pragma unroll
    for (int i = 0; i < M::RPT; ++i) lds[l][M::rhs(i)] = acc[i];
    __syncthreads();
    for (int off = kBLanes / 2; off >= 1; off >>= 1) {
        if (l < off && l + off < used) {
#pragma unroll
            for (int i = 0; i < M::RPT; ++i) lds[l][M::rhs(i)] = dd_add(lds[l][M::rhs(i)], lds[l + off][M::rhs(i)]);
        }
        __syncthreads();
    }
    if (threadIdx.x < R) out[threadIdx.x] = lds[0][threadIdx.x];
    __syncthreads();
}

struct ChunkInfo {
    int64_t row0;
    int32_t used;   // lanes holding rows
    int64_t end;
    int32_t sys;
};

__device__ __forceinline__ ChunkInfo chunk_info(int c, const int32_t *__restrict__ chunk_row,
                                                const int32_t *__restrict__ chunk_sys, const int32_t *__restrict__ sys_ptr)
{
    ChunkInfo ch;
    ch.sys = chunk_sys[c];
    ch.row0 = chunk_row[c];
    const int64_t sys_end = sys_ptr[ch.sys + 1];
    ch.end = (sys_end - ch.row0) < kBChunk ? sys_end : ch.row0 + kBChunk;
    const int64_t cnt = ch.end - ch.row0;
    ch.used = cnt < kBLanes ? (int)cnt : kBLanes;
    return ch;
}

// chunk sums of (X1, Y1) and optionally (X2, Y2), every right-hand side
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bdot2(int32_t n, const double *__restrict__ X1,
                                                            const double *__restrict__ Y1,
                                                            const double *__restrict__ X2,
                                                            const double *__restrict__ Y2, dd_t *__restrict__ part1,
                                                            dd_t *__restrict__ part2,
                                                            const int32_t *__restrict__ chunk_row,
                                                            const int32_t *__restrict__ chunk_sys,
                                                            const int32_t *__restrict__ sys_ptr)
{
    using M = BMap<R>;
    __shared__ dd_t lds[kBLanes][R];
    const int c = blockIdx.x;
    const ChunkInfo ch = chunk_info(c, chunk_row, chunk_sys, sys_ptr);
    const int64_t NR = (int64_t)n * R;
    dd_t a1[M::RPT], a2[M::RPT];
#pragma unroll
    for (int i = 0; i < M::RPT; ++i) a1[i] = a2[i] = bz();
    bool first = true;
    for (int64_t k = ch.row0 + M::lane(); k < ch.end; k += kBLanes) {
#pragma unroll
        for (int i = 0; i < M::RPT; ++i) {
            const int r = M::rhs(i);
            const dd_t p1 = dd_mul(bld(X1, NR, k, R, r), bld(Y1, NR, k, R, r));
            a1[i] = first ? p1 : dd_add(a1[i], p1);
            if (X2) {
                const dd_t p2 = dd_mul(bld(X2, NR, k, R, r), bld(Y2, NR, k, R, r));
                a2[i] = first ? p2 : dd_add(a2[i], p2);
            }
        }
        first = false;
    }
    bfold<R>(a1, ch.used, lds, part1 + (int64_t)c * R);
    if (X2) bfold<R>(a2, ch.used, lds, part2 + (int64_t)c * R);
}

// pairwise tree over the chunk sums [c0, c0+m) of right-hand side r (single workgroup)
template <int R>
__device__ __forceinline__ dd_t bpair_tree(const dd_t *__restrict__ part, int c0, int m, int r, dd_t *P)
{
    const int t = threadIdx.x;
    for (int i = t; i < m; i += kBLanes) P[i] = part[(int64_t)(c0 + i) * R + r];
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        for (int i = t; (int64_t)i * 2 * s + s < m; i += kBLanes) P[i * 2 * s] = dd_add(P[i * 2 * s], P[i * 2 * s + s]);
        __syncthreads();
    }
    const dd_t v = m > 0 ? P[0] : bz();
    __syncthreads();
    return v;
}

// ---------------------------------------------------------------------------
// element-wise kernels (one thread per row, all right-hand sides)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t row_system(const int32_t *__restrict__ sys_ptr, int nsys, int64_t row)
{
    int lo = 0, hi = nsys;   // largest s with sys_ptr[s] <= row
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sys_ptr[mid] <= row) lo = mid;
        else hi = mid;
    }
    return lo;
}

// R = B - Q for pairs in state `want` (all pairs when want < 0); one thread per
// (row, right-hand side), right-hand sides fastest (coalesced)
template <int R>
__global__ __launch_bounds__(256) void k_bresidual(int32_t n, const double *__restrict__ B, const double *__restrict__ Q,
                                                   double *__restrict__ Rv, const int32_t *__restrict__ sys_ptr, int nsys,
                                                   const BState *__restrict__ st, int want)
{
    const int64_t NR = (int64_t)n * R;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < NR; g += (int64_t)gridDim.x * 256) {
        const int64_t row = g / R;
        const int r = (int)(g % R);
        if (want >= 0 && st[row_system(sys_ptr, nsys, row) * R + r].done != want) continue;
        bst(Rv, NR, row, R, r, dd_add(bld(B, NR, row, R, r), mp_neg(bld(Q, NR, row, R, r))));
    }
}

// Z = M^-1 R and P = Z for pairs in state `want` (all when want < 0)
template <int R>
__global__ __launch_bounds__(256) void k_bprecond_copy(int32_t n, const double *__restrict__ minv,
                                                       const double *__restrict__ Rv, double *__restrict__ Z,
                                                       double *__restrict__ P, const int32_t *__restrict__ sys_ptr,
                                                       int nsys, const BState *__restrict__ st, int want)
{
    const int64_t NR = (int64_t)n * R;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < NR; g += (int64_t)gridDim.x * 256) {
        const int64_t row = g / R;
        const int r = (int)(g % R);
        if (want >= 0 && st[row_system(sys_ptr, nsys, row) * R + r].done != want) continue;
        const dd_t rv = bld(Rv, NR, row, R, r);
        const dd_t z = minv ? dd_mul_d(rv, minv[row]) : rv;
        bst(Z, NR, row, R, r, z);
        bst(P, NR, row, R, r, z);
    }
}

__global__ __launch_bounds__(256) void k_bjacobi(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ a_hi,
                                                 double *__restrict__ minv)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double m = 1.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) m = 1.0 / a_hi[k];
        minv[i] = m;
    }
}

// ---------------------------------------------------------------------------
// per-system finals (one workgroup per system, every right-hand side)
// ---------------------------------------------------------------------------

template <int R>
__global__ __launch_bounds__(256) void k_binit(const dd_t *__restrict__ pbb, const dd_t *__restrict__ prz,
                                               const dd_t *__restrict__ prr, const int32_t *__restrict__ sys_chunk,
                                               double rtol2, int32_t max_iter, BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        const dd_t bb = bpair_tree<R>(pbb, c0, m, r, P);
        const dd_t rz = bpair_tree<R>(prz, c0, m, r, P);
        const dd_t rr = bpair_tree<R>(prr, c0, m, r, P);
        if (threadIdx.x == 0) {
            BState &q = st[s * R + r];
            q.bb = bb;
            q.tol2 = dd_mul_d(bb, rtol2);
            q.rho = rz;
            q.rr = rr;
            q.iters = 0;
            q.restarts = 0;
            q.done = dd_le(rr, q.tol2) ? B_RECURRENCE_MET : (max_iter <= 0 ? B_ITER_LIMIT : B_RUN);
        }
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_balpha(const dd_t *__restrict__ ppq, const int32_t *__restrict__ sys_chunk,
                                                BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        if (st[s * R + r].done != B_RUN) continue;   // uniform in the workgroup
        const dd_t pq = bpair_tree<R>(ppq, c0, m, r, P);
        if (threadIdx.x == 0) {
            BState &q = st[s * R + r];
            q.pq = pq;
            if (!(pq.c[0] > 0.0) || !isfinite(pq.c[0]))
                q.done = B_BROKE_DOWN;
            else
                q.alpha = dd_div(q.rho, pq);
        }
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_bbeta(const dd_t *__restrict__ prz, const dd_t *__restrict__ prr,
                                               const int32_t *__restrict__ sys_chunk, int32_t max_iter,
                                               BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        if (st[s * R + r].done != B_RUN) continue;
        const dd_t rz = bpair_tree<R>(prz, c0, m, r, P);
        const dd_t rr = bpair_tree<R>(prr, c0, m, r, P);
        if (threadIdx.x == 0) {
            BState &q = st[s * R + r];
            q.iters += 1;
            q.rr = rr;
            if (!isfinite(rr.c[0]) || !isfinite(rz.c[0])) {
                q.done = B_BROKE_DOWN;
            } else {
                q.beta = dd_div(rz, q.rho);
                q.rho = rz;
                if (dd_le(rr, q.tol2))
                    q.done = B_RECURRENCE_MET;
                else if (q.iters >= max_iter)
                    q.done = B_ITER_LIMIT;
            }
        }
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_bconfirm(const dd_t *__restrict__ prr, const int32_t *__restrict__ sys_chunk,
                                                  BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        if (st[s * R + r].done != B_RECURRENCE_MET) continue;
        const dd_t rr = bpair_tree<R>(prr, c0, m, r, P);
        if (threadIdx.x == 0) {
            BState &q = st[s * R + r];
            q.rr_true = rr;
            if (dd_le(rr, q.tol2)) {
                q.done = B_CONFIRMED;
            } else {
                q.rr = rr;
                q.restarts += 1;
                q.done = B_RESTART;
            }
        }
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_brestart(const dd_t *__restrict__ prz, const int32_t *__restrict__ sys_chunk,
                                                  int32_t max_iter, BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        if (st[s * R + r].done != B_RESTART) continue;
        const dd_t rz = bpair_tree<R>(prz, c0, m, r, P);
        if (threadIdx.x == 0) {
            BState &q = st[s * R + r];
            q.rho = rz;
            q.done = q.iters >= max_iter ? B_ITER_LIMIT : B_RUN;
        }
        __syncthreads();
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_bexit(const dd_t *__restrict__ prr, const int32_t *__restrict__ sys_chunk,
                                               BState *__restrict__ st)
{
    __shared__ dd_t P[kBMaxSysChunks];
    const int s = blockIdx.x;
    const int c0 = sys_chunk[s], m = sys_chunk[s + 1] - c0;
    for (int r = 0; r < R; ++r) {
        const dd_t rr = bpair_tree<R>(prr, c0, m, r, P);
        if (threadIdx.x == 0) st[s * R + r].rr_true = rr;
    }
}

// ---------------------------------------------------------------------------
// per-chunk update kernels
// ---------------------------------------------------------------------------

// x += alpha p; r -= alpha q; chunk sums of (r, z), (r, r) with z = M^-1 r -- running
// pairs.  z is not stored: k_bp forms it again from r by the same operation.
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bupdate(int32_t n, double *__restrict__ X,
                                                              double *__restrict__ Rv,
                                                              const double *__restrict__ P,
                                                              const double *__restrict__ Q,
                                                              const double *__restrict__ minv,
                                                              dd_t *__restrict__ prz, dd_t *__restrict__ prr,
                                                              const int32_t *__restrict__ chunk_row,
                                                              const int32_t *__restrict__ chunk_sys,
                                                              const int32_t *__restrict__ sys_ptr,
                                                              const BState *__restrict__ st)
{
    using M = BMap<R>;
    __shared__ dd_t lds[kBLanes][R];
    __shared__ int s_any;
    const int c = blockIdx.x;
    const ChunkInfo ch = chunk_info(c, chunk_row, chunk_sys, sys_ptr);
    const int64_t NR = (int64_t)n * R;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int r = 0; r < R; ++r) any |= st[ch.sys * R + r].done == B_RUN;
        s_any = any;
    }
    __syncthreads();
    if (!s_any) return;   // uniform in the workgroup
    bool run[M::RPT];
    dd_t alpha[M::RPT], arz[M::RPT], arr[M::RPT];
#pragma unroll
    for (int i = 0; i < M::RPT; ++i) {
        run[i] = st[ch.sys * R + M::rhs(i)].done == B_RUN;
        alpha[i] = st[ch.sys * R + M::rhs(i)].alpha;
        arz[i] = arr[i] = bz();
    }
    bool first = true;
    for (int64_t k = ch.row0 + M::lane(); k < ch.end; k += kBLanes) {
        const double mi = minv ? minv[k] : 1.0;
#pragma unroll
        for (int i = 0; i < M::RPT; ++i) {
            if (!run[i]) continue;
            const int r = M::rhs(i);
            const dd_t xk = bld(X, NR, k, R, r), pk = bld(P, NR, k, R, r);
            const dd_t rk0 = bld(Rv, NR, k, R, r), qk = bld(Q, NR, k, R, r);
            bst(X, NR, k, R, r, dd_add(xk, dd_mul(alpha[i], pk)));
            const dd_t rk = dd_add(rk0, mp_neg(dd_mul(alpha[i], qk)));
            bst(Rv, NR, k, R, r, rk);
            const dd_t zk = minv ? dd_mul_d(rk, mi) : rk;
            const dd_t p1 = dd_mul(rk, zk), p2 = dd_mul(rk, rk);
            arz[i] = first ? p1 : dd_add(arz[i], p1);
            arr[i] = first ? p2 : dd_add(arr[i], p2);
        }
        first = false;
    }
    bfold<R>(arz, ch.used, lds, prz + (int64_t)c * R);
    bfold<R>(arr, ch.used, lds, prr + (int64_t)c * R);
}

// p = z + beta p with z = M^-1 r (minv NULL: z = r) -- running pairs
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bp(int32_t n, const double *__restrict__ Rv,
                                                         const double *__restrict__ minv, double *__restrict__ P,
                                                         const int32_t *__restrict__ chunk_row,
                                                         const int32_t *__restrict__ chunk_sys,
                                                         const int32_t *__restrict__ sys_ptr,
                                                         const BState *__restrict__ st)
{
    using M = BMap<R>;
    const int c = blockIdx.x;
    const ChunkInfo ch = chunk_info(c, chunk_row, chunk_sys, sys_ptr);
    const int64_t NR = (int64_t)n * R;
    bool run[M::RPT];
    dd_t beta[M::RPT];
#pragma unroll
    for (int i = 0; i < M::RPT; ++i) {
        run[i] = st[ch.sys * R + M::rhs(i)].done == B_RUN;
        beta[i] = st[ch.sys * R + M::rhs(i)].beta;
    }
    for (int64_t k = ch.row0 + M::lane(); k < ch.end; k += kBLanes) {
        const double mi = minv ? minv[k] : 1.0;
#pragma unroll
        for (int i = 0; i < M::RPT; ++i) {
            const int r = M::rhs(i);
            if (run[i]) {
                const dd_t rk = bld(Rv, NR, k, R, r);
                const dd_t zk = minv ? dd_mul_d(rk, mi) : rk;
                bst(P, NR, k, R, r, dd_add(zk, dd_mul(beta[i], bld(P, NR, k, R, r))));
            }
        }
    }
}

// block-diagonal check: every element's column inside its row's system
__global__ __launch_bounds__(256) void k_bcheck(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const int32_t *__restrict__ sys_ptr, int nsys, int32_t *__restrict__ bad)
{
    for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < n; row += (int64_t)gridDim.x * 256) {
        const int s = row_system(sys_ptr, nsys, row);
        const int32_t lo = sys_ptr[s], hi = sys_ptr[s + 1];
        for (int32_t k = rp[row]; k < rp[row + 1]; ++k)
            if (ci[k] < lo || ci[k] >= hi) atomicMin(bad, (int32_t)row);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

inline size_t bal(size_t b) { return (b + 255) & ~(size_t)255; }

template <int R, int TPR>
void launch_bspmm_t(const mp_csr *A, const double *a, const double *X, double *Y, hipStream_t s)
{
    const int64_t threads = (int64_t)A->n_rows * TPR;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL((k_bspmm<R, TPR>), dim3(blocks), dim3(256), 0, s, A->n_rows, A->row_ptr, A->col_idx, a, A->nnz,
                       X, Y);
}

template <int R>
mp_status launch_bspmm_r(int tpr, const mp_csr *A, const double *a, const double *X, double *Y, hipStream_t s)
{
    if (A->n_rows == 0) return MP_OK;
    if (tpr == 1) launch_bspmm_t<R, 1>(A, a, X, Y, s);
    else if (tpr == 2 && R >= 2) launch_bspmm_t<R, (R >= 2 ? 2 : 1)>(A, a, X, Y, s);
    else if (tpr == 4 && R >= 4) launch_bspmm_t<R, (R >= 4 ? 4 : 1)>(A, a, X, Y, s);
    else if (tpr == 8 && R >= 8) launch_bspmm_t<R, (R >= 8 ? 8 : 1)>(A, a, X, Y, s);
    else return fail(MP_ERR_INVALID_ARG, "invalid threads-per-row %d for %d right-hand sides", tpr, R);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

mp_status launch_bspmm(int R, int tpr, const mp_csr *A, const double *a, const double *X, double *Y, hipStream_t s)
{
    switch (R) {
        case 1: return launch_bspmm_r<1>(tpr, A, a, X, Y, s);
        case 2: return launch_bspmm_r<2>(tpr, A, a, X, Y, s);
        case 4: return launch_bspmm_r<4>(tpr, A, a, X, Y, s);
        case 8: return launch_bspmm_r<8>(tpr, A, a, X, Y, s);
        default: return fail(MP_ERR_INVALID_ARG, "nrhs must be 1, 2, 4 or 8 (got %d)", R);
    }
}

void bplan_free(mp_batch_plan *p)
{
    if (!p) return;
    if (p->d_sys_ptr) (void)hipFree(p->d_sys_ptr);
    if (p->d_sys_chunk) (void)hipFree(p->d_sys_chunk);
    if (p->d_chunk_row) (void)hipFree(p->d_chunk_row);
    if (p->d_chunk_sys) (void)hipFree(p->d_chunk_sys);
    delete p;
}

template <typename T>
mp_status bupload(const std::vector<T> &h, T **d, hipStream_t s)
{
    *d = nullptr;
    if (h.empty()) return MP_OK;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(d), h.size() * sizeof(T)));
    MP_HIP_TRY(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return MP_OK;
}

size_t batch_ws_bytes(const mp_batch_plan *p)
{
    const size_t vec = sizeof(double) * 2 * (size_t)p->n_rows * p->nrhs;
    size_t b = 4 * bal(vec);                                          // R, Z, P, Q
    b += bal(sizeof(double) * (size_t)p->n_rows);                     // minv
    b += 3 * bal(sizeof(dd_t) * (size_t)p->n_chunks * p->nrhs);       // chunk sums
    b += bal(sizeof(BState) * (size_t)p->nsys * p->nrhs);             // pair states
    return b;
}

// Batched CG driver: one instance per call.
template <int R>
struct BatchCG {
    const mp_csr *A;
    const double *a;
    const mp_batch_plan *p;
    hipStream_t s;
    int every;
    double *Rv, *Z, *P, *Q, *minv;
    dd_t *part[3];
    BState *st;
    unsigned vblocks;

    mp_status launched()
    {
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
    mp_status spmm(const double *X, double *Y) { return launch_bspmm_r<R>(p->tpr, A, a, X, Y, s); }
    void dot2(const double *X1, const double *Y1, const double *X2, const double *Y2, dd_t *p1, dd_t *p2)
    {
        hipLaunchKernelGGL(k_bdot2<R>, dim3(p->n_chunks), dim3(BMap<R>::THREADS), 0, s, A->n_rows, X1, Y1, X2, Y2, p1,
                           p2,
                           p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr);
    }
    // one CG step for every running pair
    mp_status step(double *X, int max_iter)
    {
        mp_status stt = spmm(P, Q);
        if (stt != MP_OK) return stt;
        dot2(P, Q, nullptr, nullptr, part[0], nullptr);
        hipLaunchKernelGGL(k_balpha<R>, dim3(p->nsys), dim3(256), 0, s, part[0], p->d_sys_chunk, st);
        hipLaunchKernelGGL(k_bupdate<R>, dim3(p->n_chunks), dim3(BMap<R>::THREADS), 0, s, A->n_rows, X, Rv, P, Q, minv,
                           part[1], part[2], p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr, st);
        hipLaunchKernelGGL(k_bbeta<R>, dim3(p->nsys), dim3(256), 0, s, part[1], part[2], p->d_sys_chunk, max_iter, st);
        hipLaunchKernelGGL(k_bp<R>, dim3(p->n_chunks), dim3(BMap<R>::THREADS), 0, s, A->n_rows, Rv, minv, P,
                           p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr, st);
        return launched();
    }
    mp_status true_residual(const double *B, const double *X, int want)
    {
        mp_status stt = spmm(X, Q);
        if (stt != MP_OK) return stt;
        hipLaunchKernelGGL(k_bresidual<R>, dim3(vblocks), dim3(256), 0, s, A->n_rows, B, Q, Rv, p->d_sys_ptr, p->nsys,
                           st, want);
        dot2(Rv, Rv, nullptr, nullptr, part[2], nullptr);
        return launched();
    }
};

template <int R>
mp_status run_batched(const mp_csr *A, const double *a, const double *B, double *X, const mp_solve_opts *o,
                      const mp_batch_plan *p, void *ws, int use_graph, mp_solve_info *info, hipStream_t caller)
{
    const auto t0 = std::chrono::steady_clock::now();
    BatchCG<R> S;
    S.A = A;
    S.a = a;
    S.p = p;
    S.every = o->check_every > 0 ? o->check_every : 32;
    const int64_t vb = ((int64_t)A->n_rows + 255) / 256;
    S.vblocks = (unsigned)(vb < 16384 ? vb : 16384);
    char *w = static_cast<char *>(ws);
    const size_t vec = sizeof(double) * 2 * (size_t)A->n_rows * R;
    double **vs[4] = {&S.Rv, &S.Z, &S.P, &S.Q};
    for (int i = 0; i < 4; ++i) {
        *vs[i] = reinterpret_cast<double *>(w);
        w += bal(vec);
    }
    S.minv = reinterpret_cast<double *>(w);
    w += bal(sizeof(double) * (size_t)A->n_rows);
    for (int i = 0; i < 3; ++i) {
        S.part[i] = reinterpret_cast<dd_t *>(w);
        w += bal(sizeof(dd_t) * (size_t)p->n_chunks * R);
    }
    S.st = reinterpret_cast<BState *>(w);
    const int npairs = p->nsys * R;
    const bool jacobi = o->precond == MP_PRECOND_JACOBI;

    // private stream (a graph cannot be captured on the legacy default stream)
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    MP_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    S.s = s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BState> h((size_t)npairs);
    mp_status st = MP_OK;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev) (void)hipEventDestroy(ev);
        if (s) (void)hipStreamDestroy(s);
    };
#define BTRY(call)                           \
    do {                                     \
        hipError_t e_ = (call);              \
        if (e_ != hipSuccess) {              \
            cleanup();                       \
            return hip_fail(e_, #call);      \
        }                                    \
    } while (0)
#define BST(call)                            \
    do {                                     \
        st = (call);                         \
        if (st != MP_OK) {                   \
            cleanup();                       \
            return st;                       \
        }                                    \
    } while (0)
    BTRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BTRY(hipEventRecord(ev, caller));
    BTRY(hipStreamWaitEvent(s, ev, 0));
    // start: R = B - A X, Z = M^-1 R, P = Z, per-pair bb, rho, rr
    if (jacobi) {
        hipLaunchKernelGGL(k_bjacobi, dim3(S.vblocks), dim3(256), 0, s, A->n_rows, A->row_ptr, A->col_idx, a, S.minv);
        BST(S.launched());
    }
    const double *minv = jacobi ? S.minv : nullptr;
    S.minv = const_cast<double *>(minv);
    BST(S.true_residual(B, X, -1));
    hipLaunchKernelGGL(k_bprecond_copy<R>, dim3(S.vblocks), dim3(256), 0, s, A->n_rows, minv, S.Rv, S.Z, S.P,
                       p->d_sys_ptr, p->nsys, S.st, -1);
    S.dot2(B, B, S.Rv, S.Z, S.part[0], S.part[1]);
    hipLaunchKernelGGL(k_binit<R>, dim3(p->nsys), dim3(256), 0, s, S.part[0], S.part[1], S.part[2], p->d_sys_chunk,
                       o->rtol * o->rtol, o->max_iter, S.st);
    BST(S.launched());
    if (use_graph) {
        BTRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < S.every; ++it) {
            st = S.step(X, o->max_iter);
            if (st != MP_OK) break;
        }
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (st != MP_OK) {
            cleanup();
            return st;
        }
        BTRY(ce);
        BTRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    for (;;) {
        BTRY(hipMemcpyAsync(h.data(), S.st, sizeof(BState) * npairs, hipMemcpyDeviceToHost, s));
        BTRY(hipStreamSynchronize(s));
        int nrun = 0, nmet = 0, nrestart = 0;
        for (const BState &q : h) {
            nrun += q.done == B_RUN;
            nmet += q.done == B_RECURRENCE_MET;
            nrestart += q.done == B_RESTART;
        }
        if (nmet > 0) {
            BST(S.true_residual(B, X, B_RECURRENCE_MET));
            hipLaunchKernelGGL(k_bconfirm<R>, dim3(p->nsys), dim3(256), 0, s, S.part[2], p->d_sys_chunk, S.st);
            BST(S.launched());
            continue;
        }
        if (nrestart > 0) {
            hipLaunchKernelGGL(k_bprecond_copy<R>, dim3(S.vblocks), dim3(256), 0, s, A->n_rows, minv, S.Rv, S.Z, S.P,
                               p->d_sys_ptr, p->nsys, S.st, (int)B_RESTART);
            S.dot2(S.Rv, S.Z, nullptr, nullptr, S.part[1], nullptr);
            hipLaunchKernelGGL(k_brestart<R>, dim3(p->nsys), dim3(256), 0, s, S.part[1], p->d_sys_chunk, o->max_iter,
                               S.st);
            BST(S.launched());
            continue;
        }
        if (nrun == 0) break;
        if (use_graph) {
            BTRY(hipGraphLaunch(exec, s));
        } else {
            for (int it = 0; it < S.every; ++it) BST(S.step(X, o->max_iter));
        }
    }
    // exit record: true residual of every pair
    BST(S.true_residual(B, X, -1));
    hipLaunchKernelGGL(k_bexit<R>, dim3(p->nsys), dim3(256), 0, s, S.part[2], p->d_sys_chunk, S.st);
    BST(S.launched());
    BTRY(hipMemcpyAsync(h.data(), S.st, sizeof(BState) * npairs, hipMemcpyDeviceToHost, s));
    BTRY(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = MP_OK;
    for (int i = 0; i < npairs; ++i) {
        const BState &q = h[i];
        mp_solve_info &f = info[i];
        std::memset(&f, 0, sizeof(f));
        f.status = q.done == B_CONFIRMED ? MP_OK : (q.done == B_BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        f.iters = q.iters;
        f.restarts = q.restarts;
        f.rr_true[0] = q.rr_true.c[0];
        f.rr_true[1] = q.rr_true.c[1];
        f.bb[0] = q.bb.c[0];
        f.bb[1] = q.bb.c[1];
        f.relres = q.bb.c[0] > 0 ? std::sqrt(q.rr_true.c[0] / q.bb.c[0]) : std::sqrt(q.rr_true.c[0]);
        f.seconds = secs;
        if (f.status == MP_ERR_BREAKDOWN) worst = MP_ERR_BREAKDOWN;
        else if (f.status == MP_ERR_NOT_CONVERGED && worst == MP_OK) worst = MP_ERR_NOT_CONVERGED;
    }
    BTRY(hipEventRecord(ev, s));
    BTRY(hipStreamWaitEvent(caller, ev, 0));
    BTRY(hipStreamSynchronize(s));
    cleanup();
#undef BTRY
#undef BST
    if (worst != MP_OK) return fail((mp_status)worst, "mpkrylov_cg_batched: some pairs did not converge");
    return MP_OK;
}

}  // namespace mpk

extern "C" {

mp_status mp_batch_plan_create(const mp_csr *A, const int32_t *sys_ptr_host, int32_t nsys, int32_t nrhs,
                               int32_t threads_per_row, void *stream, mp_batch_plan **out)
{
    using namespace mpk;
    clear_error();
    if (!out) return fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (nsys < 1 || !sys_ptr_host) return fail(MP_ERR_INVALID_ARG, "need nsys >= 1 and sys_ptr");
    if (A->n_rows != A->n_cols) return fail(MP_ERR_INVALID_ARG, "block-diagonal matrix must be square");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4 && nrhs != 8) return fail(MP_ERR_INVALID_ARG, "nrhs must be 1, 2, 4 or 8");
    if (threads_per_row < 1 || threads_per_row > nrhs || (threads_per_row & (threads_per_row - 1)))
        return fail(MP_ERR_INVALID_ARG, "threads_per_row must be a power of two <= nrhs");
    if (sys_ptr_host[0] != 0 || sys_ptr_host[nsys] != A->n_rows)
        return fail(MP_ERR_INVALID_ARG, "sys_ptr must start at 0 and end at n_rows");
    mp_batch_plan *p = new (std::nothrow) mp_batch_plan;
    if (!p) return fail(MP_ERR_NO_MEMORY, "plan allocation failed");
    p->n_rows = A->n_rows;
    p->nnz = A->nnz;
    p->nsys = nsys;
    p->nrhs = nrhs;
    p->tpr = threads_per_row;
    p->sys_ptr.assign(sys_ptr_host, sys_ptr_host + nsys + 1);
    std::vector<int32_t> sys_chunk((size_t)nsys + 1), chunk_row, chunk_sys;
    for (int32_t s = 0; s < nsys; ++s) {
        if (p->sys_ptr[s + 1] <= p->sys_ptr[s]) {
            bplan_free(p);
            return fail(MP_ERR_INVALID_ARG, "system %d is empty or sys_ptr decreases", s);
        }
        sys_chunk[s] = (int32_t)chunk_row.size();
        for (int64_t r0 = p->sys_ptr[s]; r0 < p->sys_ptr[s + 1]; r0 += kBChunk) {
            chunk_row.push_back((int32_t)r0);
            chunk_sys.push_back(s);
        }
        const int nc = (int)chunk_row.size() - sys_chunk[s];
        if (nc > kBMaxSysChunks) {
            bplan_free(p);
            return fail(MP_ERR_UNSUPPORTED, "system %d has more than %d rows", s, kBMaxSysChunks * kBChunk);
        }
        p->max_sys_chunks = std::max(p->max_sys_chunks, nc);
    }
    sys_chunk[nsys] = (int32_t)chunk_row.size();
    p->n_chunks = (int32_t)chunk_row.size();
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = bupload(p->sys_ptr, &p->d_sys_ptr, s);
    if (st == MP_OK) st = bupload(sys_chunk, &p->d_sys_chunk, s);
    if (st == MP_OK) st = bupload(chunk_row, &p->d_chunk_row, s);
    if (st == MP_OK) st = bupload(chunk_sys, &p->d_chunk_sys, s);
    int32_t *d_bad = nullptr;
    int32_t h_bad = INT32_MAX;
    if (st == MP_OK) {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&d_bad), sizeof(int32_t));
        if (e == hipSuccess) e = hipMemcpyAsync(d_bad, &h_bad, sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            const int64_t vb = ((int64_t)A->n_rows + 255) / 256;
            hipLaunchKernelGGL(k_bcheck, dim3((unsigned)(vb < 16384 ? vb : 16384)), dim3(256), 0, s, A->n_rows,
                               A->row_ptr, A->col_idx, p->d_sys_ptr, nsys, d_bad);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (d_bad) (void)hipFree(d_bad);
        if (e != hipSuccess) st = hip_fail(e, "block-diagonal check");
        else if (h_bad != INT32_MAX) st = fail(MP_ERR_INVALID_ARG, "row %d has an entry outside its system's block", h_bad);
    }
    if (st != MP_OK) {
        bplan_free(p);
        return st;
    }
    *out = p;
    return MP_OK;
}

mp_status mp_batch_plan_destroy(mp_batch_plan *plan)
{
    mpk::clear_error();
    mpk::bplan_free(plan);
    return MP_OK;
}

mp_status mp_batch_plan_autotune(mp_batch_plan *plan, const mp_csr *A, const double *a, const double *X, double *Y,
                                 int32_t reps, void *stream, int32_t *threads_per_row)
{
    using namespace mpk;
    clear_error();
    if (!plan || !A || (A->nnz > 0 && (!a || !X || !Y))) return fail(MP_ERR_INVALID_ARG, "NULL argument");
    if (plan->n_rows != A->n_rows || plan->nnz != A->nnz) return fail(MP_ERR_INVALID_ARG, "plan does not match A");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    MP_HIP_TRY(hipEventCreate(&e0));
    MP_HIP_TRY(hipEventCreate(&e1));
    float best = -1.f;
    int best_tpr = plan->tpr;
    mp_status st = MP_OK;
    for (int tpr = 1; tpr <= plan->nrhs && st == MP_OK; tpr <<= 1) {
        st = launch_bspmm(plan->nrhs, tpr, A, a, X, Y, s);
        if (st != MP_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < (reps > 0 ? reps : 3) && st == MP_OK; ++r) st = launch_bspmm(plan->nrhs, tpr, A, a, X, Y, s);
        (void)hipEventRecord(e1, s);
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) st = hip_fail(e, "batched autotune timing");
        if (st == MP_OK && (best < 0.f || ms < best)) {
            best = ms;
            best_tpr = tpr;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MP_OK) return st;
    plan->tpr = best_tpr;
    if (threads_per_row) *threads_per_row = best_tpr;
    return MP_OK;
}

mp_status mpspmm_csr_dd_batched(const mp_csr *A, const double *a, const double *X, double *Y, int32_t nrhs,
                                const mp_batch_plan *plan, void *stream)
{
    using namespace mpk;
    clear_error();
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (nrhs != 1 && nrhs != 2 && nrhs != 4 && nrhs != 8) return fail(MP_ERR_INVALID_ARG, "nrhs must be 1, 2, 4 or 8");
    if (A->n_rows > 0 && (!X || !Y)) return fail(MP_ERR_INVALID_ARG, "X or Y is NULL");
    if (A->nnz > 0 && !a) return fail(MP_ERR_INVALID_ARG, "a is NULL");
    if (plan && (plan->n_rows != A->n_rows || plan->nnz != A->nnz || plan->nrhs != nrhs))
        return fail(MP_ERR_INVALID_ARG, "batch plan does not match A / nrhs");
    const size_t yb = sizeof(double) * 2 * (size_t)A->n_rows * nrhs;
    const size_t xb = sizeof(double) * 2 * (size_t)A->n_cols * nrhs;
    if (overlaps(Y, yb, X, xb) || overlaps(Y, yb, a, sizeof(double) * 2 * (size_t)A->nnz))
        return fail(MP_ERR_ALIAS, "Y overlaps X or a");
    return launch_bspmm(nrhs, plan ? plan->tpr : 1, A, a, X, Y, static_cast<hipStream_t>(stream));
}

mp_status mpkrylov_batched_workspace_bytes(const mp_batch_plan *plan, size_t *bytes)
{
    mpk::clear_error();
    if (!plan || !bytes) return mpk::fail(MP_ERR_INVALID_ARG, "NULL argument");
    *bytes = mpk::batch_ws_bytes(plan);
    return MP_OK;
}

mp_status mpkrylov_cg_batched(const mp_csr *A, const double *a, const double *B, double *X, int32_t nrhs,
                              const mp_solve_opts *opts, const mp_batch_plan *plan, int32_t use_graph, void *ws,
                              size_t ws_bytes, mp_solve_info *info, void *stream)
{
    using namespace mpk;
    clear_error();
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (!opts || !plan || !info) return fail(MP_ERR_INVALID_ARG, "opts, plan or info is NULL");
    if (plan->n_rows != A->n_rows || plan->nnz != A->nnz || plan->nrhs != nrhs)
        return fail(MP_ERR_INVALID_ARG, "batch plan does not match A / nrhs");
    if (A->n_rows > 0 && (!B || !X || !ws)) return fail(MP_ERR_INVALID_ARG, "B, X or workspace is NULL");
    if (A->nnz > 0 && !a) return fail(MP_ERR_INVALID_ARG, "a is NULL");
    if (ws_bytes < batch_ws_bytes(plan))
        return fail(MP_ERR_NO_MEMORY, "workspace of %zu bytes, %zu needed", ws_bytes, batch_ws_bytes(plan));
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (opts->precond != MP_PRECOND_NONE && opts->precond != MP_PRECOND_JACOBI)
        return fail(MP_ERR_INVALID_ARG, "unknown preconditioner %d", opts->precond);
    const size_t vb = sizeof(double) * 2 * (size_t)A->n_rows * nrhs;
    if (overlaps(X, vb, B, vb) || overlaps(X, vb, ws, ws_bytes) || overlaps(B, vb, ws, ws_bytes) ||
        overlaps(X, vb, a, sizeof(double) * 2 * (size_t)A->nnz))
        return fail(MP_ERR_ALIAS, "X overlaps B, a or the workspace");
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (nrhs) {
        case 1: return run_batched<1>(A, a, B, X, opts, plan, ws, use_graph, info, s);
        case 2: return run_batched<2>(A, a, B, X, opts, plan, ws, use_graph, info, s);
        case 4: return run_batched<4>(A, a, B, X, opts, plan, ws, use_graph, info, s);
        case 8: return run_batched<8>(A, a, B, X, opts, plan, ws, use_graph, info, s);
        default: return fail(MP_ERR_INVALID_ARG, "nrhs must be 1, 2, 4 or 8");
    }
}

}  // extern "C"
