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
// step is four persistent kernels over all pairs, fed by per-XCD work queues (see
// "persistent step kernels" below); a chunk of steps is captured once into a
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
    int32_t rows_mult = 1;    // persistent SpMM: tiles of (256 / tpr) * rows_mult rows
    int32_t chunk_order = 0;  // 0: dot chunks in row order; 1: largest systems first
    int32_t n_chunks = 0;     // dot chunks (<= 4096 rows of one system)
    int32_t max_sys_chunks = 0;
    int32_t *d_sys_ptr = nullptr;
    int32_t *d_sys_chunk = nullptr;   // nsys + 1: first chunk of each system
    int32_t *d_chunk_row = nullptr;   // n_chunks: first row of each chunk
    int32_t *d_chunk_sys = nullptr;   // n_chunks: system of each chunk
    int32_t *d_chunk_big = nullptr;   // n_chunks: the chunks, largest systems first
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

// one row of Y = A X for right-hand sides r0 .. r0 + R/TPR - 1
template <int R, int TPR>
__device__ __forceinline__ void bspmm_row(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                          const double *__restrict__ a, int64_t nnz, const double *__restrict__ X,
                                          double *__restrict__ Y, int64_t row, int r0)
{
    constexpr int RPT = R / TPR;
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

template <int R, int TPR>
__global__ __launch_bounds__(256) void k_bspmm(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                               const double *__restrict__ a, int64_t nnz, const double *__restrict__ X,
                                               double *__restrict__ Y)
{
    const int64_t g = (int64_t)bxcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t row = g / TPR;
    if (row >= n) return;
    bspmm_row<R, TPR>(n, rp, ci, a, nnz, X, Y, row, (int)(g % TPR) * (R / TPR));
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

// chunk sums of (X1, Y1) and optionally (X2, Y2) of chunk c, every right-hand side
template <int R>
__device__ __forceinline__ void bdot_chunk(int32_t n, const double *__restrict__ X1, const double *__restrict__ Y1,
                                           const double *__restrict__ X2, const double *__restrict__ Y2,
                                           dd_t *__restrict__ part1, dd_t *__restrict__ part2, int c,
                                           const int32_t *__restrict__ chunk_row,
                                           const int32_t *__restrict__ chunk_sys, const int32_t *__restrict__ sys_ptr,
                                           dd_t (*lds)[R])
{
    using M = BMap<R>;
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
    __shared__ dd_t lds[kBLanes][R];
    bdot_chunk<R>(n, X1, Y1, X2, Y2, part1, part2, blockIdx.x, chunk_row, chunk_sys, sys_ptr, lds);
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

// ---------------------------------------------------------------------------
// persistent step kernels
//
// One CG step is four launches: the SpMM over row tiles, the (p, q) chunk sums, the
// update (alpha, x, r and the (r, z), (r, r) chunk sums) and the p step (beta, stop
// tests, p).  Each is a persistent kernel sized to the device's resident occupancy
// whose workgroups take work items -- row tiles, or dot chunks in the plan's order --
// from 8 queues, one per XCD: queue x holds the contiguous range
// [x floor(n/8) + min(x, n mod 8), ...) of the item order, and a workgroup launched on
// XCD x (block index mod 8) takes items from queue x through a vector-memory atomic
// counter, then from the other queues in turn.  No workgroup waits for another, every
// item is taken exactly once, and a workgroup exits after one failed take per queue.
// The per-system scalars (alpha from the (p, q) sums; beta, ||r||^2 and the stop tests
// from the (r, z), (r, r) sums) are formed by every item of the system (the same
// pairwise trees over the system's chunk sums, so the same values), and the system's first chunk
// writes the pair states, double-buffered between the update kernel (reads sa, writes
// sb) and the p kernel (reads sb, writes sa).  Each kernel clears the counters of the
// kernel that follows it in the step (which cannot start before this one ends).
// ---------------------------------------------------------------------------

constexpr int kQueues = 8;

struct BQueue {
    int32_t *cnt;            // this kernel's kQueues counters
    int32_t *cnt_next;       // the next kernel's counters, cleared by this kernel
    const int32_t *order;    // item order (NULL: natural)
    int32_t n_items;
};

__device__ __forceinline__ int32_t bq_begin(int32_t n, int x)
{
    return x * (n / kQueues) + (x < n % kQueues ? x : n % kQueues);
}

// thread 0 only: the next item for this workgroup, or -1; probe = queues exhausted
__device__ __forceinline__ int32_t bq_next(const BQueue &Q, int &probe)
{
    const int home = blockIdx.x & (kQueues - 1);
    while (probe < kQueues) {
        const int qx = (home + probe) & (kQueues - 1);
        const int32_t b = bq_begin(Q.n_items, qx), e = bq_begin(Q.n_items, qx + 1);
        const int32_t k = atomicAdd(&Q.cnt[qx], 1);
        if (b + k < e) return Q.order ? Q.order[b + k] : b + k;
        ++probe;
    }
    return -1;
}

// every thread: the workgroup's next item (-1 when none is left)
__device__ __forceinline__ int32_t bq_take(const BQueue &Q, int &probe, int32_t *s_item)
{
    if (threadIdx.x == 0) *s_item = bq_next(Q, probe);
    __syncthreads();
    const int32_t it = *s_item;
    __syncthreads();
    return it;
}

__device__ __forceinline__ void bq_clear_next(const BQueue &Q)
{
    if (blockIdx.x == 0 && threadIdx.x < kQueues) Q.cnt_next[threadIdx.x] = 0;
}

__global__ __launch_bounds__(64) void k_bfill_i32(int32_t *__restrict__ v, int n, int32_t val)
{
    for (int i = threadIdx.x; i < n; i += 64) v[i] = val;
}

__device__ __forceinline__ dd_t bshfl_down(const dd_t &v, int d)
{
    dd_t r;
    r.c[0] = __shfl_down(v.c[0], d, 64);
    r.c[1] = __shfl_down(v.c[1], d, 64);
    return r;
}

// out[r] = the pairwise tree of part[(c0 + i) * R + r], i < m (bpair_tree's order), for
// every r with want[r]; all threads return after a barrier.  m <= 64: wavefront r alone,
// by lane shuffles (level s: lane l, a multiple of 2s, adds lane l + s when l + s < m);
// otherwise through LDS, one right-hand side after the other.
template <int R>
__device__ __forceinline__ void bq_trees(const dd_t *__restrict__ part, int c0, int m, const int *want, dd_t *out,
                                         dd_t *P)
{
    const int t = threadIdx.x;
    if (m <= 64) {
        const int w = t >> 6, l = t & 63;
        if (w < R && want[w]) {
            dd_t v = l < m ? part[(int64_t)(c0 + l) * R + w] : bz();
            for (int s = 1; s < m; s <<= 1) {
                const dd_t o = bshfl_down(v, s);
                if ((l & (2 * s - 1)) == 0 && l + s < m) v = dd_add(v, o);
            }
            if (l == 0) out[w] = v;
        }
        __syncthreads();
        return;
    }
    for (int r = 0; r < R; ++r) {
        if (!want[r]) continue;   // uniform: want is in LDS
        for (int i = t; i < m; i += blockDim.x) P[i] = part[(int64_t)(c0 + i) * R + r];
        __syncthreads();
        for (int s = 1; s < m; s <<= 1) {
            for (int i = t; (int64_t)i * 2 * s + s < m; i += blockDim.x) P[i * 2 * s] = dd_add(P[i * 2 * s], P[i * 2 * s + s]);
            __syncthreads();
        }
        if (t == 0) out[r] = P[0];
        __syncthreads();
    }
}

// Y = A X over row tiles of (256 / TPR) * U rows
template <int R, int TPR, int U>
__global__ __launch_bounds__(256) void k_bq_spmm(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ a,
                                                 int64_t nnz, const double *__restrict__ X, double *__restrict__ Y,
                                                 BQueue Q)
{
    constexpr int RW = 256 / TPR;   // rows of one pass of the workgroup
    __shared__ int32_t s_item;
    bq_clear_next(Q);
    int probe = 0;
    for (;;) {
        const int32_t item = bq_take(Q, probe, &s_item);
        if (item < 0) break;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = (int64_t)item * (RW * U) + u * RW + threadIdx.x / TPR;
            if (row < n) bspmm_row<R, TPR>(n, rp, ci, a, nnz, X, Y, row, (int)(threadIdx.x % TPR) * (R / TPR));
        }
    }
}

// chunk sums of (P, Q) over dot chunks
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bq_pq(int32_t n, const double *__restrict__ P,
                                                            const double *__restrict__ Qv, dd_t *__restrict__ ppq,
                                                            const int32_t *__restrict__ chunk_row,
                                                            const int32_t *__restrict__ chunk_sys,
                                                            const int32_t *__restrict__ sys_ptr, BQueue Q)
{
    __shared__ dd_t lds[kBLanes][R];
    __shared__ int32_t s_item;
    bq_clear_next(Q);
    int probe = 0;
    for (;;) {
        const int32_t c = bq_take(Q, probe, &s_item);
        if (c < 0) break;
        bdot_chunk<R>(n, P, Qv, nullptr, nullptr, ppq, nullptr, c, chunk_row, chunk_sys, sys_ptr, lds);
    }
}

// alpha = rho / (p, q) per running pair (breakdown unless (p, q) > 0 and finite), then
// r -= alpha q and the chunk sums of (r, z), (r, r) with z = M^-1 r (z is not stored:
// k_bq_p forms it again from r by the same operation), per dot chunk.  x += alpha p is
// left to k_bq_p, which loads p anyway.
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bq_upd(int32_t n, double *__restrict__ Rv,
                                                             const double *__restrict__ Qv,
                                                             const double *__restrict__ minv,
                                                             const dd_t *__restrict__ ppq, dd_t *__restrict__ prz,
                                                             dd_t *__restrict__ prr,
                                                             const int32_t *__restrict__ chunk_row,
                                                             const int32_t *__restrict__ chunk_sys,
                                                             const int32_t *__restrict__ sys_ptr,
                                                             const int32_t *__restrict__ sys_chunk,
                                                             const BState *__restrict__ sa, BState *__restrict__ sb,
                                                             BQueue Q)
{
    using M = BMap<R>;
    __shared__ dd_t lds[kBLanes][R];
    __shared__ dd_t P_[kBMaxSysChunks];
    __shared__ dd_t s_pq[R], s_alpha[R];
    __shared__ int s_want[R], s_run[R];
    __shared__ int32_t s_item;
    bq_clear_next(Q);
    int probe = 0;
    const int64_t NR = (int64_t)n * R;
    for (;;) {
        const int32_t c = bq_take(Q, probe, &s_item);
        if (c < 0) break;
        const ChunkInfo ch = chunk_info(c, chunk_row, chunk_sys, sys_ptr);
        const int c0 = sys_chunk[ch.sys], m = sys_chunk[ch.sys + 1] - c0;
        if (threadIdx.x < R) s_want[threadIdx.x] = sa[ch.sys * R + threadIdx.x].done == B_RUN;
        __syncthreads();
        bq_trees<R>(ppq, c0, m, s_want, s_pq, P_);
        if (threadIdx.x < R) {
            const int r = threadIdx.x;
            BState q = sa[ch.sys * R + r];
            int run = 0;
            if (q.done == B_RUN) {
                const dd_t pq = s_pq[r];
                q.pq = pq;
                if (!(pq.c[0] > 0.0) || !isfinite(pq.c[0])) {
                    q.done = B_BROKE_DOWN;
                } else {
                    q.alpha = dd_div(q.rho, pq);
                    run = 1;
                }
            }
            s_run[r] = run;
            s_alpha[r] = q.alpha;
            if (c == c0) sb[ch.sys * R + r] = q;
        }
        __syncthreads();
        int any = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) any |= s_run[r];
        if (!any) continue;   // uniform in the workgroup
        bool run[M::RPT];
        dd_t alpha[M::RPT], arz[M::RPT], arr[M::RPT];
#pragma unroll
        for (int i = 0; i < M::RPT; ++i) {
            run[i] = s_run[M::rhs(i)] != 0;
            alpha[i] = s_alpha[M::rhs(i)];
            arz[i] = arr[i] = bz();
        }
        bool first = true;
        for (int64_t k = ch.row0 + M::lane(); k < ch.end; k += kBLanes) {
            const double mi = minv ? minv[k] : 1.0;
#pragma unroll
            for (int i = 0; i < M::RPT; ++i) {
                if (!run[i]) continue;
                const int r = M::rhs(i);
                const dd_t rk0 = bld(Rv, NR, k, R, r), qk = bld(Qv, NR, k, R, r);
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
}

// x += alpha p for the pairs k_bq_upd stepped (with the p this kernel loads anyway);
// iterations + 1, ||r||^2, beta = (r, z) / rho and the stop tests per running pair,
// then p = z + beta p for the pairs still running, per dot chunk
template <int R>
__global__ __launch_bounds__(BMap<R>::THREADS) void k_bq_p(int32_t n, double *__restrict__ X,
                                                           const double *__restrict__ Rv,
                                                           const double *__restrict__ minv, double *__restrict__ P,
                                                           const dd_t *__restrict__ prz, const dd_t *__restrict__ prr,
                                                           const int32_t *__restrict__ chunk_row,
                                                           const int32_t *__restrict__ chunk_sys,
                                                           const int32_t *__restrict__ sys_ptr,
                                                           const int32_t *__restrict__ sys_chunk, int32_t max_iter,
                                                           const BState *__restrict__ sb, BState *__restrict__ sa,
                                                           BQueue Q)
{
    using M = BMap<R>;
    __shared__ dd_t P_[kBMaxSysChunks];
    __shared__ dd_t s_rz[R], s_rr[R], s_beta[R], s_alpha[R];
    __shared__ int s_want[R], s_run[R], s_xrun[R];
    __shared__ int32_t s_item;
    bq_clear_next(Q);
    int probe = 0;
    const int64_t NR = (int64_t)n * R;
    for (;;) {
        const int32_t c = bq_take(Q, probe, &s_item);
        if (c < 0) break;
        const ChunkInfo ch = chunk_info(c, chunk_row, chunk_sys, sys_ptr);
        const int c0 = sys_chunk[ch.sys], m = sys_chunk[ch.sys + 1] - c0;
        if (threadIdx.x < R) s_want[threadIdx.x] = sb[ch.sys * R + threadIdx.x].done == B_RUN;
        __syncthreads();
        bq_trees<R>(prz, c0, m, s_want, s_rz, P_);
        bq_trees<R>(prr, c0, m, s_want, s_rr, P_);
        if (threadIdx.x < R) {
            const int r = threadIdx.x;
            BState q = sb[ch.sys * R + r];
            s_xrun[r] = q.done == B_RUN;   // k_bq_upd stepped r with this alpha
            s_alpha[r] = q.alpha;
            if (q.done == B_RUN) {
                const dd_t rz = s_rz[r], rr = s_rr[r];
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
            s_run[r] = q.done == B_RUN;
            s_beta[r] = q.beta;
            if (c == c0) sa[ch.sys * R + r] = q;
        }
        __syncthreads();
        int any = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) any |= s_xrun[r];
        if (!any) {
            __syncthreads();   // s_xrun / s_run / s_alpha / s_beta are rewritten by the next item
            continue;          // uniform in the workgroup
        }
        bool run[M::RPT], xrun[M::RPT];
        dd_t beta[M::RPT], alpha[M::RPT];
#pragma unroll
        for (int i = 0; i < M::RPT; ++i) {
            run[i] = s_run[M::rhs(i)] != 0;
            xrun[i] = s_xrun[M::rhs(i)] != 0;
            beta[i] = s_beta[M::rhs(i)];
            alpha[i] = s_alpha[M::rhs(i)];
        }
        for (int64_t k = ch.row0 + M::lane(); k < ch.end; k += kBLanes) {
            const double mi = minv ? minv[k] : 1.0;
#pragma unroll
            for (int i = 0; i < M::RPT; ++i) {
                const int r = M::rhs(i);
                if (xrun[i]) {
                    const dd_t pk = bld(P, NR, k, R, r);
                    bst(X, NR, k, R, r, dd_add(bld(X, NR, k, R, r), dd_mul(alpha[i], pk)));
                    if (run[i]) {
                        const dd_t rk = bld(Rv, NR, k, R, r);
                        const dd_t zk = minv ? dd_mul_d(rk, mi) : rk;
                        bst(P, NR, k, R, r, dd_add(zk, dd_mul(beta[i], pk)));
                    }
                }
            }
        }
        __syncthreads();   // s_xrun / s_run / s_alpha / s_beta are rewritten by the next item
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
    if (p->d_chunk_big) (void)hipFree(p->d_chunk_big);
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
    b += 2 * bal(sizeof(BState) * (size_t)p->nsys * p->nrhs);         // pair states (double-buffered)
    b += bal(sizeof(int32_t) * 4 * kQueues);                          // queue counters of the step kernels
    return b;
}

// resident workgroups of a kernel on the current device (at least one per compute unit)
template <typename F>
int resident_grid(F kernel, int threads)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
    return cus * per;
}

// grid <= 0: the kernel's resident workgroups (an occupancy query: not under capture)
template <int R, int TPR, int U>
mp_status launch_bq_spmm_t(const mp_csr *A, const double *a, const double *X, double *Y, int32_t *cnt,
                           int32_t *cnt_next, int grid, hipStream_t s)
{
    const int rows = (256 / TPR) * U;
    BQueue Q{cnt, cnt_next, nullptr, (int32_t)(((int64_t)A->n_rows + rows - 1) / rows)};
    if (Q.n_items == 0) return MP_OK;
    if (grid <= 0) grid = resident_grid(k_bq_spmm<R, TPR, U>, 256);
    if (grid > Q.n_items) grid = Q.n_items;
    hipLaunchKernelGGL((k_bq_spmm<R, TPR, U>), dim3(grid), dim3(256), 0, s, A->n_rows, A->row_ptr, A->col_idx, a,
                       A->nnz, X, Y, Q);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

template <int R, int TPR>
mp_status launch_bq_spmm_u(int U, const mp_csr *A, const double *a, const double *X, double *Y, int32_t *cnt,
                           int32_t *cnt_next, int grid, hipStream_t s)
{
    switch (U) {
        case 1: return launch_bq_spmm_t<R, TPR, 1>(A, a, X, Y, cnt, cnt_next, grid, s);
        case 2: return launch_bq_spmm_t<R, TPR, 2>(A, a, X, Y, cnt, cnt_next, grid, s);
        case 4: return launch_bq_spmm_t<R, TPR, 4>(A, a, X, Y, cnt, cnt_next, grid, s);
        default: return fail(MP_ERR_INVALID_ARG, "rows multiple must be 1, 2 or 4 (got %d)", U);
    }
}

// persistent SpMM of the CG step: tiles of (256 / tpr) * U rows from the queues
template <int R>
mp_status launch_bq_spmm(int tpr, int U, const mp_csr *A, const double *a, const double *X, double *Y, int32_t *cnt,
                         int32_t *cnt_next, hipStream_t s, int grid = 0)
{
    if (tpr == 1) return launch_bq_spmm_u<R, 1>(U, A, a, X, Y, cnt, cnt_next, grid, s);
    if (tpr == 2 && R >= 2) return launch_bq_spmm_u<R, (R >= 2 ? 2 : 1)>(U, A, a, X, Y, cnt, cnt_next, grid, s);
    if (tpr == 4 && R >= 4) return launch_bq_spmm_u<R, (R >= 4 ? 4 : 1)>(U, A, a, X, Y, cnt, cnt_next, grid, s);
    if (tpr == 8 && R >= 8) return launch_bq_spmm_u<R, (R >= 8 ? 8 : 1)>(U, A, a, X, Y, cnt, cnt_next, grid, s);
    return fail(MP_ERR_INVALID_ARG, "invalid threads-per-row %d for %d right-hand sides", tpr, R);
}

template <int R, int TPR>
int bq_spmm_grid_u(int U)
{
    switch (U) {
        case 1: return resident_grid(k_bq_spmm<R, TPR, 1>, 256);
        case 2: return resident_grid(k_bq_spmm<R, TPR, 2>, 256);
        default: return resident_grid(k_bq_spmm<R, TPR, 4>, 256);
    }
}

template <int R>
int bq_spmm_grid(int tpr, int U)
{
    if (tpr == 2 && R >= 2) return bq_spmm_grid_u<R, (R >= 2 ? 2 : 1)>(U);
    if (tpr == 4 && R >= 4) return bq_spmm_grid_u<R, (R >= 4 ? 4 : 1)>(U);
    if (tpr == 8 && R >= 8) return bq_spmm_grid_u<R, (R >= 8 ? 8 : 1)>(U);
    return bq_spmm_grid_u<R, 1>(U);
}

template <int R>
BQueue chunk_queue(const mp_batch_plan *p, int32_t *cnt, int32_t *cnt_next)
{
    return BQueue{cnt, cnt_next, p->chunk_order ? p->d_chunk_big : nullptr, p->n_chunks};
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
    BState *st2;     // the second buffer of the pair states inside a step
    int32_t *cnt;    // queue counters: SpMM, (p, q) sums, update, p step
    unsigned vblocks;
    int grid_c;      // resident workgroups of the chunk kernels
    int grid_s;      // resident workgroups of the plan's SpMM kernel

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
    // one CG step for every running pair: four persistent kernels
    mp_status step(double *X, int max_iter)
    {
        int32_t *c0 = cnt, *c1 = cnt + kQueues, *c2 = cnt + 2 * kQueues, *c3 = cnt + 3 * kQueues;
        mp_status stt = launch_bq_spmm<R>(p->tpr, p->rows_mult, A, a, P, Q, c0, c1, s, grid_s);
        if (stt != MP_OK) return stt;
        const int g = grid_c < p->n_chunks ? grid_c : p->n_chunks;
        hipLaunchKernelGGL(k_bq_pq<R>, dim3(g), dim3(BMap<R>::THREADS), 0, s, A->n_rows, P, Q, part[0],
                           p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr, chunk_queue<R>(p, c1, c2));
        hipLaunchKernelGGL(k_bq_upd<R>, dim3(g), dim3(BMap<R>::THREADS), 0, s, A->n_rows, Rv, Q, minv, part[0],
                           part[1], part[2], p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr, p->d_sys_chunk, st, st2,
                           chunk_queue<R>(p, c2, c3));
        hipLaunchKernelGGL(k_bq_p<R>, dim3(g), dim3(BMap<R>::THREADS), 0, s, A->n_rows, X, Rv, minv, P, part[1],
                           part[2],
                           p->d_chunk_row, p->d_chunk_sys, p->d_sys_ptr, p->d_sys_chunk, max_iter, st2, st,
                           chunk_queue<R>(p, c3, c0));
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
    w += bal(sizeof(BState) * (size_t)p->nsys * R);
    S.st2 = reinterpret_cast<BState *>(w);
    w += bal(sizeof(BState) * (size_t)p->nsys * R);
    S.cnt = reinterpret_cast<int32_t *>(w);
    S.grid_c = std::min(resident_grid(k_bq_upd<R>, BMap<R>::THREADS),
                        std::min(resident_grid(k_bq_p<R>, BMap<R>::THREADS),
                                 resident_grid(k_bq_pq<R>, BMap<R>::THREADS)));
    S.grid_s = bq_spmm_grid<R>(p->tpr, p->rows_mult);
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
    hipLaunchKernelGGL(k_bfill_i32, dim3(1), dim3(64), 0, s, S.cnt, 4 * kQueues, 0);
    BST(S.launched());
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
    // the alternative item order of the chunk kernels: systems by decreasing chunk count
    // (ties by index), each system's chunks in row order
    std::vector<int32_t> by_size((size_t)nsys), chunk_big;
    for (int32_t q = 0; q < nsys; ++q) by_size[q] = q;
    std::stable_sort(by_size.begin(), by_size.end(), [&](int32_t x, int32_t y) {
        return sys_chunk[x + 1] - sys_chunk[x] > sys_chunk[y + 1] - sys_chunk[y];
    });
    chunk_big.reserve(chunk_row.size());
    for (int32_t q : by_size)
        for (int32_t c = sys_chunk[q]; c < sys_chunk[q + 1]; ++c) chunk_big.push_back(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = bupload(p->sys_ptr, &p->d_sys_ptr, s);
    if (st == MP_OK) st = bupload(sys_chunk, &p->d_sys_chunk, s);
    if (st == MP_OK) st = bupload(chunk_row, &p->d_chunk_row, s);
    if (st == MP_OK) st = bupload(chunk_sys, &p->d_chunk_sys, s);
    if (st == MP_OK) st = bupload(chunk_big, &p->d_chunk_big, s);
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
    if (reps < 1) reps = 3;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // two counter sets, used alternately (each launch clears the other)
    int32_t *cnt = nullptr;
    dd_t *part = nullptr;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&cnt), sizeof(int32_t) * 2 * kQueues));
    hipError_t he = hipMalloc(reinterpret_cast<void **>(&part), sizeof(dd_t) * (size_t)plan->n_chunks * plan->nrhs);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    mp_status st = he == hipSuccess ? MP_OK : hip_fail(he, "batched autotune set-up");
    int flip = 0;
    auto timed = [&](auto launch, float *ms) -> mp_status {
        hipLaunchKernelGGL(k_bfill_i32, dim3(1), dim3(64), 0, s, cnt, 2 * kQueues, 0);
        flip = 0;
        mp_status t = launch();   // warm-up
        hipError_t e = hipEventRecord(e0, s);
        for (int r = 0; t == MP_OK && e == hipSuccess && r < reps; ++r) t = launch();
        if (t == MP_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (t == MP_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        if (t == MP_OK && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        if (t == MP_OK && e != hipSuccess) t = hip_fail(e, "batched autotune timing");
        return t;
    };
    // the persistent SpMM: threads per row x rows per tile
    float best = -1.f;
    int best_tpr = plan->tpr, best_u = plan->rows_mult;
    for (int tpr = 1; tpr <= plan->nrhs && st == MP_OK; tpr <<= 1) {
        for (int U = 1; U <= 4 && st == MP_OK; U <<= 1) {
            float ms = 0.f;
            auto launch = [&]() -> mp_status {
                int32_t *c0 = cnt + flip * kQueues, *c1 = cnt + (1 - flip) * kQueues;
                flip = 1 - flip;
                switch (plan->nrhs) {
                    case 1: return launch_bq_spmm<1>(tpr, U, A, a, X, Y, c0, c1, s);
                    case 2: return launch_bq_spmm<2>(tpr, U, A, a, X, Y, c0, c1, s);
                    case 4: return launch_bq_spmm<4>(tpr, U, A, a, X, Y, c0, c1, s);
                    default: return launch_bq_spmm<8>(tpr, U, A, a, X, Y, c0, c1, s);
                }
            };
            st = timed(launch, &ms);
            if (st == MP_OK && (best < 0.f || ms < best)) {
                best = ms;
                best_tpr = tpr;
                best_u = U;
            }
        }
    }
    // the chunk kernels' item order, timed on the (p, q) sums of (X, Y)
    int best_order = plan->chunk_order;
    float best_c = -1.f;
    for (int order = 0; order < 2 && st == MP_OK; ++order) {
        plan->chunk_order = order;
        float ms = 0.f;
        auto launch = [&]() -> mp_status {
            int32_t *c0 = cnt + flip * kQueues, *c1 = cnt + (1 - flip) * kQueues;
            flip = 1 - flip;
            switch (plan->nrhs) {
                case 1: {
                    const int g = std::min(resident_grid(k_bq_pq<1>, BMap<1>::THREADS), plan->n_chunks);
                    hipLaunchKernelGGL(k_bq_pq<1>, dim3(g), dim3(BMap<1>::THREADS), 0, s, A->n_rows, X, Y, part,
                                       plan->d_chunk_row, plan->d_chunk_sys, plan->d_sys_ptr, chunk_queue<1>(plan, c0, c1));
                    break;
                }
                case 2: {
                    const int g = std::min(resident_grid(k_bq_pq<2>, BMap<2>::THREADS), plan->n_chunks);
                    hipLaunchKernelGGL(k_bq_pq<2>, dim3(g), dim3(BMap<2>::THREADS), 0, s, A->n_rows, X, Y, part,
                                       plan->d_chunk_row, plan->d_chunk_sys, plan->d_sys_ptr, chunk_queue<2>(plan, c0, c1));
                    break;
                }
                case 4: {
                    const int g = std::min(resident_grid(k_bq_pq<4>, BMap<4>::THREADS), plan->n_chunks);
                    hipLaunchKernelGGL(k_bq_pq<4>, dim3(g), dim3(BMap<4>::THREADS), 0, s, A->n_rows, X, Y, part,
                                       plan->d_chunk_row, plan->d_chunk_sys, plan->d_sys_ptr, chunk_queue<4>(plan, c0, c1));
                    break;
                }
                default: {
                    const int g = std::min(resident_grid(k_bq_pq<8>, BMap<8>::THREADS), plan->n_chunks);
                    hipLaunchKernelGGL(k_bq_pq<8>, dim3(g), dim3(BMap<8>::THREADS), 0, s, A->n_rows, X, Y, part,
                                       plan->d_chunk_row, plan->d_chunk_sys, plan->d_sys_ptr, chunk_queue<8>(plan, c0, c1));
                }
            }
            MP_HIP_TRY(hipGetLastError());
            return MP_OK;
        };
        st = timed(launch, &ms);
        if (st == MP_OK && (best_c < 0.f || ms < best_c)) {
            best_c = ms;
            best_order = order;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == MP_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (part) (void)hipFree(part);
    (void)hipFree(cnt);
    if (st != MP_OK) return st;
    plan->tpr = best_tpr;
    plan->rows_mult = best_u;
    plan->chunk_order = best_order;
    if (threads_per_row) *threads_per_row = best_tpr;
    return MP_OK;
}

mp_status mp_batch_plan_set_schedule(mp_batch_plan *plan, int32_t threads_per_row, int32_t rows_mult,
                                     int32_t chunk_order)
{
    mpk::clear_error();
    if (!plan) return mpk::fail(MP_ERR_INVALID_ARG, "plan is NULL");
    if (threads_per_row < 1 || threads_per_row > plan->nrhs || (threads_per_row & (threads_per_row - 1)))
        return mpk::fail(MP_ERR_INVALID_ARG, "threads_per_row must be a power of two <= nrhs");
    if (rows_mult != 1 && rows_mult != 2 && rows_mult != 4)
        return mpk::fail(MP_ERR_INVALID_ARG, "rows_mult must be 1, 2 or 4");
    if (chunk_order != 0 && chunk_order != 1) return mpk::fail(MP_ERR_INVALID_ARG, "chunk_order must be 0 or 1");
    plan->tpr = threads_per_row;
    plan->rows_mult = rows_mult;
    plan->chunk_order = chunk_order;
    return MP_OK;
}

mp_status mp_batch_plan_schedule(const mp_batch_plan *plan, int32_t *threads_per_row, int32_t *rows_per_tile,
                                 int32_t *chunk_order)
{
    mpk::clear_error();
    if (!plan) return mpk::fail(MP_ERR_INVALID_ARG, "plan is NULL");
    if (threads_per_row) *threads_per_row = plan->tpr;
    if (rows_per_tile) *rows_per_tile = (256 / plan->tpr) * plan->rows_mult;
    if (chunk_order) *chunk_order = plan->chunk_order;
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
