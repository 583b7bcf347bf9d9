// krylov.hip -- double-double CG and BiCGSTAB on the device (Sec. 4.2 of Kouya,
// arXiv 2412.17510: Krylov subspace methods built on the multi-component SpMV).
//
// Every step is a kernel on the caller's stream: the DD SpMV of spmv.hip, and fused
// DD vector kernels that update the iterate vectors and form the partial sums of the
// dot products in the same pass.  Dot products follow one fixed tree -- chunks of
// 4096 elements, each summed by 256 lanes in the lane order of the SpMV (lane l takes
// elements l, l+256, ...; halving fold), chunk sums combined pairwise -- so every
// iterate is reproducible bit for bit.  Scalars live in a device state block; the
// single-workgroup "final" kernels fold the chunk sums, form alpha / beta / omega with
// DD division and raise a `done` flag (converged on the recurrence, breakdown, or
// iteration limit) that makes every later kernel of the step a no-op.  The host reads
// the state back every `check_every` iterations, confirms convergence with the true
// residual b - A x, and restarts the recurrence from it when the confirmation fails.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "mp_arith.hpp"
#include "plan.hpp"

namespace mpk {

constexpr int kDotLanes = 256;
constexpr int kDotChunk = 4096;
constexpr int kMaxChunks = 2048;   // n <= 8,388,608
constexpr int kPerLane = kDotChunk / kDotLanes;   // elements per lane and chunk
constexpr int kBatch = 8;                          // loads issued ahead of the arithmetic
constexpr int kGroups = 4;                         // thread groups of a chunk workgroup
constexpr int kChunkThreads = kDotLanes * kGroups; // threads of a chunk workgroup
constexpr int kPerThread = kPerLane / kGroups;     // elements of a lane per thread

enum : int32_t { RUN = 0, RECURRENCE_MET = 1, BROKE_DOWN = 2, ITER_LIMIT = 3, CONFIRMED = 4, RESTART = 5 };

struct KState {
    dd_t rho, rho_old, rr, bb, tol2, pq, alpha, beta, omega, rv, ss, ts, tt, rr_true, zeta, eta;
    int32_t done;
    int32_t iters;
    int32_t max_iter;
    int32_t fresh;      // BiCGSTAB: the next step starts with p = r
    int32_t half;       // BiCGSTAB: the half step met the tolerance
    int32_t restarts;
    int32_t pad[2];
};

__device__ __forceinline__ dd_t ldd(const double *__restrict__ v, int64_t n, int64_t i)
{
    dd_t r;
    r.c[0] = v[i];
    r.c[1] = v[n + i];
    return r;
}

__device__ __forceinline__ void sdd(double *__restrict__ v, int64_t n, int64_t i, const dd_t &x)
{
    v[i] = x.c[0];
    v[n + i] = x.c[1];
}

__device__ __forceinline__ dd_t dd_zero()
{
    dd_t r;
    r.c[0] = 0.0;
    r.c[1] = 0.0;
    return r;
}

__device__ __forceinline__ dd_t dd_sub(const dd_t &a, const dd_t &b) { return dd_add(a, mp_neg(b)); }

__device__ __forceinline__ bool dd_finite(const dd_t &a) { return isfinite(a.c[0]); }

// Fold the lane sums of one chunk: lanes [0, used) hold values; acc[l] += acc[l+off]
// for off = 128..1 when lane l+off holds a value.
__device__ __forceinline__ dd_t chunk_fold(const dd_t &v, int used, dd_t *lds)
{
    const int t = threadIdx.x;
    if (t < kDotLanes) lds[t] = v;
    __syncthreads();
    for (int off = kDotLanes / 2; off >= 1; off >>= 1) {
        if (t < off && t + off < used) lds[t] = dd_add(lds[t], lds[t + off]);
        __syncthreads();
    }
    const dd_t r = lds[0];
    __syncthreads();
    return r;
}

// Pairwise tree over m chunk sums (single workgroup): level s combines node i*2s
// with node i*2s + s when that node exists; an unpaired node passes up unchanged.
__device__ __forceinline__ dd_t pair_tree(const dd_t *__restrict__ part, int m, dd_t *P)
{
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    for (int i = t; i < m; i += nt) P[i] = part[i];
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        for (int i = t; (int64_t)i * 2 * s + s < m; i += nt) P[i * 2 * s] = dd_add(P[i * 2 * s], P[i * 2 * s + s]);
        __syncthreads();
    }
    const dd_t r = m > 0 ? P[0] : dd_zero();
    __syncthreads();
    return r;
}

__device__ __forceinline__ int chunk_used(int64_t n, int c)
{
    const int64_t left = n - (int64_t)c * kDotChunk;
    return left < kDotLanes ? (int)left : kDotLanes;
}

// Chunk workgroups of kChunkThreads threads: thread (g, t) = (tid / 256, tid % 256)
// holds elements j = g*kPerThread .. g*kPerThread + kPerThread - 1 of lane t (element
// c*4096 + t + 256 j).  Their loads and element-wise work run in parallel; the lane's
// sums are then carried from group to group through LDS, so each lane still adds its
// products one at a time in j order, starting from its first product.
__device__ __forceinline__ dd_t vadd(const dd_t &a, const dd_t &b) { return dd_add(a, b); }
__device__ __forceinline__ double vadd(double a, double b) { return a + b; }
__device__ __forceinline__ float vadd(float a, float b) { return a + b; }

// prod[q][jj]: product jj of sum q of this thread (valid for jj < nvalid); chain[q]:
// LDS of kDotLanes values.  Leaves lane t's sum q in chain[q][t] for lanes holding
// at least one element.
template <typename V, int NS>
__device__ __forceinline__ void lane_chain(const V (&prod)[NS][kPerThread], int nvalid, V (*chain)[kDotLanes])
{
    const int g = threadIdx.x / kDotLanes, t = threadIdx.x % kDotLanes;
    for (int st = 0; st < kGroups; ++st) {
        if (g == st && nvalid > 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                V a = st == 0 ? prod[q][0] : vadd(chain[q][t], prod[q][0]);
#pragma unroll
                for (int jj = 1; jj < kPerThread; ++jj)
                    if (jj < nvalid) a = vadd(a, prod[q][jj]);
                chain[q][t] = a;
            }
        }
        __syncthreads();
    }
}

// fold of the lane sums left by lane_chain: lds[l] += lds[l + off] for off = 128..1
// where lane l + off holds a value; returns lds[0] (to every thread)
template <typename V>
__device__ __forceinline__ V chain_fold(V *lds, int used)
{
    const int t = threadIdx.x;
    for (int off = kDotLanes / 2; off >= 1; off >>= 1) {
        if (t < off && t + off < used) lds[t] = vadd(lds[t], lds[t + off]);
        __syncthreads();
    }
    const V r = lds[0];
    __syncthreads();
    return r;
}

// Lane shuffles within a wavefront (64 lanes): the value of lane l + d (own value past
// the end), and lane 0's value.
__device__ __forceinline__ double shfl_down_v(double v, int d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ float shfl_down_v(float v, int d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ dd_t shfl_down_v(const dd_t &v, int d)
{
    dd_t r;
    r.c[0] = __shfl_down(v.c[0], d, 64);
    r.c[1] = __shfl_down(v.c[1], d, 64);
    return r;
}
__device__ __forceinline__ double shfl0_v(double v) { return __shfl(v, 0, 64); }
__device__ __forceinline__ float shfl0_v(float v) { return __shfl(v, 0, 64); }
__device__ __forceinline__ dd_t shfl0_v(const dd_t &v)
{
    dd_t r;
    r.c[0] = __shfl(v.c[0], 0, 64);
    r.c[1] = __shfl(v.c[1], 0, 64);
    return r;
}
template <typename V>
__device__ __forceinline__ V vzero()
{
    return V{};
}

// chain_fold of NS sums at once with the result in thread 0 only (the same additions in
// the same order): the two levels that cross wavefronts (off = 128, 64) through LDS, the
// levels off = 32..1 by lane shuffles in wavefront 0, which leaves no barrier after the
// last LDS level.
template <typename V, int NS>
__device__ __forceinline__ void chain_fold_lead(V (*chain)[kDotLanes], int used, V (&out)[NS])
{
    const int t = threadIdx.x;
    for (int off = kDotLanes / 2; off >= 64; off >>= 1) {
        for (int k = t; k < NS * off; k += blockDim.x) {
            const int q = k / off, l = k % off;
            if (l + off < used) chain[q][l] = vadd(chain[q][l], chain[q][l + off]);
        }
        __syncthreads();
    }
    if (t < 64) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            V v = chain[q][t];
            for (int off = 32; off >= 1; off >>= 1) {
                const V o = shfl_down_v(v, off);
                if (t < off && t + off < used) v = vadd(v, o);
            }
            out[q] = v;
        }
    }
}

// pair_tree for m <= 64 without LDS or barriers: every wavefront reduces all m chunk sums
// itself (level s: lane l, a multiple of 2s, adds lane l + s when l + s < m), starting from
// tree_pre, this lane's chunk sum, which a caller loads ahead of its other work.
template <typename V>
__device__ __forceinline__ V tree_pre(const V *__restrict__ part, int m)
{
    const int l = threadIdx.x & 63;
    return l < m ? part[l] : vzero<V>();
}

template <typename V>
__device__ __forceinline__ V tree_wave(V v, int m)
{
    const int l = threadIdx.x & 63;
    for (int s = 1; s < 64; s <<= 1) {
        const V o = shfl_down_v(v, s);
        if ((l & (2 * s - 1)) == 0 && l + s < m) v = vadd(v, o);
    }
    return shfl0_v(v);
}

// valid elements of this thread in chunk c (a prefix of its kPerThread elements)
__device__ __forceinline__ int thread_valid(int64_t n, int c)
{
    const int g = threadIdx.x / kDotLanes, t = threadIdx.x % kDotLanes;
    const int64_t first = (int64_t)c * kDotChunk + t + (int64_t)g * kPerThread * kDotLanes;
    if (first >= n) return 0;
    const int64_t left = (n - 1 - first) / kDotLanes + 1;
    return left < kPerThread ? (int)left : kPerThread;
}

__device__ __forceinline__ int64_t thread_elem(int c, int jj)
{
    const int g = threadIdx.x / kDotLanes, t = threadIdx.x % kDotLanes;
    return (int64_t)c * kDotChunk + t + (int64_t)(g * kPerThread + jj) * kDotLanes;
}

// Workgroup index -> logical block such that each XCD (workgroups are dealt round-robin
// to the 8 XCDs) takes one contiguous range of blocks, as the SpMV's tiles do, so the
// vector kernels of a step touch on each XCD about the rows its SpMV work produced.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int xcd = b & 7;
    const int idx = b >> 3;
    const int per = nb >> 3;
    const int rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// ---------------------------------------------------------------------------
// generic kernels
// ---------------------------------------------------------------------------

// chunk sums of dot(x1, y1) and (optionally) dot(x2, y2); one workgroup per chunk
__global__ __launch_bounds__(kChunkThreads) void k_dot2(int64_t n, const double *__restrict__ x1,
                                                        const double *__restrict__ y1, const double *__restrict__ x2,
                                                        const double *__restrict__ y2, dd_t *__restrict__ part1,
                                                        dd_t *__restrict__ part2, const KState *__restrict__ st)
{
    __shared__ dd_t chain[2][kDotLanes];
    if (st && st->done != RUN) return;
    const int c = xcd_block(blockIdx.x, gridDim.x);
    const int nv = thread_valid(n, c);
    dd_t pr[2][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            pr[0][jj] = dd_mul(ldd(x1, n, k), ldd(y1, n, k));
            if (x2) pr[1][jj] = dd_mul(ldd(x2, n, k), ldd(y2, n, k));
        }
    }
    const int used = chunk_used(n, c);
    if (x2) {
        lane_chain<dd_t, 2>(pr, nv, chain);
        dd_t s[2];
        chain_fold_lead<dd_t, 2>(chain, used, s);
        if (threadIdx.x == 0) {
            part1[c] = s[0];
            part2[c] = s[1];
        }
    } else {
        lane_chain<dd_t, 1>(reinterpret_cast<const dd_t(&)[1][kPerThread]>(pr[0]), nv, chain);
        dd_t s[1];
        chain_fold_lead<dd_t, 1>(chain, used, s);
        if (threadIdx.x == 0) part1[c] = s[0];
    }
}

// r = b - q
__global__ __launch_bounds__(256) void k_residual(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ q, double *__restrict__ r)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        sdd(r, n, i, dd_sub(ldd(b, n, i), ldd(q, n, i)));
}

// z = M^-1 r (Jacobi: DD times the binary64 inverse diagonal, Alg. 3; or a copy)
__global__ __launch_bounds__(256) void k_precond(int64_t n, const double *__restrict__ minv,
                                                 const double *__restrict__ r, double *__restrict__ z,
                                                 const KState *__restrict__ st)
{
    if (st && st->done != RUN) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        sdd(z, n, i, minv ? dd_mul_d(ldd(r, n, i), minv[i]) : ldd(r, n, i));
}

__global__ __launch_bounds__(256) void k_copy(int64_t n2, const double *__restrict__ src, double *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

// Jacobi inverse diagonal fl(1 / hi(a_ii)); 1 where the row has no diagonal entry
__global__ __launch_bounds__(256) void k_jacobi_minv(int64_t n, const int32_t *__restrict__ rp,
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

// confirmation of a recurrence convergence: rr_true from chunk sums
__global__ __launch_bounds__(256) void k_confirm(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rr_true = rr;
        if (dd_le(rr, st->tol2)) {
            st->done = CONFIRMED;
        } else {
            st->rr = rr;
            st->restarts += 1;
            st->done = RESTART;
        }
    }
}

// exit record: rr_true of the returned x
__global__ __launch_bounds__(256) void k_exit_rr(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) st->rr_true = rr;
}

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------

// bb, rho = (r, z), rr = (r, r) of the start vectors; tolerance; first test
__global__ __launch_bounds__(256) void k_cg_init(const dd_t *__restrict__ pbb, const dd_t *__restrict__ prz,
                                                 const dd_t *__restrict__ prr, int m, double rtol2, int32_t max_iter,
                                                 KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t bb = pair_tree(pbb, m, P);
    const dd_t rz = pair_tree(prz, m, P);
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->tol2 = dd_mul_d(bb, rtol2);
        st->rho = rz;
        st->rr = rr;
        st->iters = 0;
        st->max_iter = max_iter;
        st->restarts = 0;
        st->done = dd_le(rr, st->tol2) ? RECURRENCE_MET : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

// after a restart from the true residual: rho = (r, z)
__global__ __launch_bounds__(256) void k_cg_restart(const dd_t *__restrict__ prz, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t rz = pair_tree(prz, m, P);
    if (threadIdx.x == 0) {
        st->rho = rz;
        st->done = st->iters >= st->max_iter ? ITER_LIMIT : RUN;
    }
}

// One CG step after q = A p and the chunk sums of (p, q) is two kernels:
//   k_cg_update: alpha = rho / (p, q) (breakdown unless (p, q) > 0), then
//                r -= alpha q; z = M^-1 r; chunk sums of (r, z), (r, r)
//   k_cg_p:      x += alpha p (with the p it loads anyway, on the whole grid rather than
//                the chunk workgroups); rho_new = (r, z), rr = (r, r); beta = rho_new / rho;
//                stop tests; p = z + beta p (also into the SpMV's staged copy of x)
// Every workgroup reduces the chunk sums itself (the same tree, so the same values),
// which needs no separate scalar kernel.  The state is double-buffered across the two
// kernels of a step: k_cg_p reads state `sr` and workgroup 0 writes the next state to
// `sw`, so no workgroup reads a field that another workgroup of the same kernel is
// writing.  A step with state sr = S[j & 1] writes S[(j + 1) & 1].

__device__ __forceinline__ int32_t block_state(const KState *st)
{
    __shared__ int32_t s_done;
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    return s_done;
}

__global__ __launch_bounds__(kChunkThreads) void k_cg_update(int64_t n, double *__restrict__ r,
                                                             double *__restrict__ z, const double *__restrict__ q,
                                                             const double *__restrict__ minv,
                                                             const dd_t *__restrict__ ppq, int m,
                                                             dd_t *__restrict__ prz, dd_t *__restrict__ prr,
                                                             KState *__restrict__ st)
{
    __shared__ dd_t chain[2][kDotLanes];
    __shared__ dd_t P[kMaxChunks];
    __shared__ dd_t s_rho;
    // the element loads do not depend on the scalars: issue them first
    const int c = xcd_block(blockIdx.x, gridDim.x);
    const int nv = thread_valid(n, c);
    dd_t rv[kPerThread], qv[kPerThread];
    double mv[kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            rv[jj] = ldd(r, n, k);
            qv[jj] = ldd(q, n, k);
            mv[jj] = minv ? minv[k] : 0.0;
        }
    }
    const bool small = m <= 64;
    const dd_t pq_pre = small ? tree_pre(ppq, m) : dd_zero();
    if (threadIdx.x == 0) s_rho = st->rho;
    if (block_state(st) != RUN) return;
    const dd_t pq = small ? tree_wave(pq_pre, m) : pair_tree(ppq, m, P);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(pq.c[0] > 0.0) || !dd_finite(pq)) {
        if (lead) {
            st->pq = pq;
            st->done = BROKE_DOWN;
        }
        return;
    }
    const dd_t alpha = dd_div(s_rho, pq);
    if (lead) {
        st->pq = pq;
        st->alpha = alpha;
    }
    dd_t pr[2][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            const dd_t rk = dd_sub(rv[jj], dd_mul(alpha, qv[jj]));
            sdd(r, n, k, rk);
            const dd_t zk = minv ? dd_mul_d(rk, mv[jj]) : rk;
            sdd(z, n, k, zk);
            pr[0][jj] = dd_mul(rk, zk);
            pr[1][jj] = dd_mul(rk, rk);
        }
    }
    lane_chain<dd_t, 2>(pr, nv, chain);
    const int used = chunk_used(n, c);
    dd_t s[2];
    chain_fold_lead<dd_t, 2>(chain, used, s);
    if (threadIdx.x == 0) {
        prz[c] = s[0];
        prr[c] = s[1];
    }
}

// xs: NULL, or the plan's staged copy of x (interleaved hi, lo) that the next SpMV reads
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, double *__restrict__ x, const double *__restrict__ z,
                                              double *__restrict__ p, double *__restrict__ xs,
                                              const dd_t *__restrict__ prz, const dd_t *__restrict__ prr, int m,
                                              const KState *__restrict__ sr, KState *__restrict__ sw)
{
    __shared__ dd_t P[kMaxChunks];
    __shared__ dd_t s_rho, s_tol2, s_alpha;
    __shared__ int32_t s_iters, s_max;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // this thread's first element, loaded ahead of the scalars
    const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    dd_t z0 = dd_zero(), p0 = dd_zero();
    if (i0 < n) {
        z0 = ldd(z, n, i0);
        p0 = ldd(p, n, i0);
    }
    const bool small = m <= 64;
    const dd_t rz_pre = small ? tree_pre(prz, m) : dd_zero();
    const dd_t rr_pre = small ? tree_pre(prr, m) : dd_zero();
    if (threadIdx.x == 0) {
        s_rho = sr->rho;
        s_tol2 = sr->tol2;
        s_alpha = sr->alpha;
        s_iters = sr->iters;
        s_max = sr->max_iter;
    }
    if (block_state(sr) != RUN) {
        if (lead) *sw = *sr;
        return;
    }
    // the update kernel ran to the end with this alpha: x += alpha p (old p)
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * 256)
        sdd(x, n, i, dd_add(ldd(x, n, i), dd_mul(s_alpha, i == i0 ? p0 : ldd(p, n, i))));
    // wavefront 0 reduces the chunk sums (a single tree per workgroup) and thread 0 decides
    // the step for the workgroup
    __shared__ dd_t s_rz, s_rr, s_beta;
    __shared__ int32_t s_next;
    dd_t rz = dd_zero(), rr = dd_zero();
    if (small) {
        if (threadIdx.x < 64) {
            rz = tree_wave(rz_pre, m);
            rr = tree_wave(rr_pre, m);
        }
    } else {
        rz = pair_tree(prz, m, P);
        rr = pair_tree(prr, m, P);
    }
    if (threadIdx.x == 0) {
        int32_t d = RUN;
        dd_t bt = dd_zero();
        if (!dd_finite(rr) || !dd_finite(rz)) {
            d = BROKE_DOWN;
        } else {
            bt = dd_div(rz, s_rho);
            if (dd_le(rr, s_tol2))
                d = RECURRENCE_MET;
            else if (s_iters + 1 >= s_max)
                d = ITER_LIMIT;
        }
        s_rz = rz;
        s_rr = rr;
        s_beta = bt;
        s_next = d;
    }
    __syncthreads();
    const int32_t iters = s_iters + 1;
    const int32_t done = s_next;
    const dd_t beta = s_beta;
    rz = s_rz;
    rr = s_rr;
    if (lead) {
        KState o = *sr;
        o.iters = iters;
        o.rr = rr;
        if (done != BROKE_DOWN) {
            o.beta = beta;
            o.rho = rz;
        }
        o.done = done;
        *sw = o;
    }
    if (done != RUN) return;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * 256) {
        const dd_t zi = i == i0 ? z0 : ldd(z, n, i);
        const dd_t pi = dd_add(zi, dd_mul(beta, i == i0 ? p0 : ldd(p, n, i)));
        sdd(p, n, i, pi);
        if (xs) {
            xs[2 * i] = pi.c[0];
            xs[2 * i + 1] = pi.c[1];
        }
    }
}

// ---------------------------------------------------------------------------
// BiCG (Fletcher), with A^T given explicitly
// ---------------------------------------------------------------------------

// sigma = (p~, q); alpha = rho / sigma; breakdown when sigma is 0 or not finite
__global__ __launch_bounds__(256) void k_bicg_alpha(const dd_t *__restrict__ ppq, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t pq = pair_tree(ppq, m, P);
    if (threadIdx.x == 0) {
        st->pq = pq;
        if (pq.c[0] == 0.0 || !dd_finite(pq))
            st->done = BROKE_DOWN;
        else
            st->alpha = dd_div(st->rho, pq);
    }
}

// x += alpha p; r -= alpha q; r~ -= alpha q~; z = M^-1 r; z~ = M^-1 r~;
// chunk sums of (r~, z) and (r, r)
__global__ __launch_bounds__(256) void k_bicg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ z, const double *__restrict__ p,
                                                     const double *__restrict__ q, double *__restrict__ rt,
                                                     double *__restrict__ zt, const double *__restrict__ qt,
                                                     const double *__restrict__ minv, dd_t *__restrict__ prz,
                                                     dd_t *__restrict__ prr, const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const dd_t alpha = st->alpha;
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t arz = dd_zero(), arr = dd_zero();
    bool first = true;
    for (int64_t k = base + t; k < end; k += kDotLanes) {
        sdd(x, n, k, dd_add(ldd(x, n, k), dd_mul(alpha, ldd(p, n, k))));
        const dd_t rk = dd_sub(ldd(r, n, k), dd_mul(alpha, ldd(q, n, k)));
        const dd_t rtk = dd_sub(ldd(rt, n, k), dd_mul(alpha, ldd(qt, n, k)));
        sdd(r, n, k, rk);
        sdd(rt, n, k, rtk);
        const dd_t zk = minv ? dd_mul_d(rk, minv[k]) : rk;
        const dd_t ztk = minv ? dd_mul_d(rtk, minv[k]) : rtk;
        sdd(z, n, k, zk);
        sdd(zt, n, k, ztk);
        const dd_t p1 = dd_mul(rtk, zk), p2 = dd_mul(rk, rk);
        arz = first ? p1 : dd_add(arz, p1);
        arr = first ? p2 : dd_add(arr, p2);
        first = false;
    }
    const dd_t s1 = chunk_fold(arz, used, lds);
    const dd_t s2 = chunk_fold(arr, used, lds);
    if (t == 0) {
        prz[c] = s1;
        prr[c] = s2;
    }
}

// rho' = (r~, z), rr = (r, r); beta = rho' / rho; stop tests
__global__ __launch_bounds__(256) void k_bicg_beta(const dd_t *__restrict__ prz, const dd_t *__restrict__ prr, int m,
                                                   KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rz = pair_tree(prz, m, P);
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = rr;
        if (!dd_finite(rr) || !dd_finite(rz) || (rz.c[0] == 0.0 && !dd_le(rr, st->tol2))) {
            st->done = BROKE_DOWN;
            return;
        }
        st->beta = dd_div(rz, st->rho);
        st->rho = rz;
        if (dd_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// p = z + beta p; p~ = z~ + beta p~
__global__ __launch_bounds__(256) void k_bicg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                                const double *__restrict__ zt, double *__restrict__ pt,
                                                const KState *__restrict__ st)
{
    if (st->done != RUN) return;
    const dd_t beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        sdd(p, n, i, dd_add(ldd(z, n, i), dd_mul(beta, ldd(p, n, i))));
        sdd(pt, n, i, dd_add(ldd(zt, n, i), dd_mul(beta, ldd(pt, n, i))));
    }
}

// ---------------------------------------------------------------------------
// CGS (Sonneveld), right Jacobi preconditioning
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_cgs_init(const dd_t *__restrict__ pbb, const dd_t *__restrict__ prr, int m,
                                                  double rtol2, int32_t max_iter, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t bb = pair_tree(pbb, m, P);
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->tol2 = dd_mul_d(bb, rtol2);
        st->rr = rr;
        st->iters = 0;
        st->max_iter = max_iter;
        st->restarts = 0;
        st->fresh = 1;
        st->done = dd_le(rr, st->tol2) ? RECURRENCE_MET : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

// after a failed confirmation: the shadow is reset by the host, the next step is fresh
__global__ __launch_bounds__(64) void k_cgs_restart(KState *__restrict__ st)
{
    if (threadIdx.x == 0) {
        st->fresh = 1;
        st->done = st->iters >= st->max_iter ? ITER_LIMIT : RUN;
    }
}

// rho = (r~, r): breakdown when 0 or not finite; beta = rho / rho_old unless fresh
__global__ __launch_bounds__(256) void k_cgs_rho(const dd_t *__restrict__ prho, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rho = pair_tree(prho, m, P);
    if (threadIdx.x == 0) {
        if (rho.c[0] == 0.0 || !dd_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho = rho;
        if (!st->fresh) st->beta = dd_div(rho, st->rho_old);
    }
}

// fresh: u = p = r; else u = r + beta q, p = u + beta (q + beta p); p^ = M^-1 p
__global__ __launch_bounds__(256) void k_cgs_up(int64_t n, const double *__restrict__ r, const double *__restrict__ q,
                                                double *__restrict__ u, double *__restrict__ p,
                                                double *__restrict__ ph, const double *__restrict__ minv,
                                                const KState *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const dd_t ri = ldd(r, n, i);
        dd_t pi;
        if (fresh) {
            sdd(u, n, i, ri);
            pi = ri;
        } else {
            const dd_t qi = ldd(q, n, i);
            const dd_t ui = dd_add(ri, dd_mul(beta, qi));
            const dd_t w = dd_add(qi, dd_mul(beta, ldd(p, n, i)));
            sdd(u, n, i, ui);
            pi = dd_add(ui, dd_mul(beta, w));
        }
        sdd(p, n, i, pi);
        sdd(ph, n, i, minv ? dd_mul_d(pi, minv[i]) : pi);
    }
}

// sigma = (r~, v): breakdown when 0 or not finite; alpha = rho / sigma
__global__ __launch_bounds__(256) void k_cgs_alpha(const dd_t *__restrict__ psig, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t sigma = pair_tree(psig, m, P);
    if (threadIdx.x == 0) {
        st->fresh = 0;
        st->pq = sigma;
        if (sigma.c[0] == 0.0 || !dd_finite(sigma))
            st->done = BROKE_DOWN;
        else
            st->alpha = dd_div(st->rho, sigma);
    }
}

// q = u - alpha v; u^ = M^-1 (u + q); x += alpha u^
__global__ __launch_bounds__(256) void k_cgs_q(int64_t n, const double *__restrict__ u, const double *__restrict__ v,
                                               double *__restrict__ q, double *__restrict__ uh, double *__restrict__ x,
                                               const double *__restrict__ minv, const KState *__restrict__ st)
{
    if (st->done != RUN) return;
    const dd_t alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const dd_t ui = ldd(u, n, i);
        const dd_t qi = dd_sub(ui, dd_mul(alpha, ldd(v, n, i)));
        const dd_t s = dd_add(ui, qi);
        const dd_t uhi = minv ? dd_mul_d(s, minv[i]) : s;
        sdd(q, n, i, qi);
        sdd(uh, n, i, uhi);
        sdd(x, n, i, dd_add(ldd(x, n, i), dd_mul(alpha, uhi)));
    }
}

// r -= alpha t; chunk sums of (r, r)
__global__ __launch_bounds__(256) void k_cgs_r(int64_t n, double *__restrict__ r, const double *__restrict__ t,
                                               dd_t *__restrict__ prr, const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const dd_t alpha = st->alpha;
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t arr = dd_zero();
    bool first = true;
    for (int64_t k = base + tid; k < end; k += kDotLanes) {
        const dd_t rk = dd_sub(ldd(r, n, k), dd_mul(alpha, ldd(t, n, k)));
        sdd(r, n, k, rk);
        const dd_t p2 = dd_mul(rk, rk);
        arr = first ? p2 : dd_add(arr, p2);
        first = false;
    }
    const dd_t s = chunk_fold(arr, used, lds);
    if (tid == 0) prr[c] = s;
}

__global__ __launch_bounds__(256) void k_cgs_rr(const dd_t *__restrict__ prr, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = rr;
        if (!dd_finite(rr)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        if (dd_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// ---------------------------------------------------------------------------
// GPBiCG (Zhang), right Jacobi preconditioning.  Vectors: r, r~, p, q = A M p,
// t = r - alpha q, c = A M t, y, u, z, w, t' (the previous t), and one scratch for
// M p / M t.  A step is counted when t is formed; a t that meets the tolerance ends
// the step early (x += M alpha p, r = t) and the next step is fresh.
// ---------------------------------------------------------------------------

// rho = (r~, r): breakdown when 0 or not finite; later steps beta = (alpha/zeta)(rho/rho_old)
__global__ __launch_bounds__(256) void k_gp_rho(const dd_t *__restrict__ prho, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rho = pair_tree(prho, m, P);
    if (threadIdx.x == 0) {
        if (rho.c[0] == 0.0 || !dd_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho = rho;
        if (!st->fresh) st->beta = dd_mul(dd_div(st->alpha, st->zeta), dd_div(rho, st->rho_old));
    }
}

// fresh: p = r; else p = r + beta (p - u), w = c + beta q; tmp = M p
__global__ __launch_bounds__(256) void k_gp_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                              const double *__restrict__ u, const double *__restrict__ c,
                                              const double *__restrict__ q, double *__restrict__ w,
                                              double *__restrict__ tmp, const double *__restrict__ minv,
                                              const KState *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const dd_t ri = ldd(r, n, i);
        dd_t pi;
        if (fresh) {
            pi = ri;
        } else {
            const dd_t ui = ldd(u, n, i), ci = ldd(c, n, i), qi = ldd(q, n, i), po = ldd(p, n, i);
            pi = dd_add(ri, dd_mul(beta, dd_sub(po, ui)));
            sdd(w, n, i, dd_add(ci, dd_mul(beta, qi)));
        }
        sdd(p, n, i, pi);
        sdd(tmp, n, i, minv ? dd_mul_d(pi, minv[i]) : pi);
    }
}

// sigma = (r~, q): breakdown when 0 or not finite; alpha = rho / sigma
__global__ __launch_bounds__(256) void k_gp_alpha(const dd_t *__restrict__ psig, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t sigma = pair_tree(psig, m, P);
    if (threadIdx.x == 0) {
        st->pq = sigma;
        if (sigma.c[0] == 0.0 || !dd_finite(sigma))
            st->done = BROKE_DOWN;
        else
            st->alpha = dd_div(st->rho, sigma);
    }
}

// t = r - alpha q; later steps y = (t' - t) - alpha w; tmp = M t; chunk sums of (t, t)
__global__ __launch_bounds__(256) void k_gp_t(int64_t n, const double *__restrict__ r, const double *__restrict__ q,
                                              const double *__restrict__ tp, const double *__restrict__ w,
                                              double *__restrict__ t, double *__restrict__ y,
                                              double *__restrict__ tmp, const double *__restrict__ minv,
                                              dd_t *__restrict__ ptt, const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t alpha = st->alpha;
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t acc = dd_zero();
    bool first = true;
    for (int64_t k = base + tid; k < end; k += kDotLanes) {
        const dd_t tk = dd_sub(ldd(r, n, k), dd_mul(alpha, ldd(q, n, k)));
        sdd(t, n, k, tk);
        if (!fresh) sdd(y, n, k, dd_sub(dd_sub(ldd(tp, n, k), tk), dd_mul(alpha, ldd(w, n, k))));
        sdd(tmp, n, k, minv ? dd_mul_d(tk, minv[k]) : tk);
        const dd_t p2 = dd_mul(tk, tk);
        acc = first ? p2 : dd_add(acc, p2);
        first = false;
    }
    const dd_t sum = chunk_fold(acc, used, lds);
    if (tid == 0) ptt[c] = sum;
}

// tt = (t, t); the step is counted; half-step test
__global__ __launch_bounds__(256) void k_gp_tt(const dd_t *__restrict__ ptt, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t tt = pair_tree(ptt, m, P);
    if (threadIdx.x == 0) {
        st->tt = tt;
        st->iters += 1;
        st->half = dd_le(tt, st->tol2) ? 1 : 0;
    }
}

// half step met the tolerance: x += M (alpha p); r = t
__global__ __launch_bounds__(256) void k_gp_half(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ p, const double *__restrict__ t,
                                                 const double *__restrict__ minv, const KState *__restrict__ st)
{
    if (st->done != RUN || !st->half) return;
    const dd_t alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const dd_t d = dd_mul(alpha, ldd(p, n, i));
        sdd(x, n, i, dd_add(ldd(x, n, i), minv ? dd_mul_d(d, minv[i]) : d));
        sdd(r, n, i, ldd(t, n, i));
    }
}

__global__ __launch_bounds__(64) void k_gp_half_final(KState *__restrict__ st)
{
    if (threadIdx.x != 0 || st->done != RUN || !st->half) return;
    st->rr = st->tt;
    st->rho_old = st->rho;
    st->fresh = 1;
    st->half = 0;
    st->done = RECURRENCE_MET;
}

// chunk sums of (c, c), (c, t) and, after the first step, (y, y), (y, c), (y, t)
__global__ __launch_bounds__(kChunkThreads) void k_gp_dots(int64_t n, const double *__restrict__ cv,
                                                           const double *__restrict__ t, const double *__restrict__ y,
                                                           dd_t *__restrict__ pcc, dd_t *__restrict__ pct,
                                                           dd_t *__restrict__ pyy, dd_t *__restrict__ pyc,
                                                           dd_t *__restrict__ pyt, const KState *__restrict__ st)
{
    __shared__ dd_t chain[5][kDotLanes];
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const int c = blockIdx.x;
    const int nv = thread_valid(n, c);
    dd_t pr[5][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            const dd_t ck = ldd(cv, n, k), tk = ldd(t, n, k);
            pr[0][jj] = dd_mul(ck, ck);
            pr[1][jj] = dd_mul(ck, tk);
            if (!fresh) {
                const dd_t yk = ldd(y, n, k);
                pr[2][jj] = dd_mul(yk, yk);
                pr[3][jj] = dd_mul(yk, ck);
                pr[4][jj] = dd_mul(yk, tk);
            }
        }
    }
    const int used = chunk_used(n, c);
    dd_t *outs[5] = {pcc, pct, pyy, pyc, pyt};
    if (fresh) {
        lane_chain<dd_t, 2>(reinterpret_cast<const dd_t(&)[2][kPerThread]>(pr[0]), nv, chain);
        for (int q = 0; q < 2; ++q) {
            const dd_t sq = chain_fold(chain[q], used);
            if (threadIdx.x == 0) outs[q][c] = sq;
        }
    } else {
        lane_chain<dd_t, 5>(pr, nv, chain);
        for (int q = 0; q < 5; ++q) {
            const dd_t sq = chain_fold(chain[q], used);
            if (threadIdx.x == 0) outs[q][c] = sq;
        }
    }
}

// zeta and eta: first step zeta = (c,t)/(c,c), eta = 0; later steps from the 2x2
// normal equations with d = (c,c)(y,y) - (y,c)^2; breakdown on a zero (c,c) or d, a
// zero zeta or a non-finite zeta / eta
__global__ __launch_bounds__(256) void k_gp_zeta(const dd_t *__restrict__ pcc, const dd_t *__restrict__ pct,
                                                 const dd_t *__restrict__ pyy, const dd_t *__restrict__ pyc,
                                                 const dd_t *__restrict__ pyt, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t cc = pair_tree(pcc, m, P);
    const dd_t ct = pair_tree(pct, m, P);
    dd_t yy = dd_zero(), yc = dd_zero(), yt = dd_zero();
    if (!fresh) {
        yy = pair_tree(pyy, m, P);
        yc = pair_tree(pyc, m, P);
        yt = pair_tree(pyt, m, P);
    }
    if (threadIdx.x == 0) {
        dd_t zeta, eta;
        if (fresh) {
            if (cc.c[0] == 0.0 || !dd_finite(cc)) {
                st->done = BROKE_DOWN;
                return;
            }
            zeta = dd_div(ct, cc);
            eta = dd_zero();
        } else {
            const dd_t den = dd_sub(dd_mul(cc, yy), dd_mul(yc, yc));
            if (den.c[0] == 0.0 || !dd_finite(den)) {
                st->done = BROKE_DOWN;
                return;
            }
            zeta = dd_div(dd_sub(dd_mul(yy, ct), dd_mul(yt, yc)), den);
            eta = dd_div(dd_sub(dd_mul(cc, yt), dd_mul(yc, ct)), den);
        }
        if (zeta.c[0] == 0.0 || !dd_finite(zeta) || !dd_finite(eta)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->zeta = zeta;
        st->eta = eta;
    }
}

// u = zeta q + eta (t' - r + beta u), z = zeta r + eta z - alpha u (first step:
// u = zeta q, z = zeta r - alpha u); x += M (alpha p + z); r = t - eta y - zeta c
// (first step: r = t - zeta c); t' = t; chunk sums of (r, r)
__global__ __launch_bounds__(256) void k_gp_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   const double *__restrict__ t, const double *__restrict__ cv,
                                                   const double *__restrict__ y, double *__restrict__ u,
                                                   double *__restrict__ z, double *__restrict__ tp,
                                                   const double *__restrict__ minv, dd_t *__restrict__ prr,
                                                   const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t alpha = st->alpha, beta = st->beta, zeta = st->zeta, eta = st->eta;
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t acc = dd_zero();
    bool first = true;
    for (int64_t k = base + tid; k < end; k += kDotLanes) {
        const dd_t rk = ldd(r, n, k), tk = ldd(t, n, k), qk = ldd(q, n, k), ck = ldd(cv, n, k);
        dd_t uk, zk, rn;
        if (fresh) {
            uk = dd_mul(zeta, qk);
            zk = dd_sub(dd_mul(zeta, rk), dd_mul(alpha, uk));
            rn = dd_sub(tk, dd_mul(zeta, ck));
        } else {
            const dd_t g = dd_add(dd_sub(ldd(tp, n, k), rk), dd_mul(beta, ldd(u, n, k)));
            uk = dd_add(dd_mul(zeta, qk), dd_mul(eta, g));
            zk = dd_sub(dd_add(dd_mul(zeta, rk), dd_mul(eta, ldd(z, n, k))), dd_mul(alpha, uk));
            rn = dd_sub(dd_sub(tk, dd_mul(eta, ldd(y, n, k))), dd_mul(zeta, ck));
        }
        sdd(u, n, k, uk);
        sdd(z, n, k, zk);
        const dd_t d = dd_add(dd_mul(alpha, ldd(p, n, k)), zk);
        sdd(x, n, k, dd_add(ldd(x, n, k), minv ? dd_mul_d(d, minv[k]) : d));
        sdd(r, n, k, rn);
        sdd(tp, n, k, tk);
        const dd_t p2 = dd_mul(rn, rn);
        acc = first ? p2 : dd_add(acc, p2);
        first = false;
    }
    const dd_t sum = chunk_fold(acc, used, lds);
    if (tid == 0) prr[c] = sum;
}

// rr = (r, r): breakdown when not finite; the next step is not fresh; stop tests
__global__ __launch_bounds__(256) void k_gp_rr(const dd_t *__restrict__ prr, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (!dd_finite(rr)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        st->fresh = 0;
        if (dd_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// ---------------------------------------------------------------------------
// BiCGSTAB
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bi_init(const dd_t *__restrict__ pbb, const dd_t *__restrict__ prr, int m,
                                                 double rtol2, int32_t max_iter, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t bb = pair_tree(pbb, m, P);
    const dd_t rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        dd_t one;
        one.c[0] = 1.0;
        one.c[1] = 0.0;
        st->bb = bb;
        st->tol2 = dd_mul_d(bb, rtol2);
        st->rr = rr;
        st->rho_old = one;
        st->alpha = one;
        st->omega = one;
        st->iters = 0;
        st->max_iter = max_iter;
        st->restarts = 0;
        st->fresh = 1;
        st->half = 0;
        st->done = dd_le(rr, st->tol2) ? RECURRENCE_MET : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

// after a restart: the shadow residual is the new residual, next step starts fresh
__global__ __launch_bounds__(256) void k_bi_restart(KState *__restrict__ st)
{
    if (threadIdx.x == 0) {
        st->fresh = 1;
        st->done = st->iters >= st->max_iter ? ITER_LIMIT : RUN;
    }
}

// rho = (rh, r); beta = (rho / rho_old)(alpha / omega) unless the step is fresh
__global__ __launch_bounds__(256) void k_bi_rho(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rho = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rho = rho;
        if (rho.c[0] == 0.0 || !dd_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        if (!st->fresh) st->beta = dd_mul(dd_div(rho, st->rho_old), dd_div(st->alpha, st->omega));
    }
}

// p = r (fresh) or p = r + beta (p - omega v)
__global__ __launch_bounds__(256) void k_bi_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                              const double *__restrict__ v, const KState *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const dd_t beta = st->beta, omega = st->omega;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (fresh) {
            sdd(p, n, i, ldd(r, n, i));
        } else {
            const dd_t pv = dd_sub(ldd(p, n, i), dd_mul(omega, ldd(v, n, i)));
            sdd(p, n, i, dd_add(ldd(r, n, i), dd_mul(beta, pv)));
        }
    }
}

// alpha = rho / (rh, v)
__global__ __launch_bounds__(256) void k_bi_alpha(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rv = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->fresh = 0;
        st->rv = rv;
        if (rv.c[0] == 0.0 || !dd_finite(rv)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->alpha = dd_div(st->rho, rv);
    }
}

// s = r - alpha v; chunk sums of (s, s)
__global__ __launch_bounds__(256) void k_bi_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                              double *__restrict__ s, dd_t *__restrict__ pss,
                                              const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const dd_t alpha = st->alpha;
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t acc = dd_zero();
    bool first = true;
    for (int64_t k = base + t; k < end; k += kDotLanes) {
        const dd_t sk = dd_sub(ldd(r, n, k), dd_mul(alpha, ldd(v, n, k)));
        sdd(s, n, k, sk);
        acc = first ? dd_mul(sk, sk) : dd_add(acc, dd_mul(sk, sk));
        first = false;
    }
    const dd_t sum = chunk_fold(acc, used, lds);
    if (t == 0) pss[c] = sum;
}

// ss = (s, s); one step counted; half-step test
__global__ __launch_bounds__(256) void k_bi_ss(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t ss = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->ss = ss;
        st->iters += 1;
        st->half = dd_le(ss, st->tol2) ? 1 : 0;
    }
}

// half step met the tolerance: x += alpha ph; r = s
__global__ __launch_bounds__(256) void k_bi_half(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ ph, const double *__restrict__ s,
                                                 const KState *__restrict__ st)
{
    if (st->done != RUN || !st->half) return;
    const dd_t alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        sdd(x, n, i, dd_add(ldd(x, n, i), dd_mul(alpha, ldd(ph, n, i))));
        sdd(r, n, i, ldd(s, n, i));
    }
}

__global__ __launch_bounds__(256) void k_bi_half_final(KState *__restrict__ st)
{
    if (threadIdx.x != 0 || st->done != RUN || !st->half) return;
    dd_t one;
    one.c[0] = 1.0;
    one.c[1] = 0.0;
    st->rr = st->ss;
    st->rho_old = st->rho;
    st->omega = one;
    st->fresh = 1;
    st->half = 0;
    st->done = RECURRENCE_MET;
}

// omega = (t, s) / (t, t)
__global__ __launch_bounds__(256) void k_bi_omega(const dd_t *__restrict__ pts, const dd_t *__restrict__ ptt, int m,
                                                  KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t ts = pair_tree(pts, m, P);
    const dd_t tt = pair_tree(ptt, m, P);
    if (threadIdx.x == 0) {
        st->ts = ts;
        st->tt = tt;
        if (tt.c[0] == 0.0 || !dd_finite(tt)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->omega = dd_div(ts, tt);
    }
}

// x = (x + alpha ph) + omega sh; r = s - omega t; chunk sums of (r, r)
__global__ __launch_bounds__(256) void k_bi_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                               const double *__restrict__ ph, const double *__restrict__ sh,
                                               const double *__restrict__ s, const double *__restrict__ tv,
                                               dd_t *__restrict__ prr, const KState *__restrict__ st)
{
    __shared__ dd_t lds[kDotLanes];
    if (st->done != RUN) return;
    const dd_t alpha = st->alpha, omega = st->omega;
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    const int used = chunk_used(n, c);
    dd_t acc = dd_zero();
    bool first = true;
    for (int64_t k = base + t; k < end; k += kDotLanes) {
        const dd_t xv = dd_add(ldd(x, n, k), dd_mul(alpha, ldd(ph, n, k)));
        sdd(x, n, k, dd_add(xv, dd_mul(omega, ldd(sh, n, k))));
        const dd_t rk = dd_sub(ldd(s, n, k), dd_mul(omega, ldd(tv, n, k)));
        sdd(r, n, k, rk);
        acc = first ? dd_mul(rk, rk) : dd_add(acc, dd_mul(rk, rk));
        first = false;
    }
    const dd_t sum = chunk_fold(acc, used, lds);
    if (t == 0) prr[c] = sum;
}

// rr = (r, r); breakdown on omega = 0; convergence / limit tests
__global__ __launch_bounds__(256) void k_bi_rr(const dd_t *__restrict__ part, int m, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    if (st->done != RUN) return;
    const dd_t rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (!dd_finite(rr) || st->omega.c[0] == 0.0) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        if (dd_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// ---------------------------------------------------------------------------
// mixed-precision iterative refinement: plain-precision inner PCG (T = double or
// float) on hi(A), in the same reduction shapes as the DD solver
// ---------------------------------------------------------------------------

template <typename T>
struct InState {
    T rho, rr, rr0, tol, pq, alpha, beta;
    int32_t done;
    int32_t iters;
    int32_t max_iter;
    int32_t pad;
    double maxabs;   // max |hi(r)| of the current DD residual (outer loop)
};

template <typename T>
__device__ __forceinline__ T chunk_fold_t(T v, int used, T *lds)
{
    const int t = threadIdx.x;
    if (t < kDotLanes) lds[t] = v;
    __syncthreads();
    for (int off = kDotLanes / 2; off >= 1; off >>= 1) {
        if (t < off && t + off < used) lds[t] = lds[t] + lds[t + off];
        __syncthreads();
    }
    const T r = lds[0];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T pair_tree_t(const T *__restrict__ part, int m, T *P)
{
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    for (int i = t; i < m; i += nt) P[i] = part[i];
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        for (int i = t; (int64_t)i * 2 * s + s < m; i += nt) P[i * 2 * s] = P[i * 2 * s] + P[i * 2 * s + s];
        __syncthreads();
    }
    const T r = m > 0 ? P[0] : T(0);
    __syncthreads();
    return r;
}

// inner right-hand side: hi(r) * 2^-e rounded to T
template <typename T>
__global__ __launch_bounds__(256) void k_in_stage(int64_t n, const double *__restrict__ r_dd, int e,
                                                  T *__restrict__ r0)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        r0[i] = (T)ldexp(r_dd[i], -e);
}

// d = 0, r = r0, z = M^-1 r, p = z
template <typename T>
__global__ __launch_bounds__(256) void k_in_init(int64_t n, const T *__restrict__ r0, const T *__restrict__ minv,
                                                 T *__restrict__ d, T *__restrict__ r, T *__restrict__ z,
                                                 T *__restrict__ p)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const T ri = r0[i];
        const T zi = minv ? ri * minv[i] : ri;
        d[i] = T(0);
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
    }
}

template <typename T>
__global__ __launch_bounds__(kChunkThreads) void k_in_dot2(int64_t n, const T *__restrict__ x1,
                                                           const T *__restrict__ y1, const T *__restrict__ x2,
                                                           const T *__restrict__ y2, T *__restrict__ part1,
                                                           T *__restrict__ part2, const InState<T> *__restrict__ st)
{
    __shared__ T chain[2][kDotLanes];
    if (st && st->done != RUN) return;
    const int c = xcd_block(blockIdx.x, gridDim.x);
    const int nv = thread_valid(n, c);
    T pr[2][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            pr[0][jj] = x1[k] * y1[k];
            if (x2) pr[1][jj] = x2[k] * y2[k];
        }
    }
    const int used = chunk_used(n, c);
    if (x2) {
        lane_chain<T, 2>(pr, nv, chain);
        T s[2];
        chain_fold_lead<T, 2>(chain, used, s);
        if (threadIdx.x == 0) {
            part1[c] = s[0];
            part2[c] = s[1];
        }
    } else {
        lane_chain<T, 1>(reinterpret_cast<const T(&)[1][kPerThread]>(pr[0]), nv, chain);
        T s[1];
        chain_fold_lead<T, 1>(chain, used, s);
        if (threadIdx.x == 0) part1[c] = s[0];
    }
}

// rho = (r, z), rr0 = (r, r), tolerance
template <typename T>
__global__ __launch_bounds__(256) void k_in_start(const T *__restrict__ prz, const T *__restrict__ prr, int m,
                                                  T irt2, int32_t max_iter, InState<T> *__restrict__ st)
{
    __shared__ T P[kMaxChunks];
    const T rz = pair_tree_t(prz, m, P);
    const T rr = pair_tree_t(prr, m, P);
    if (threadIdx.x == 0) {
        st->rho = rz;
        st->rr0 = rr;
        st->rr = rr;
        st->tol = irt2 * rr;
        st->iters = 0;
        st->max_iter = max_iter;
        st->done = rr <= st->tol ? CONFIRMED : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

// y = A x with each row summed sequentially (one thread per row; the loads of up to
// eight elements are issued before their products are added)
template <typename T>
__global__ __launch_bounds__(256) void k_in_spmv(int64_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                 const T *__restrict__ x, T *__restrict__ y,
                                                 const InState<T> *__restrict__ st)
{
    if (st && st->done != RUN) return;
    for (int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int32_t b = rp[i], e = rp[i + 1];
        T s = T(0);
        for (int32_t k0 = b; k0 < e; k0 += 8) {
            T av[8], xv[8];
            int32_t cv[8];
            // branch-free loads and gathers (a slot past the row's end re-reads its first
            // element), so every gather of the group is in flight at once
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t k = k0 + j < e ? k0 + j : b;
                av[j] = a[k];
                cv[j] = ci[k];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) xv[j] = x[cv[j]];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < e) {
                    const T prod = av[j] * xv[j];
                    s = (k0 + j == b) ? prod : s + prod;
                }
        }
        y[i] = s;
    }
}

// An inner step after q = A p and the chunk sums of (p, q) is, as in the DD CG, an
// update kernel that forms alpha itself and a p kernel that forms beta itself, with
// the inner state double-buffered across the p kernel (st[j & 1] -> st[(j + 1) & 1]).

template <typename T>
__device__ __forceinline__ int32_t in_block_state(const InState<T> *st)
{
    __shared__ int32_t s_done;
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    return s_done;
}

// alpha = rho / (p, q) (breakdown unless (p, q) > 0 and finite); false when not running.
// pre: tree_pre(ppq, m) when m <= 64.
template <typename T>
__device__ __forceinline__ bool in_alpha(const T *__restrict__ ppq, int m, T pre, InState<T> *__restrict__ st,
                                         T *P, T *alpha)
{
    __shared__ T s_rho;
    if (threadIdx.x == 0) s_rho = st->rho;
    if (in_block_state(st) != RUN) return false;
    const T pq = m <= 64 ? tree_wave(pre, m) : pair_tree_t(ppq, m, P);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(pq > T(0)) || !isfinite((double)pq)) {
        if (lead) {
            st->pq = pq;
            st->done = BROKE_DOWN;
        }
        return false;
    }
    *alpha = s_rho / pq;
    if (lead) {
        st->pq = pq;
        st->alpha = *alpha;
    }
    return true;
}

// r -= alpha q; z = M^-1 r (Jacobi or none); chunk sums of (r, z), (r, r) (d += alpha p
// follows in k_in_p).
template <typename T>
__global__ __launch_bounds__(kChunkThreads) void k_in_update(int64_t n, T *__restrict__ r, T *__restrict__ z,
                                                             const T *__restrict__ q, const T *__restrict__ minv,
                                                             const T *__restrict__ ppq, int m, T *__restrict__ prz,
                                                             T *__restrict__ prr, InState<T> *__restrict__ st)
{
    __shared__ T chain[2][kDotLanes];
    __shared__ T P[kMaxChunks];
    const int c = xcd_block(blockIdx.x, gridDim.x);
    const int nv = thread_valid(n, c);
    T rv[kPerThread], qv[kPerThread], mv[kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            rv[jj] = r[k];
            qv[jj] = q[k];
            mv[jj] = minv ? minv[k] : T(0);
        }
    }
    const T pq_pre = m <= 64 ? tree_pre(ppq, m) : T(0);
    T alpha;
    if (!in_alpha(ppq, m, pq_pre, st, P, &alpha)) return;
    T pr[2][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            const T aq = alpha * qv[jj];
            const T rk = rv[jj] - aq;
            r[k] = rk;
            const T zk = minv ? rk * mv[jj] : rk;
            z[k] = zk;
            pr[0][jj] = rk * zk;
            pr[1][jj] = rk * rk;
        }
    }
    lane_chain<T, 2>(pr, nv, chain);
    const int used = chunk_used(n, c);
    T s[2];
    chain_fold_lead<T, 2>(chain, used, s);
    if (threadIdx.x == 0) {
        prz[c] = s[0];
        prr[c] = s[1];
    }
}

// d += alpha p (old p, on the whole grid); rho_new = (r, z), rr = (r, r);
// beta = rho_new / rho; stop tests; p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void k_in_p(int64_t n, T *__restrict__ d, const T *__restrict__ z,
                                              T *__restrict__ p, const T *__restrict__ prz, const T *__restrict__ prr,
                                              int m, const InState<T> *__restrict__ sr, InState<T> *__restrict__ sw)
{
    __shared__ T P[kMaxChunks];
    __shared__ T s_rho, s_tol, s_alpha;
    __shared__ int32_t s_iters, s_max;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const int64_t i0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    T z0 = T(0), p0 = T(0);
    if (i0 < n) {
        z0 = z[i0];
        p0 = p[i0];
    }
    const bool small = m <= 64;
    const T rz_pre = small ? tree_pre(prz, m) : T(0);
    const T rr_pre = small ? tree_pre(prr, m) : T(0);
    if (threadIdx.x == 0) {
        s_rho = sr->rho;
        s_tol = sr->tol;
        s_alpha = sr->alpha;
        s_iters = sr->iters;
        s_max = sr->max_iter;
    }
    if (in_block_state(sr) != RUN) {
        if (lead) *sw = *sr;
        return;
    }
    // the update kernel ran to the end with this alpha
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * 256) {
        const T ap = s_alpha * (i == i0 ? p0 : p[i]);
        d[i] = d[i] + ap;
    }
    // wavefront 0 reduces the chunk sums (a single tree per workgroup) and thread 0 decides
    // the step for the workgroup
    __shared__ T s_rz, s_rr, s_beta;
    __shared__ int32_t s_next;
    T rz = T(0), rr = T(0);
    if (small) {
        if (threadIdx.x < 64) {
            rz = tree_wave(rz_pre, m);
            rr = tree_wave(rr_pre, m);
        }
    } else {
        rz = pair_tree_t(prz, m, P);
        rr = pair_tree_t(prr, m, P);
    }
    if (threadIdx.x == 0) {
        int32_t d = RUN;
        T bt = T(0);
        if (!isfinite((double)rr) || !isfinite((double)rz)) {
            d = BROKE_DOWN;
        } else {
            bt = rz / s_rho;
            if (rr <= s_tol)
                d = CONFIRMED;
            else if (s_iters + 1 >= s_max)
                d = ITER_LIMIT;
        }
        s_rz = rz;
        s_rr = rr;
        s_beta = bt;
        s_next = d;
    }
    __syncthreads();
    const int32_t iters = s_iters + 1;
    const int32_t done = s_next;
    const T beta = s_beta;
    rz = s_rz;
    rr = s_rr;
    if (lead) {
        InState<T> o = *sr;
        o.iters = iters;
        o.rr = rr;
        if (done != BROKE_DOWN) {
            o.beta = beta;
            o.rho = rz;
        }
        o.done = done;
        *sw = o;
    }
    if (done != RUN) return;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * 256) {
        const T bp = beta * (i == i0 ? p0 : p[i]);
        p[i] = (i == i0 ? z0 : z[i]) + bp;
    }
}

// An inner step with the learned preconditioner, after q = A p and the chunk sums of
// (p, q): alpha = rho / (p, q) in every workgroup, then for each row i
//   r_next[i] = r[i] - alpha q[i],   z[i] = sum_k M[i,k] (r[c_k] - alpha q[c_k]),
// the neighbours' new residual recomputed from the old r and q with the same two
// roundings, so z = M r_next without a grid-wide wait for r_next.  r and r_next are
// two buffers that alternate from step to step.
template <typename T>
__global__ __launch_bounds__(256) void k_in_mupdate(int64_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, const T *__restrict__ mv,
                                                    const T *__restrict__ r, const T *__restrict__ q,
                                                    T *__restrict__ r_next, T *__restrict__ z,
                                                    const T *__restrict__ ppq, int m, InState<T> *__restrict__ st)
{
    __shared__ T P[kMaxChunks];
    const T pq_pre = m <= 64 ? tree_pre(ppq, m) : T(0);
    T alpha;
    if (!in_alpha(ppq, m, pq_pre, st, P, &alpha)) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t b = rp[i], e = rp[i + 1];
        const T aqi = alpha * q[i];
        r_next[i] = r[i] - aqi;
        T s = T(0);
        for (int32_t k0 = b; k0 < e; k0 += 8) {
            T av[8], rv[8], qv[8];
            int32_t cv[8];
            // branch-free loads and gathers (a slot past the row's end re-reads its first
            // element), so every gather of the group is in flight at once
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t k = k0 + j < e ? k0 + j : b;
                av[j] = mv[k];
                cv[j] = ci[k];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                rv[j] = r[cv[j]];
                qv[j] = q[cv[j]];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < e) {
                    const T aq = alpha * qv[j];
                    const T rn = rv[j] - aq;
                    const T prod = av[j] * rn;
                    s = (k0 + j == b) ? prod : s + prod;
                }
        }
        z[i] = s;
    }
}

// z = M r with M given by its values on A's pattern, rows summed sequentially; when
// p is given, p = z as well (start of the inner solve, st may then be NULL)
template <typename T>
__global__ __launch_bounds__(256) void k_in_mspmv(int64_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const T *__restrict__ mv,
                                                  const T *__restrict__ r, T *__restrict__ z, T *__restrict__ p,
                                                  const InState<T> *__restrict__ st)
{
    if (st && st->done != RUN) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t b = rp[i], e = rp[i + 1];
        T s = T(0);
        for (int32_t k0 = b; k0 < e; k0 += 8) {
            T av[8], xv[8];
            int32_t cv[8];
            // branch-free loads and gathers (a slot past the row's end re-reads its first
            // element), so every gather of the group is in flight at once
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int32_t k = k0 + j < e ? k0 + j : b;
                av[j] = mv[k];
                cv[j] = ci[k];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) xv[j] = r[cv[j]];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < e) {
                    const T prod = av[j] * xv[j];
                    s = (k0 + j == b) ? prod : s + prod;
                }
        }
        z[i] = s;
        if (p) p[i] = s;
    }
}

// x_i = DDadd(x_i, (d_i * 2^e, 0))
template <typename T>
__global__ __launch_bounds__(256) void k_ir_update(int64_t n, double *__restrict__ x, const T *__restrict__ d, int e)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        dd_t dv;
        dv.c[0] = ldexp((double)d[i], e);
        dv.c[1] = 0.0;
        sdd(x, n, i, dd_add(ldd(x, n, i), dv));
    }
}

// max |v_i| per chunk of 4096 (exact, order-free)
__global__ __launch_bounds__(256) void k_maxabs(int64_t n, const double *__restrict__ v, double *__restrict__ part)
{
    __shared__ double lds[kDotLanes];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)c * kDotChunk;
    const int64_t end = (n - base) < kDotChunk ? n : base + kDotChunk;
    double m = 0.0;
    for (int64_t k = base + t; k < end; k += kDotLanes) m = fmax(m, fabs(v[k]));
    lds[t] = m;
    __syncthreads();
    for (int off = kDotLanes / 2; off >= 1; off >>= 1) {
        if (t < off) lds[t] = fmax(lds[t], lds[t + off]);
        __syncthreads();
    }
    if (t == 0) part[c] = lds[0];
}

__global__ __launch_bounds__(256) void k_maxabs_final(const double *__restrict__ part, int m, double *__restrict__ out)
{
    __shared__ double lds[kDotLanes];
    const int t = threadIdx.x;
    double v = 0.0;
    for (int i = t; i < m; i += kDotLanes) v = fmax(v, part[i]);
    lds[t] = v;
    __syncthreads();
    for (int off = kDotLanes / 2; off >= 1; off >>= 1) {
        if (t < off) lds[t] = fmax(lds[t], lds[t + off]);
        __syncthreads();
    }
    if (t == 0) *out = lds[0];
}

__global__ __launch_bounds__(256) void k_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = (float)src[i];
}

// bb and tolerance of the refinement, rr of the current residual
__global__ __launch_bounds__(256) void k_ir_norms(const dd_t *__restrict__ pbb, const dd_t *__restrict__ prr, int m,
                                                  double rtol2, int first, KState *__restrict__ st)
{
    __shared__ dd_t P[kMaxChunks];
    const dd_t rr = pair_tree(prr, m, P);
    dd_t bb = dd_zero();
    if (first) bb = pair_tree(pbb, m, P);
    if (threadIdx.x == 0) {
        if (first) {
            st->bb = bb;
            st->tol2 = dd_mul_d(bb, rtol2);
        }
        st->rr = rr;
        st->rr_true = rr;
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

constexpr int kVecs = 12;   // DD work vectors (GPBiCG uses all of them)
constexpr int kParts = 6;   // chunk-sum arrays

struct Workspace {
    KState *st;
    KState *st2;   // second state buffer of the CG step (double-buffered)
    double *minv;
    double *v[kVecs];
    dd_t *part[kParts];
    double *xs;    // interleaved copy of x that the planned SpMV gathers from
    void *inner;   // InState<T>
    float *a32;
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t workspace_bytes(int64_t n, int64_t nnz_f32 = 0)
{
    size_t b = 2 * align256(sizeof(KState));
    b += align256(sizeof(double) * (size_t)n);
    b += kVecs * align256(sizeof(double) * 2 * (size_t)n);
    b += kParts * align256(sizeof(dd_t) * kMaxChunks);
    b += align256(sizeof(double) * 2 * (size_t)n);    // staged x of the planned SpMV
    b += 256;                                         // inner-solver state
    b += align256(sizeof(float) * (size_t)nnz_f32);   // binary32 copies of hi(A) (and of M)
    return b;
}

Workspace carve(void *ws, int64_t n)
{
    Workspace w;
    char *p = static_cast<char *>(ws);
    w.st = reinterpret_cast<KState *>(p);
    p += align256(sizeof(KState));
    w.st2 = reinterpret_cast<KState *>(p);
    p += align256(sizeof(KState));
    w.minv = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * (size_t)n);
    for (int i = 0; i < kVecs; ++i) {
        w.v[i] = reinterpret_cast<double *>(p);
        p += align256(sizeof(double) * 2 * (size_t)n);
    }
    for (int i = 0; i < kParts; ++i) {
        w.part[i] = reinterpret_cast<dd_t *>(p);
        p += align256(sizeof(dd_t) * kMaxChunks);
    }
    w.xs = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * 2 * (size_t)n);
    w.inner = p;
    p += 256;
    w.a32 = reinterpret_cast<float *>(p);
    return w;
}

bool host_dd_le(const double *a, const double *b) { return (a[0] < b[0]) || (a[0] == b[0] && a[1] <= b[1]); }

mp_status spmv_dispatch(int K, bool cplx, const mp_csr *A, const double *a_re, const double *a_im,
                        const double *x_re, const double *x_im, double *y_re, double *y_im, const mp_plan *plan,
                        double *xs, hipStream_t s);

struct Solver {
    const mp_csr *A;
    const double *a;
    const mp_plan *plan;
    hipStream_t s;
    int64_t n;
    int m;            // chunks
    unsigned vblocks;  // blocks of the element-wise kernels
    Workspace w;

    mp_status spmv(const double *xin, double *yout)
    {
        return spmv_dispatch(2, false, A, a, nullptr, xin, nullptr, yout, nullptr, plan, w.xs, s);
    }
    mp_status launched()
    {
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
    mp_status dot2(const double *x1, const double *y1, const double *x2, const double *y2, dd_t *p1, dd_t *p2,
                   const KState *guard)
    {
        hipLaunchKernelGGL(k_dot2, dim3(m), dim3(kChunkThreads), 0, s, n, x1, y1, x2, y2, p1, p2, guard);
        return launched();
    }
    // r = b - A x (q scratch)
    mp_status residual(const double *b, const double *x, double *q, double *r)
    {
        mp_status st = spmv(x, q);
        if (st != MP_OK) return st;
        hipLaunchKernelGGL(k_residual, dim3(vblocks), dim3(256), 0, s, n, b, q, r);
        return launched();
    }
    mp_status read_state(KState *h)
    {
        MP_HIP_TRY(hipMemcpyAsync(h, w.st, sizeof(KState), hipMemcpyDeviceToHost, s));
        MP_HIP_TRY(hipStreamSynchronize(s));
        return MP_OK;
    }
    // true residual of x into r, rr_true into the state (confirm = test against tol2)
    mp_status true_residual(const double *b, const double *x, double *q, double *r, bool confirm)
    {
        mp_status st = residual(b, x, q, r);
        if (st == MP_OK) st = dot2(r, r, nullptr, nullptr, w.part[0], nullptr, nullptr);
        if (st != MP_OK) return st;
        if (confirm)
            hipLaunchKernelGGL(k_confirm, dim3(1), dim3(256), 0, s, w.part[0], m, w.st);
        else
            hipLaunchKernelGGL(k_exit_rr, dim3(1), dim3(256), 0, s, w.part[0], m, w.st);
        return launched();
    }
};

mp_status check_solver_args(const char *name, const mp_csr *A, const double *a, const double *b, const double *x,
                            const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes, size_t need,
                            mp_solve_info *info, bool learned)
{
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (!opts || !info) return fail(MP_ERR_INVALID_ARG, "%s: opts or info is NULL", name);
    if (A->n_rows != A->n_cols) return fail(MP_ERR_INVALID_ARG, "%s: matrix must be square", name);
    if (A->n_rows > 0 && (!b || !x || !ws)) return fail(MP_ERR_INVALID_ARG, "%s: b, x or workspace is NULL", name);
    if (A->nnz > 0 && !a) return fail(MP_ERR_INVALID_ARG, "%s: a is NULL", name);
    if ((int64_t)A->n_rows > (int64_t)kMaxChunks * kDotChunk)
        return fail(MP_ERR_UNSUPPORTED, "%s: n = %d exceeds the solver limit %d", name, A->n_rows,
                    kMaxChunks * kDotChunk);
    if (ws_bytes < need)
        return fail(MP_ERR_NO_MEMORY, "%s: workspace of %zu bytes, %zu needed", name, ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MP_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", name);
    if (opts->precond == MP_PRECOND_LEARNED) {
        if (!learned) return fail(MP_ERR_INVALID_ARG, "%s: the learned preconditioner needs mpkrylov_ir_learned", name);
    } else if (learned) {
        return fail(MP_ERR_INVALID_ARG, "%s: opts.precond must be MP_PRECOND_LEARNED", name);
    } else if (opts->precond != MP_PRECOND_NONE && opts->precond != MP_PRECOND_JACOBI) {
        return fail(MP_ERR_INVALID_ARG, "%s: unknown preconditioner %d", name, opts->precond);
    }
    if (!(opts->rtol >= 0.0)) return fail(MP_ERR_INVALID_ARG, "%s: rtol must be >= 0", name);
    if (plan && (plan->ncomp != 2 || plan->cplx || plan->n_rows != A->n_rows || plan->nnz != A->nnz))
        return fail(MP_ERR_INVALID_ARG, "%s: plan is not a DD real plan of this matrix", name);
    const size_t vb = sizeof(double) * 2 * (size_t)A->n_rows;
    if (overlaps(x, vb, b, vb) || overlaps(x, vb, a, sizeof(double) * 2 * (size_t)A->nnz) ||
        overlaps(x, vb, ws, ws_bytes) || overlaps(b, vb, ws, ws_bytes))
        return fail(MP_ERR_ALIAS, "%s: x overlaps b, a or the workspace", name);
    return MP_OK;
}

void fill_info(const KState &h, int status, double secs, mp_solve_info *info)
{
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->iters = h.iters;
    info->restarts = h.restarts;
    info->rr_true[0] = h.rr_true.c[0];
    info->rr_true[1] = h.rr_true.c[1];
    info->bb[0] = h.bb.c[0];
    info->bb[1] = h.bb.c[1];
    info->relres = h.bb.c[0] > 0 ? std::sqrt(h.rr_true.c[0] / h.bb.c[0]) : std::sqrt(h.rr_true.c[0]);
    info->seconds = secs;
    info->fell_back = 0;
}

mp_status run_cg(Solver &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.w.v[0], *z = S.w.v[1], *p = S.w.v[2], *q = S.w.v[3];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.w.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    mp_status st = MP_OK;
    KState h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    if (minv) {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                           S.w.minv);
        if ((st = S.launched()) != MP_OK) return st;
    }
    // start: r = b - A x, z = M^-1 r, p = z, bb, rho, rr
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_precond, dim3(S.vblocks), dim3(256), 0, S.s, n, minv, r, z, nullptr);
    hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, z, p);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = spmv_stage_x(2, false, S.A, p, nullptr, S.plan, S.w.xs, S.s)) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, z, S.w.part[0], S.w.part[1], nullptr)) != MP_OK) return st;
    if ((st = S.dot2(r, r, nullptr, nullptr, S.w.part[2], nullptr, nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], S.w.part[2], m,
                       o->rtol * o->rtol, o->max_iter, S.w.st);
    if ((st = S.launched()) != MP_OK) return st;
    int status = MP_ERR_NOT_CONVERGED;
    double *xs = plan_stage_bytes(S.plan) ? S.w.xs : nullptr;   // k_cg_p stages the next p there
    KState *sb[2] = {S.w.st, S.w.st2};
    const int steps = (every + 1) & ~1;   // even: a chunk ends with the state in sb[0]
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < steps; ++it) {
                KState *sr = sb[it & 1], *sw = sb[(it + 1) & 1];
                if ((st = spmv_dd_prestaged(S.A, S.a, p, q, S.plan, S.w.xs, S.s)) != MP_OK) return st;
                if ((st = S.dot2(p, q, nullptr, nullptr, S.w.part[0], nullptr, sr)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cg_update, dim3(m), dim3(kChunkThreads), 0, S.s, n, r, z, q, minv, S.w.part[0], m,
                                   S.w.part[1], S.w.part[2], sr);
                hipLaunchKernelGGL(k_cg_p, dim3(S.vblocks), dim3(256), 0, S.s, n, x, z, p, xs, S.w.part[1],
                                   S.w.part[2], m, sr, sw);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, q, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_precond, dim3(S.vblocks), dim3(256), 0, S.s, n, minv, r, z, nullptr);
            hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, z, p);
            if ((st = S.launched()) != MP_OK) return st;
            if ((st = spmv_stage_x(2, false, S.A, p, nullptr, S.plan, S.w.xs, S.s)) != MP_OK) return st;
            if ((st = S.dot2(r, z, nullptr, nullptr, S.w.part[1], nullptr, nullptr)) != MP_OK) return st;
            hipLaunchKernelGGL(k_cg_restart, dim3(1), dim3(256), 0, S.s, S.w.part[1], m, S.w.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        break;
    }
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_cg: no convergence in %d iterations", h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "mpkrylov_cg: breakdown at iteration %d", h.iters);
    return MP_OK;
}

// BiCG driver: A^T (At, at) with an optional plan of its own
mp_status run_bicg(Solver &S, const mp_csr *At, const double *at, const mp_plan *plan_t, const double *b, double *x,
                   const mp_solve_opts *o, mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.w.v[0], *z = S.w.v[1], *p = S.w.v[2], *q = S.w.v[3];
    double *rt = S.w.v[4], *zt = S.w.v[5], *pt = S.w.v[6], *qt = S.w.v[7];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.w.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    mp_status st = MP_OK;
    KState h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    if (minv) {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                           S.w.minv);
        if ((st = S.launched()) != MP_OK) return st;
    }
    // shadow start r~ = r; z = M^-1 r; z~ = p = p~ = z
    auto reset = [&]() -> mp_status {
        hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rt);
        hipLaunchKernelGGL(k_precond, dim3(S.vblocks), dim3(256), 0, S.s, n, minv, r, z, nullptr);
        hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, z, zt);
        hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, z, p);
        hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, z, pt);
        return S.launched();
    };
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    if ((st = reset()) != MP_OK) return st;
    if ((st = S.dot2(b, b, rt, z, S.w.part[0], S.w.part[1], nullptr)) != MP_OK) return st;
    if ((st = S.dot2(r, r, nullptr, nullptr, S.w.part[2], nullptr, nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], S.w.part[2], m,
                       o->rtol * o->rtol, o->max_iter, S.w.st);
    if ((st = S.launched()) != MP_OK) return st;
    int status = MP_ERR_NOT_CONVERGED;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.spmv(p, q)) != MP_OK) return st;
                if ((st = spmv_dispatch(2, false, At, at, nullptr, pt, nullptr, qt, nullptr, plan_t, S.w.xs, S.s)) != MP_OK)
                    return st;
                if ((st = S.dot2(pt, q, nullptr, nullptr, S.w.part[0], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bicg_alpha, dim3(1), dim3(256), 0, S.s, S.w.part[0], m, S.w.st);
                hipLaunchKernelGGL(k_bicg_update, dim3(m), dim3(256), 0, S.s, n, x, r, z, p, q, rt, zt, qt, minv,
                                   S.w.part[1], S.w.part[2], S.w.st);
                hipLaunchKernelGGL(k_bicg_beta, dim3(1), dim3(256), 0, S.s, S.w.part[1], S.w.part[2], m, S.w.st);
                hipLaunchKernelGGL(k_bicg_p, dim3(S.vblocks), dim3(256), 0, S.s, n, z, p, zt, pt, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, q, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            if ((st = reset()) != MP_OK) return st;
            if ((st = S.dot2(rt, z, nullptr, nullptr, S.w.part[1], nullptr, nullptr)) != MP_OK) return st;
            hipLaunchKernelGGL(k_cg_restart, dim3(1), dim3(256), 0, S.s, S.w.part[1], m, S.w.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        break;
    }
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    if (status == MP_ERR_NOT_CONVERGED)
        return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_bicg: no convergence in %d iterations", h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "mpkrylov_bicg: breakdown at iteration %d", h.iters);
    return MP_OK;
}

mp_status run_cgs(Solver &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.w.v[0], *rh = S.w.v[1], *u = S.w.v[2], *p = S.w.v[3], *q = S.w.v[4], *v = S.w.v[5];
    double *uh = S.w.v[6], *t = S.w.v[7], *ph = S.w.v[8];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.w.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    mp_status st = MP_OK;
    KState h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    if (minv) {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                           S.w.minv);
        if ((st = S.launched()) != MP_OK) return st;
    }
    if ((st = S.residual(b, x, t, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, S.w.part[0], S.w.part[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cgs_init, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], m, o->rtol * o->rtol,
                       o->max_iter, S.w.st);
    if ((st = S.launched()) != MP_OK) return st;
    int status = MP_ERR_NOT_CONVERGED;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, S.w.part[0], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_rho, dim3(1), dim3(256), 0, S.s, S.w.part[0], m, S.w.st);
                hipLaunchKernelGGL(k_cgs_up, dim3(S.vblocks), dim3(256), 0, S.s, n, r, q, u, p, ph, minv, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(ph, v)) != MP_OK) return st;
                if ((st = S.dot2(rh, v, nullptr, nullptr, S.w.part[1], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_alpha, dim3(1), dim3(256), 0, S.s, S.w.part[1], m, S.w.st);
                hipLaunchKernelGGL(k_cgs_q, dim3(S.vblocks), dim3(256), 0, S.s, n, u, v, q, uh, x, minv, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(uh, t)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_r, dim3(m), dim3(256), 0, S.s, n, r, t, S.w.part[2], S.w.st);
                hipLaunchKernelGGL(k_cgs_rr, dim3(1), dim3(256), 0, S.s, S.w.part[2], m, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, t, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
            hipLaunchKernelGGL(k_cgs_restart, dim3(1), dim3(64), 0, S.s, S.w.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        break;
    }
    if ((st = S.true_residual(b, x, t, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    if (status == MP_ERR_NOT_CONVERGED)
        return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_cgs: no convergence in %d iterations", h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "mpkrylov_cgs: breakdown at iteration %d", h.iters);
    return MP_OK;
}

mp_status run_gpbicg(Solver &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.w.v[0], *rh = S.w.v[1], *p = S.w.v[2], *q = S.w.v[3], *t = S.w.v[4], *c = S.w.v[5];
    double *y = S.w.v[6], *u = S.w.v[7], *z = S.w.v[8], *w = S.w.v[9], *tp = S.w.v[10], *tmp = S.w.v[11];
    dd_t **P = S.w.part;
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.w.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    mp_status st = MP_OK;
    KState h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    if (minv) {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                           S.w.minv);
        if ((st = S.launched()) != MP_OK) return st;
    }
    if ((st = S.residual(b, x, tmp, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, P[0], P[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cgs_init, dim3(1), dim3(256), 0, S.s, P[0], P[1], m, o->rtol * o->rtol, o->max_iter,
                       S.w.st);
    if ((st = S.launched()) != MP_OK) return st;
    int status = MP_ERR_NOT_CONVERGED;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, P[0], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_rho, dim3(1), dim3(256), 0, S.s, P[0], m, S.w.st);
                hipLaunchKernelGGL(k_gp_p, dim3(S.vblocks), dim3(256), 0, S.s, n, r, p, u, c, q, w, tmp, minv, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(tmp, q)) != MP_OK) return st;
                if ((st = S.dot2(rh, q, nullptr, nullptr, P[1], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_alpha, dim3(1), dim3(256), 0, S.s, P[1], m, S.w.st);
                hipLaunchKernelGGL(k_gp_t, dim3(m), dim3(256), 0, S.s, n, r, q, tp, w, t, y, tmp, minv, P[2], S.w.st);
                hipLaunchKernelGGL(k_gp_tt, dim3(1), dim3(256), 0, S.s, P[2], m, S.w.st);
                hipLaunchKernelGGL(k_gp_half, dim3(S.vblocks), dim3(256), 0, S.s, n, x, r, p, t, minv, S.w.st);
                hipLaunchKernelGGL(k_gp_half_final, dim3(1), dim3(64), 0, S.s, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(tmp, c)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_dots, dim3(m), dim3(kChunkThreads), 0, S.s, n, c, t, y, P[0], P[1], P[2], P[3],
                                   P[4], S.w.st);
                hipLaunchKernelGGL(k_gp_zeta, dim3(1), dim3(256), 0, S.s, P[0], P[1], P[2], P[3], P[4], m, S.w.st);
                hipLaunchKernelGGL(k_gp_update, dim3(m), dim3(256), 0, S.s, n, x, r, p, q, t, c, y, u, z, tp, minv,
                                   P[5], S.w.st);
                hipLaunchKernelGGL(k_gp_rr, dim3(1), dim3(256), 0, S.s, P[5], m, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, tmp, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
            hipLaunchKernelGGL(k_cgs_restart, dim3(1), dim3(64), 0, S.s, S.w.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        break;
    }
    if ((st = S.true_residual(b, x, tmp, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    if (status == MP_ERR_NOT_CONVERGED)
        return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_gpbicg: no convergence in %d iterations", h.iters);
    if (status == MP_ERR_BREAKDOWN)
        return fail(MP_ERR_BREAKDOWN, "mpkrylov_gpbicg: breakdown at iteration %d", h.iters);
    return MP_OK;
}

mp_status run_bicgstab(Solver &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.w.v[0], *rh = S.w.v[1], *p = S.w.v[2], *v = S.w.v[3], *ph = S.w.v[4], *s = S.w.v[5];
    double *sh = S.w.v[6], *tv = S.w.v[7], *q = S.w.v[8];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.w.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    mp_status st = MP_OK;
    KState h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    if (minv) {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                           S.w.minv);
        if ((st = S.launched()) != MP_OK) return st;
    }
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, S.w.part[0], S.w.part[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_bi_init, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], m, o->rtol * o->rtol,
                       o->max_iter, S.w.st);
    if ((st = S.launched()) != MP_OK) return st;
    int status = MP_ERR_NOT_CONVERGED;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, S.w.part[0], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_rho, dim3(1), dim3(256), 0, S.s, S.w.part[0], m, S.w.st);
                hipLaunchKernelGGL(k_bi_p, dim3(S.vblocks), dim3(256), 0, S.s, n, r, p, v, S.w.st);
                hipLaunchKernelGGL(k_precond, dim3(S.vblocks), dim3(256), 0, S.s, n, minv, p, ph, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(ph, v)) != MP_OK) return st;
                if ((st = S.dot2(rh, v, nullptr, nullptr, S.w.part[0], nullptr, S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_alpha, dim3(1), dim3(256), 0, S.s, S.w.part[0], m, S.w.st);
                hipLaunchKernelGGL(k_bi_s, dim3(m), dim3(256), 0, S.s, n, r, v, s, S.w.part[0], S.w.st);
                hipLaunchKernelGGL(k_bi_ss, dim3(1), dim3(256), 0, S.s, S.w.part[0], m, S.w.st);
                hipLaunchKernelGGL(k_bi_half, dim3(S.vblocks), dim3(256), 0, S.s, n, x, r, ph, s, S.w.st);
                hipLaunchKernelGGL(k_bi_half_final, dim3(1), dim3(64), 0, S.s, S.w.st);
                hipLaunchKernelGGL(k_precond, dim3(S.vblocks), dim3(256), 0, S.s, n, minv, s, sh, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(sh, tv)) != MP_OK) return st;
                if ((st = S.dot2(tv, s, tv, tv, S.w.part[0], S.w.part[1], S.w.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_omega, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], m, S.w.st);
                hipLaunchKernelGGL(k_bi_xr, dim3(m), dim3(256), 0, S.s, n, x, r, ph, sh, s, tv, S.w.part[2], S.w.st);
                hipLaunchKernelGGL(k_bi_rr, dim3(1), dim3(256), 0, S.s, S.w.part[2], m, S.w.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, q, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, 2 * n, r, rh);
            hipLaunchKernelGGL(k_bi_restart, dim3(1), dim3(64), 0, S.s, S.w.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
        break;
    }
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    if (status == MP_ERR_NOT_CONVERGED)
        return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_bicgstab: no convergence in %d iterations", h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "mpkrylov_bicgstab: breakdown at iteration %d", h.iters);
    return MP_OK;
}

template <typename T>
mp_status inner_solve(Solver &S, const double *r_dd, int e, const T *a_in, const T *minv, const T *mv, T *d,
                      double inner_rtol, int max_iter, int every, int *iters, int *status)
{
    const int64_t n = S.n;
    const int m = S.m;
    InState<T> *ist = static_cast<InState<T> *>(S.w.inner);
    T *r0 = reinterpret_cast<T *>(S.w.v[5]);
    T *r = r0 + n, *z = reinterpret_cast<T *>(S.w.v[6]), *p = z + n, *q = reinterpret_cast<T *>(S.w.v[7]);
    T *part0 = reinterpret_cast<T *>(S.w.part[0]), *part1 = reinterpret_cast<T *>(S.w.part[1]);
    T *part2 = reinterpret_cast<T *>(S.w.part[2]);
    mp_status st;
    hipLaunchKernelGGL(k_in_stage<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, r_dd, e, r0);
    hipLaunchKernelGGL(k_in_init<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, r0, mv ? nullptr : minv, d, r, z, p);
    if (mv)
        hipLaunchKernelGGL(k_in_mspmv<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, mv, r, z,
                           p, nullptr);
    hipLaunchKernelGGL(k_in_dot2<T>, dim3(m), dim3(kChunkThreads), 0, S.s, n, r, z, r, r, part1, part2, nullptr);
    hipLaunchKernelGGL(k_in_start<T>, dim3(1), dim3(256), 0, S.s, part1, part2, m, (T)(inner_rtol * inner_rtol),
                       max_iter, ist);
    if ((st = S.launched()) != MP_OK) return st;
    InState<T> h;
    InState<T> *sb[2] = {ist, ist + 1};
    const int steps = (every + 1) & ~1;   // even: a chunk ends with the state in sb[0]
    for (;;) {
        MP_HIP_TRY(hipMemcpyAsync(&h, ist, sizeof(h), hipMemcpyDeviceToHost, S.s));
        MP_HIP_TRY(hipStreamSynchronize(S.s));
        if (h.done != RUN) break;
        for (int it = 0; it < steps; ++it) {
            InState<T> *sr = sb[it & 1], *sw = sb[(it + 1) & 1];
            hipLaunchKernelGGL(k_in_spmv<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx,
                               a_in, p, q, sr);
            hipLaunchKernelGGL(k_in_dot2<T>, dim3(m), dim3(kChunkThreads), 0, S.s, n, p, q, nullptr, nullptr, part0, nullptr,
                               sr);
            if (mv) {
                // the residual alternates between r and r0 (free after the start)
                T *rc = (it & 1) ? r0 : r, *rn = (it & 1) ? r : r0;
                hipLaunchKernelGGL(k_in_mupdate<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr,
                                   S.A->col_idx, mv, rc, q, rn, z, part0, m, sr);
                hipLaunchKernelGGL(k_in_dot2<T>, dim3(m), dim3(kChunkThreads), 0, S.s, n, rn, z, rn, rn, part1, part2,
                                   sr);
            } else {
                hipLaunchKernelGGL(k_in_update<T>, dim3(m), dim3(kChunkThreads), 0, S.s, n, r, z, q, minv, part0, m,
                                   part1, part2, sr);
            }
            hipLaunchKernelGGL(k_in_p<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, d, z, p, part1, part2, m, sr, sw);
            if ((st = S.launched()) != MP_OK) return st;
        }
    }
    *iters = h.iters;
    *status = h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
    return MP_OK;
}

template <typename T>
mp_status run_ir_t(Solver &S, const double *b, double *x, const double *mvals, const mp_solve_opts *o,
                   mp_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    const bool jacobi = o->precond == MP_PRECOND_JACOBI;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int inner_max = o->inner_max_iter > 0 ? o->inner_max_iter : o->max_iter;
    double *r = S.w.v[0], *q = S.w.v[3];
    T *d = reinterpret_cast<T *>(S.w.v[4]);
    T *minvT = reinterpret_cast<T *>(S.w.v[8]);
    double *maxpart = reinterpret_cast<double *>(S.w.v[8]) + n;   // after the inner inverse diagonal
    double *maxabs = &static_cast<InState<T> *>(S.w.inner)->maxabs;
    const T *a_in;
    const T *mv_in = nullptr;
    mp_status st;
    MP_HIP_TRY(hipMemsetAsync(S.w.st, 0, sizeof(KState), S.s));
    hipLaunchKernelGGL(k_jacobi_minv, dim3(S.vblocks), dim3(256), 0, S.s, n, S.A->row_ptr, S.A->col_idx, S.a,
                       S.w.minv);
    if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL(k_to_f32, dim3(S.vblocks), dim3(256), 0, S.s, n, S.w.minv, reinterpret_cast<float *>(minvT));
        const int64_t ab = (S.A->nnz + 255) / 256;
        if (S.A->nnz > 0)
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)(ab < 8192 ? ab : 8192)), dim3(256), 0, S.s, S.A->nnz, S.a,
                               S.w.a32);
        a_in = reinterpret_cast<const T *>(S.w.a32);
        if (mvals) {
            float *m32 = S.w.a32 + ((S.A->nnz + 63) & ~(int64_t)63);
            if (S.A->nnz > 0)
                hipLaunchKernelGGL(k_to_f32, dim3((unsigned)(ab < 8192 ? ab : 8192)), dim3(256), 0, S.s, S.A->nnz,
                                   mvals, m32);
            mv_in = reinterpret_cast<const T *>(m32);
        }
    } else {
        hipLaunchKernelGGL(k_copy, dim3(S.vblocks), dim3(256), 0, S.s, n, S.w.minv, reinterpret_cast<double *>(minvT));
        a_in = reinterpret_cast<const T *>(S.a);
        if (mvals) mv_in = reinterpret_cast<const T *>(mvals);
    }
    if ((st = S.launched()) != MP_OK) return st;
    const T *minv_in = jacobi ? minvT : nullptr;
    KState h;
    std::memset(&h, 0, sizeof(h));
    int outer = 0, status = MP_ERR_NOT_CONVERGED, total_inner = 0;
    bool stalled = false;
    double prev = 0.0, prev2 = 0.0;
    for (;;) {
        if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
        if ((st = S.dot2(r, r, b, b, S.w.part[1], S.w.part[0], nullptr)) != MP_OK) return st;
        hipLaunchKernelGGL(k_ir_norms, dim3(1), dim3(256), 0, S.s, S.w.part[0], S.w.part[1], m, o->rtol * o->rtol,
                           outer == 0 ? 1 : 0, S.w.st);
        hipLaunchKernelGGL(k_maxabs, dim3(m), dim3(256), 0, S.s, n, r, maxpart);
        hipLaunchKernelGGL(k_maxabs_final, dim3(1), dim3(256), 0, S.s, maxpart, m, maxabs);
        if ((st = S.launched()) != MP_OK) return st;
        if ((st = S.read_state(&h)) != MP_OK) return st;
        double mx = 0.0;
        MP_HIP_TRY(hipMemcpyAsync(&mx, maxabs, sizeof(double), hipMemcpyDeviceToHost, S.s));
        MP_HIP_TRY(hipStreamSynchronize(S.s));
        const double rr[2] = {h.rr.c[0], h.rr.c[1]}, tol2[2] = {h.tol2.c[0], h.tol2.c[1]};
        if (host_dd_le(rr, tol2)) {
            status = MP_OK;
            break;
        }
        if (!std::isfinite(rr[0])) {
            status = MP_ERR_BREAKDOWN;
            break;
        }
        if ((outer >= 2 && rr[0] > 0.25 * prev && prev > 0.25 * prev2) || outer >= o->max_outer) {
            stalled = true;
            break;
        }
        prev2 = prev;
        prev = rr[0];
        int e = 0;
        (void)std::frexp(mx, &e);
        int it = 0, ist = 0;
        if ((st = inner_solve<T>(S, r, e, a_in, minv_in, mv_in, d, o->inner_rtol, inner_max, every, &it, &ist)) !=
            MP_OK)
            return st;
        total_inner += it;
        hipLaunchKernelGGL(k_ir_update<T>, dim3(S.vblocks), dim3(256), 0, S.s, n, x, d, e);
        if ((st = S.launched()) != MP_OK) return st;
        outer++;
    }
    int fell_back = 0, restarts = 0;
    if (stalled) {
        mp_solve_opts co = *o;
        mp_solve_info ci;
        fell_back = 1;
        if (mvals) co.precond = MP_PRECOND_JACOBI;   // a learned inner M falls back to plain Jacobi DD CG
        st = run_cg(S, b, x, &co, &ci);
        if (st != MP_OK && st != MP_ERR_NOT_CONVERGED && st != MP_ERR_BREAKDOWN) return st;
        status = ci.status;
        total_inner += ci.iters;
        restarts = ci.restarts;
    }
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(h, status, secs, info);
    info->iters = total_inner;
    info->outer_iters = outer;
    info->restarts = restarts;
    info->fell_back = fell_back;
    clear_error();
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "mpkrylov_ir: not converged");
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "mpkrylov_ir: breakdown");
    return MP_OK;
}

// bytes of workspace: binary32 copies of hi(A) (and of M for the learned inner
// preconditioner) only for a binary32 inner solve
size_t solver_bytes(const mp_csr *A, const mp_solve_opts *o)
{
    if (!A) return 0;
    int64_t f32 = 0;
    if (o && o->inner == MP_INNER_FP32) {
        f32 = A->nnz;
        if (o->precond == MP_PRECOND_LEARNED) f32 = ((A->nnz + 63) & ~(int64_t)63) + A->nnz;
    }
    return workspace_bytes(A->n_rows, f32);
}

// kind: 0 CG, 1 BiCGSTAB, 2 refinement, 3 refinement with a learned inner M (mvals), 4 CGS, 5 GPBiCG
mp_status solve_entry(const char *name, int kind, const mp_csr *A, const double *a, const double *mvals,
                      const double *b, double *x, const mp_solve_opts *opts, const mp_plan *plan, void *ws,
                      size_t ws_bytes, mp_solve_info *info, void *stream)
{
    clear_error();
    const bool refine = kind == 2 || kind == 3;
    if (refine && opts && opts->inner != MP_INNER_FP64 && opts->inner != MP_INNER_FP32)
        return fail(MP_ERR_INVALID_ARG, "%s: unknown inner precision %d", name, opts->inner);
    const size_t need = refine ? solver_bytes(A, opts) : (A ? workspace_bytes(A->n_rows) : 0);
    mp_status st = check_solver_args(name, A, a, b, x, opts, plan, ws, ws_bytes, need, info, kind == 3);
    if (st != MP_OK) return st;
    if (kind == 3) {
        if (A->nnz > 0 && !mvals) return fail(MP_ERR_INVALID_ARG, "%s: m_values is NULL", name);
        const size_t vb = sizeof(double) * 2 * (size_t)A->n_rows, mb = sizeof(double) * (size_t)A->nnz;
        if (overlaps(x, vb, mvals, mb) || overlaps(ws, ws_bytes, mvals, mb))
            return fail(MP_ERR_ALIAS, "%s: m_values overlaps x or the workspace", name);
    }
    if (A->n_rows == 0) {
        std::memset(info, 0, sizeof(*info));
        return MP_OK;
    }
    Solver S;
    S.A = A;
    S.a = a;
    S.plan = plan;
    S.s = static_cast<hipStream_t>(stream);
    S.n = A->n_rows;
    S.m = (int)((S.n + kDotChunk - 1) / kDotChunk);
    const int64_t vb = (S.n + 255) / 256;
    S.vblocks = (unsigned)(vb < 8192 ? vb : 8192);
    S.w = carve(ws, S.n);
    if (kind == 0) return run_cg(S, b, x, opts, info);
    if (kind == 1) return run_bicgstab(S, b, x, opts, info);
    if (kind == 4) return run_cgs(S, b, x, opts, info);
    if (kind == 5) return run_gpbicg(S, b, x, opts, info);
    const double *mv = kind == 3 ? mvals : nullptr;
    return opts->inner == MP_INNER_FP32 ? run_ir_t<float>(S, b, x, mv, opts, info)
                                        : run_ir_t<double>(S, b, x, mv, opts, info);
}

}  // namespace mpk

extern "C" {

mp_status mpvec_dd_sub(int64_t n, const double *x, const double *y, double *z, void *stream)
{
    mpk::clear_error();
    if (n < 0) return mpk::fail(MP_ERR_INVALID_ARG, "mpvec_dd_sub: n < 0");
    if (n == 0) return MP_OK;
    if (!x || !y || !z) return mpk::fail(MP_ERR_INVALID_ARG, "mpvec_dd_sub: NULL vector");
    const size_t vb = sizeof(double) * 2 * (size_t)n;
    if ((z != x && mpk::overlaps(z, vb, x, vb)) || (z != y && mpk::overlaps(z, vb, y, vb)))
        return mpk::fail(MP_ERR_ALIAS, "mpvec_dd_sub: z overlaps x or y without being equal to it");
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(mpk::k_residual, dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n, x, y, z);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

mp_status mpkrylov_workspace_bytes(const mp_csr *A, const mp_solve_opts *opts, size_t *bytes)
{
    mpk::clear_error();
    mp_status st = mpk::check_csr(A);
    if (st != MP_OK) return st;
    if (!bytes) return mpk::fail(MP_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = mpk::solver_bytes(A, opts);
    return MP_OK;
}

mp_status mpkrylov_cg(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                      const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_cg", 0, A, a, nullptr, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_bicgstab(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                            const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_bicgstab", 1, A, a, nullptr, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_cgs(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                       const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_cgs", 4, A, a, nullptr, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_gpbicg(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                          const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_gpbicg", 5, A, a, nullptr, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_ir(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                      const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_ir", 2, A, a, nullptr, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_bicg(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                        double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                        size_t ws_bytes, mp_solve_info *info, void *stream)
{
    using namespace mpk;
    clear_error();
    const size_t need = A ? workspace_bytes(A->n_rows) : 0;
    mp_status st = check_solver_args("mpkrylov_bicg", A, a, b, x, opts, plan, ws, ws_bytes, need, info, false);
    if (st != MP_OK) return st;
    if ((st = check_csr(At)) != MP_OK) return st;
    if (At->n_rows != A->n_cols || At->n_cols != A->n_rows || At->nnz != A->nnz)
        return fail(MP_ERR_INVALID_ARG, "mpkrylov_bicg: At is not the transpose's shape");
    if (At->nnz > 0 && !at) return fail(MP_ERR_INVALID_ARG, "mpkrylov_bicg: at is NULL");
    if (plan_t && (plan_t->ncomp != 2 || plan_t->cplx || plan_t->n_rows != At->n_rows || plan_t->nnz != At->nnz))
        return fail(MP_ERR_INVALID_ARG, "mpkrylov_bicg: plan_t is not a DD real plan of At");
    const size_t vb = sizeof(double) * 2 * (size_t)A->n_rows;
    if (overlaps(x, vb, at, sizeof(double) * 2 * (size_t)At->nnz))
        return fail(MP_ERR_ALIAS, "mpkrylov_bicg: x overlaps at");
    if (A->n_rows == 0) {
        std::memset(info, 0, sizeof(*info));
        return MP_OK;
    }
    Solver S;
    S.A = A;
    S.a = a;
    S.plan = plan;
    S.s = static_cast<hipStream_t>(stream);
    S.n = A->n_rows;
    S.m = (int)((S.n + kDotChunk - 1) / kDotChunk);
    const int64_t vblk = (S.n + 255) / 256;
    S.vblocks = (unsigned)(vblk < 8192 ? vblk : 8192);
    S.w = carve(ws, S.n);
    return run_bicg(S, At, at, plan_t, b, x, opts, info);
}

mp_status mpkrylov_ir_learned(const mp_csr *A, const double *a, const double *m_values, const double *b, double *x,
                              const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                              mp_solve_info *info, void *stream)
{
    return mpk::solve_entry("mpkrylov_ir_learned", 3, A, a, m_values, b, x, opts, plan, ws, ws_bytes, info, stream);
}

}  // extern "C"
