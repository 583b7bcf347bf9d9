// krylov_mp.hip -- CG and BiCGSTAB in triple-double and quad-double (Sec. 4.2 runs
// the Krylov methods in DD, TD and QD on top of the multi-component SpMV).
//
// The steps, stopping rule, confirmation and restarts are those of the DD solvers
// (krylov.hip) with K-component operations: additions, products and products with a
// binary64 (TD = the QD operation on zero-padded values, three components kept),
// a K-component division (long division: q0 = a0/b0, three times r = r - b*q_i and
// q_{i+1} = r0/b0, then the renormalisation of q0..q3), a lexicographic comparison for
// the stop tests, and the dot product tree of the DD solvers (chunks of 4096, 256
// strided lanes, halving fold, pairwise tree over the chunk sums).  The kernels are
// plain (one vector operation per launch): at these precisions the arithmetic, not the
// launch sequence, dominates a step.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "mp_arith.hpp"
#include "plan.hpp"

namespace mpk {
namespace kmp {

constexpr int kLanes = 256;
constexpr int kChunk = 4096;
constexpr int kMaxChunks = 1024;   // n <= 4,194,304 (the chunk sums of a QD dot fit 32 KiB of LDS)
// chunk workgroups: kGroups groups of kLanes lanes, kPerThread elements of a lane each
constexpr int kGroups = 4;
constexpr int kPerThread = kChunk / kLanes / kGroups;
constexpr int kChunkThreads = kLanes * kGroups;

enum : int32_t { RUN = 0, RECURRENCE_MET = 1, BROKE_DOWN = 2, ITER_LIMIT = 3, CONFIRMED = 4, RESTART = 5 };

template <int K>
struct State {
    mpn<K> rho, rho_old, rr, bb, tol2, pq, alpha, beta, omega, rv, ss, ts, tt, rr_true;
    int32_t done;
    int32_t iters;
    int32_t max_iter;
    int32_t fresh;
    int32_t half;
    int32_t restarts;
};

template <int K>
__device__ __forceinline__ mpn<K> ldk(const double *__restrict__ v, int64_t n, int64_t i)
{
    mpn<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) r.c[c] = v[c * n + i];
    return r;
}

template <int K>
__device__ __forceinline__ void stk(double *__restrict__ v, int64_t n, int64_t i, const mpn<K> &x)
{
#pragma unroll
    for (int c = 0; c < K; ++c) v[c * n + i] = x.c[c];
}

template <int K>
__device__ __forceinline__ mpn<K> k_sub(const mpn<K> &a, const mpn<K> &b)
{
    return mp_add(a, mp_neg(b));
}

template <int K>
__device__ __forceinline__ bool k_finite(const mpn<K> &a)
{
    return isfinite(a.c[0]);
}

// a <= b: the first component that differs decides; a comparison that is not an
// equality (greater, or a NaN) is false
template <int K>
__device__ __forceinline__ bool k_le(const mpn<K> &a, const mpn<K> &b)
{
#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (a.c[c] < b.c[c]) return true;
        if (!(a.c[c] == b.c[c])) return false;
    }
    return true;
}

// a / b by long division (TD: the QD division of the zero-padded values, three
// components kept)
template <int K>
__device__ __forceinline__ mpn<K> k_div(const mpn<K> &a, const mpn<K> &b)
{
    double q[4];
    mpn<K> r = a;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        q[i] = r.c[0] / b.c[0];
        if (i < 3) r = mp_add(r, mp_neg(mp_mul_d(b, q[i])));
    }
    const qd_t o = renorm5(q[0], q[1], q[2], q[3], 0.0);
    mpn<K> out;
#pragma unroll
    for (int c = 0; c < K; ++c) out.c[c] = o.c[c];
    return out;
}

template <int K>
__device__ __forceinline__ mpn<K> k_one()
{
    mpn<K> r = mp_zero<K>();
    r.c[0] = 1.0;
    return r;
}

// pairwise tree over m chunk sums (all threads of the workgroup take part)
template <int K>
__device__ __forceinline__ mpn<K> pair_tree(const mpn<K> *__restrict__ part, int m, mpn<K> *P)
{
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < m; i += nt) P[i] = part[i];
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        for (int i = t; (int64_t)i * 2 * s + s < m; i += nt) P[i * 2 * s] = mp_add(P[i * 2 * s], P[i * 2 * s + s]);
        __syncthreads();
    }
    const mpn<K> r = m > 0 ? P[0] : mp_zero<K>();
    __syncthreads();
    return r;
}

// the pairwise trees of two sets of m chunk sums, level by level together (the same
// additions as two pair_tree calls, with half the dependent levels); falls back to two
// passes when both sets do not fit P
template <int K>
__device__ __forceinline__ void pair_tree2(const mpn<K> *__restrict__ a, const mpn<K> *__restrict__ b, int m,
                                           mpn<K> *P, mpn<K> &ra, mpn<K> &rb)
{
    if (2 * m > kMaxChunks) {
        ra = pair_tree(a, m, P);
        rb = pair_tree(b, m, P);
        return;
    }
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < m; i += nt) {
        P[i] = a[i];
        P[m + i] = b[i];
    }
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        const int cnt = (m - s + 2 * s - 1) / (2 * s);   // pairs per set at this level
        for (int i = t; i < 2 * cnt; i += nt) {
            const int base = i < cnt ? 0 : m;
            const int j = (i < cnt ? i : i - cnt) * 2 * s;
            P[base + j] = mp_add(P[base + j], P[base + j + s]);
        }
        __syncthreads();
    }
    ra = m > 0 ? P[0] : mp_zero<K>();
    rb = m > 0 ? P[m] : mp_zero<K>();
    __syncthreads();
}

__device__ __forceinline__ int chunk_used(int64_t n, int c)
{
    const int64_t left = n - (int64_t)c * kChunk;
    return left < kLanes ? (int)left : kLanes;
}

// Chunk workgroups of kChunkThreads threads: thread (g, t) = (tid / 256, tid % 256)
// holds elements j = g*kPerThread .. g*kPerThread + kPerThread - 1 of lane t (element
// c*4096 + t + 256 j).  Their loads and products run in parallel; each lane's sum is
// then carried from group to group through LDS, so the lane still adds its products
// one at a time in j order, starting from its first product -- the order of a single
// 256-lane pass over the chunk.

// valid elements of this thread in chunk c (a prefix of its kPerThread elements)
__device__ __forceinline__ int thread_valid(int64_t n, int c)
{
    const int g = threadIdx.x / kLanes, t = threadIdx.x % kLanes;
    const int64_t first = (int64_t)c * kChunk + t + (int64_t)g * kPerThread * kLanes;
    if (first >= n) return 0;
    const int64_t left = (n - 1 - first) / kLanes + 1;
    return left < kPerThread ? (int)left : kPerThread;
}

__device__ __forceinline__ int64_t thread_elem(int c, int jj)
{
    const int g = threadIdx.x / kLanes, t = threadIdx.x % kLanes;
    return (int64_t)c * kChunk + t + (int64_t)(g * kPerThread + jj) * kLanes;
}

// prod[q][jj]: product jj of sum q of this thread (valid for jj < nvalid); leaves lane
// t's sum q in chain[q][t] for the lanes that hold at least one element
template <int K, int NS>
__device__ __forceinline__ void lane_chain(const mpn<K> (&prod)[NS][kPerThread], int nvalid, mpn<K> (*chain)[kLanes])
{
    const int g = threadIdx.x / kLanes, t = threadIdx.x % kLanes;
    for (int st = 0; st < kGroups; ++st) {
        if (g == st && nvalid > 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                mpn<K> a = st == 0 ? prod[q][0] : mp_add(chain[q][t], prod[q][0]);
#pragma unroll
                for (int jj = 1; jj < kPerThread; ++jj)
                    if (jj < nvalid) a = mp_add(a, prod[q][jj]);
                chain[q][t] = a;
            }
        }
        __syncthreads();
    }
}

// fold of the lane sums left by lane_chain: lds[l] += lds[l + off] for off = 128..1
// where lane l + off holds a value; returns lds[0] to every thread
template <int K>
__device__ __forceinline__ mpn<K> chain_fold(mpn<K> *lds, int used)
{
    const int t = threadIdx.x;
    for (int off = kLanes / 2; off >= 1; off >>= 1) {
        if (t < off && t + off < used) lds[t] = mp_add(lds[t], lds[t + off]);
        __syncthreads();
    }
    const mpn<K> r = lds[0];
    __syncthreads();
    return r;
}

// chunk sums of (x1, y1) and optionally (x2, y2): lane l of chunk c adds the products of
// elements c*4096 + l + 256 j in j order, starting from its first product
template <int K>
__global__ __launch_bounds__(kChunkThreads) void k_dot2(int64_t n, const double *__restrict__ x1,
                                                        const double *__restrict__ y1, const double *__restrict__ x2,
                                                        const double *__restrict__ y2, mpn<K> *__restrict__ p1,
                                                        mpn<K> *__restrict__ p2, const State<K> *__restrict__ st)
{
    __shared__ mpn<K> chain[2][kLanes];
    if (st && st->done != RUN) return;
    const int c = blockIdx.x;
    const int nv = thread_valid(n, c);
    const int used = chunk_used(n, c);
    if (x2) {
        mpn<K> pr[2][kPerThread];
#pragma unroll
        for (int jj = 0; jj < kPerThread; ++jj) {
            if (jj < nv) {
                const int64_t k = thread_elem(c, jj);
                pr[0][jj] = mp_mul(ldk<K>(x1, n, k), ldk<K>(y1, n, k));
                pr[1][jj] = mp_mul(ldk<K>(x2, n, k), ldk<K>(y2, n, k));
            }
        }
        lane_chain<K, 2>(pr, nv, chain);
        const mpn<K> s1 = chain_fold(chain[0], used);
        const mpn<K> s2 = chain_fold(chain[1], used);
        if (threadIdx.x == 0) {
            p1[c] = s1;
            p2[c] = s2;
        }
    } else {
        mpn<K> pr[1][kPerThread];
#pragma unroll
        for (int jj = 0; jj < kPerThread; ++jj) {
            if (jj < nv) {
                const int64_t k = thread_elem(c, jj);
                pr[0][jj] = mp_mul(ldk<K>(x1, n, k), ldk<K>(y1, n, k));
            }
        }
        lane_chain<K, 1>(pr, nv, chain);
        const mpn<K> s1 = chain_fold(chain[0], used);
        if (threadIdx.x == 0) p1[c] = s1;
    }
}

#define KMP_FOR(i, n) for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (n); i += (int64_t)gridDim.x * 256)

// r = b - q
template <int K>
__global__ __launch_bounds__(256) void k_residual(int64_t n, const double *__restrict__ b, const double *__restrict__ q,
                                                  double *__restrict__ r)
{
    KMP_FOR(i, n) stk<K>(r, n, i, k_sub(ldk<K>(b, n, i), ldk<K>(q, n, i)));
}

// z = M^-1 r (Jacobi: K components times the binary64 inverse diagonal) or a copy
template <int K>
__global__ __launch_bounds__(256) void k_precond(int64_t n, const double *__restrict__ minv, const double *__restrict__ r,
                                                 double *__restrict__ z, const State<K> *__restrict__ st)
{
    if (st && st->done != RUN) return;
    KMP_FOR(i, n) stk<K>(z, n, i, minv ? mp_mul_d(ldk<K>(r, n, i), minv[i]) : ldk<K>(r, n, i));
}

__global__ __launch_bounds__(256) void k_copy(int64_t len, const double *__restrict__ src, double *__restrict__ dst)
{
    KMP_FOR(i, len) dst[i] = src[i];
}

// Jacobi inverse diagonal fl(1 / leading component of a_ii); 1 without a diagonal entry
__global__ __launch_bounds__(256) void k_jacobi_minv(int64_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const double *__restrict__ a_hi,
                                                     double *__restrict__ minv)
{
    KMP_FOR(i, n)
    {
        double m = 1.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) m = 1.0 / a_hi[k];
        minv[i] = m;
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_confirm(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    const mpn<K> rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rr_true = rr;
        if (k_le(rr, st->tol2)) {
            st->done = CONFIRMED;
        } else {
            st->rr = rr;
            st->restarts += 1;
            st->done = RESTART;
        }
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_exit_rr(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    const mpn<K> rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) st->rr_true = rr;
}

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(256) void k_cg_init(const mpn<K> *__restrict__ pbb, const mpn<K> *__restrict__ prz,
                                                 const mpn<K> *__restrict__ prr, int m, double rtol2, int32_t max_iter,
                                                 State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    const mpn<K> bb = pair_tree(pbb, m, P);
    const mpn<K> rz = pair_tree(prz, m, P);
    const mpn<K> rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->tol2 = mp_mul_d(bb, rtol2);
        st->rho = rz;
        st->rr = rr;
        st->iters = 0;
        st->max_iter = max_iter;
        st->restarts = 0;
        st->done = k_le(rr, st->tol2) ? RECURRENCE_MET : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_cg_restart(const mpn<K> *__restrict__ prz, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    const mpn<K> rz = pair_tree(prz, m, P);
    if (threadIdx.x == 0) {
        st->rho = rz;
        st->done = st->iters >= st->max_iter ? ITER_LIMIT : RUN;
    }
}

// One CG step after q = A p and the chunk sums of (p, q) is two kernels:
//   k_cg_update: alpha = rho / (p, q) (breakdown unless (p, q) > 0 and finite), then
//                r -= alpha q; z = M^-1 r; chunk sums of (r, z), (r, r)
//                (one workgroup per chunk, lane l over the chunk's elements l + 256 j
//                in j order, as k_dot2)
//   k_cg_pstep:  x += alpha p when the update kernel ran to the end (on the whole grid
//                rather than the chunk workgroups); rho_new = (r, z), rr = (r, r); one
//                step counted; breakdown when not
//                finite; beta = rho_new / rho; stop tests; p = z + beta p unless the
//                step broke down
// Every workgroup reduces the chunk sums itself (the same tree, so the same values),
// so no scalar kernel runs between them.  The state is double-buffered across the
// p kernel: it reads `sr` and its first workgroup writes the next state to `sw`, so
// no workgroup reads a field that another workgroup of the same kernel writes.
template <int K>
__global__ __launch_bounds__(kChunkThreads) void k_cg_update(int64_t n, double *__restrict__ r,
                                                             double *__restrict__ z, const double *__restrict__ q,
                                                             const double *__restrict__ minv,
                                                             const mpn<K> *__restrict__ ppq, int m,
                                                             mpn<K> *__restrict__ prz, mpn<K> *__restrict__ prr,
                                                             State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    __shared__ mpn<K> chain[2][kLanes];
    __shared__ mpn<K> s_rho;
    __shared__ int32_t s_done;
    if (threadIdx.x == 0) {
        s_done = st->done;
        s_rho = st->rho;
    }
    __syncthreads();
    if (s_done != RUN) return;   // uniform in the workgroup
    const mpn<K> pq = pair_tree(ppq, m, P);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(pq.c[0] > 0.0) || !k_finite(pq)) {
        if (lead) {
            st->pq = pq;
            st->done = BROKE_DOWN;
        }
        return;
    }
    // thread 0 alone performs the K-component division
    __shared__ mpn<K> s_alpha;
    if (threadIdx.x == 0) s_alpha = k_div(s_rho, pq);
    __syncthreads();
    const mpn<K> alpha = s_alpha;
    if (lead) {
        st->pq = pq;
        st->alpha = alpha;
    }
    const int c = blockIdx.x;
    const int nv = thread_valid(n, c);
    mpn<K> pr[2][kPerThread];
#pragma unroll
    for (int jj = 0; jj < kPerThread; ++jj) {
        if (jj < nv) {
            const int64_t k = thread_elem(c, jj);
            const mpn<K> rk = k_sub(ldk<K>(r, n, k), mp_mul(alpha, ldk<K>(q, n, k)));
            stk<K>(r, n, k, rk);
            const mpn<K> zk = minv ? mp_mul_d(rk, minv[k]) : rk;
            stk<K>(z, n, k, zk);
            pr[0][jj] = mp_mul(rk, zk);
            pr[1][jj] = mp_mul(rk, rk);
        }
    }
    lane_chain<K, 2>(pr, nv, chain);
    const int used = chunk_used(n, c);
    const mpn<K> s1 = chain_fold(chain[0], used);
    const mpn<K> s2 = chain_fold(chain[1], used);
    if (threadIdx.x == 0) {
        prz[c] = s1;
        prr[c] = s2;
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_cg_pstep(int64_t n, double *__restrict__ x, const double *__restrict__ z,
                                                  double *__restrict__ p, const mpn<K> *__restrict__ prz,
                                                  const mpn<K> *__restrict__ prr, int m,
                                                  const State<K> *__restrict__ sr, State<K> *__restrict__ sw)
{
    __shared__ mpn<K> P[kMaxChunks];
    __shared__ mpn<K> s_rho, s_tol2, s_alpha;
    __shared__ int32_t s_done, s_iters, s_max;
    if (threadIdx.x == 0) {
        s_done = sr->done;
        s_rho = sr->rho;
        s_tol2 = sr->tol2;
        s_alpha = sr->alpha;
        s_iters = sr->iters;
        s_max = sr->max_iter;
    }
    __syncthreads();
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (s_done != RUN) {
        if (lead) *sw = *sr;
        return;
    }
    // the update kernel ran to the end with this alpha: x += alpha p (old p)
    KMP_FOR(i, n) stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), mp_mul(s_alpha, ldk<K>(p, n, i))));
    mpn<K> rz, rr;
    pair_tree2(prz, prr, m, P, rz, rr);
    const int32_t iters = s_iters + 1;
    // thread 0 forms beta (one K-component division per workgroup) and the stop decision
    __shared__ mpn<K> s_beta;
    __shared__ int32_t s_next;
    if (threadIdx.x == 0) {
        int32_t d = RUN;
        mpn<K> bt = mp_zero<K>();
        if (!k_finite(rr) || !k_finite(rz)) {
            d = BROKE_DOWN;
        } else {
            bt = k_div(rz, s_rho);
            if (k_le(rr, s_tol2))
                d = RECURRENCE_MET;
            else if (iters >= s_max)
                d = ITER_LIMIT;
        }
        s_beta = bt;
        s_next = d;
    }
    __syncthreads();
    const int32_t done = s_next;
    const mpn<K> beta = s_beta;
    if (lead) {
        *sw = *sr;
        sw->iters = iters;
        sw->rr = rr;
        if (done != BROKE_DOWN) {
            sw->beta = beta;
            sw->rho = rz;
        }
        sw->done = done;
    }
    if (done == BROKE_DOWN) return;
    KMP_FOR(i, n) stk<K>(p, n, i, mp_add(ldk<K>(z, n, i), mp_mul(beta, ldk<K>(p, n, i))));
}

// ---------------------------------------------------------------------------
// BiCGSTAB (right Jacobi preconditioning, shadow r0)
// ---------------------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(256) void k_bi_init(const mpn<K> *__restrict__ pbb, const mpn<K> *__restrict__ prr, int m,
                                                 double rtol2, int32_t max_iter, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    const mpn<K> bb = pair_tree(pbb, m, P);
    const mpn<K> rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->tol2 = mp_mul_d(bb, rtol2);
        st->rr = rr;
        st->rho_old = k_one<K>();
        st->alpha = k_one<K>();
        st->omega = k_one<K>();
        st->iters = 0;
        st->max_iter = max_iter;
        st->restarts = 0;
        st->fresh = 1;
        st->half = 0;
        st->done = k_le(rr, st->tol2) ? RECURRENCE_MET : (max_iter <= 0 ? ITER_LIMIT : RUN);
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_bi_restart(State<K> *__restrict__ st)
{
    if (threadIdx.x == 0) {
        st->fresh = 1;
        st->done = st->iters >= st->max_iter ? ITER_LIMIT : RUN;
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_bi_rho(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rho = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rho = rho;
        if (rho.c[0] == 0.0 || !k_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        if (!st->fresh) st->beta = mp_mul(k_div(rho, st->rho_old), k_div(st->alpha, st->omega));
    }
}

// p = r (fresh) or p = r + beta (p - omega v); ph = M^-1 p
template <int K>
__global__ __launch_bounds__(256) void k_bi_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                              const double *__restrict__ v, double *__restrict__ ph,
                                              const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> beta = st->beta, omega = st->omega;
    KMP_FOR(i, n)
    {
        mpn<K> pi;
        if (fresh) {
            pi = ldk<K>(r, n, i);
        } else {
            const mpn<K> pv = k_sub(ldk<K>(p, n, i), mp_mul(omega, ldk<K>(v, n, i)));
            pi = mp_add(ldk<K>(r, n, i), mp_mul(beta, pv));
        }
        stk<K>(p, n, i, pi);
        stk<K>(ph, n, i, minv ? mp_mul_d(pi, minv[i]) : pi);
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_bi_alpha(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rv = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->fresh = 0;
        st->rv = rv;
        if (rv.c[0] == 0.0 || !k_finite(rv)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->alpha = k_div(st->rho, rv);
    }
}

// s = r - alpha v
template <int K>
__global__ __launch_bounds__(256) void k_bi_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                              double *__restrict__ s, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> alpha = st->alpha;
    KMP_FOR(i, n) stk<K>(s, n, i, k_sub(ldk<K>(r, n, i), mp_mul(alpha, ldk<K>(v, n, i))));
}

// ss = (s, s); one step counted; half-step test
template <int K>
__global__ __launch_bounds__(256) void k_bi_ss(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> ss = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->ss = ss;
        st->iters += 1;
        st->half = k_le(ss, st->tol2) ? 1 : 0;
    }
}

// half step met the tolerance: x += alpha ph; r = s
template <int K>
__global__ __launch_bounds__(256) void k_bi_half(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ ph, const double *__restrict__ s,
                                                 const State<K> *__restrict__ st)
{
    if (st->done != RUN || !st->half) return;
    const mpn<K> alpha = st->alpha;
    KMP_FOR(i, n)
    {
        stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), mp_mul(alpha, ldk<K>(ph, n, i))));
        stk<K>(r, n, i, ldk<K>(s, n, i));
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_bi_half_final(State<K> *__restrict__ st)
{
    if (threadIdx.x != 0 || st->done != RUN || !st->half) return;
    st->rr = st->ss;
    st->rho_old = st->rho;
    st->omega = k_one<K>();
    st->fresh = 1;
    st->half = 0;
    st->done = RECURRENCE_MET;
}

// omega = (t, s) / (t, t)
template <int K>
__global__ __launch_bounds__(256) void k_bi_omega(const mpn<K> *__restrict__ pts, const mpn<K> *__restrict__ ptt, int m,
                                                  State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> ts = pair_tree(pts, m, P);
    const mpn<K> tt = pair_tree(ptt, m, P);
    if (threadIdx.x == 0) {
        st->ts = ts;
        st->tt = tt;
        if (tt.c[0] == 0.0 || !k_finite(tt)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->omega = k_div(ts, tt);
    }
}

// x = (x + alpha ph) + omega sh; r = s - omega t
template <int K>
__global__ __launch_bounds__(256) void k_bi_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                               const double *__restrict__ ph, const double *__restrict__ sh,
                                               const double *__restrict__ s, const double *__restrict__ tv,
                                               const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> alpha = st->alpha, omega = st->omega;
    KMP_FOR(i, n)
    {
        const mpn<K> xv = mp_add(ldk<K>(x, n, i), mp_mul(alpha, ldk<K>(ph, n, i)));
        stk<K>(x, n, i, mp_add(xv, mp_mul(omega, ldk<K>(sh, n, i))));
        stk<K>(r, n, i, k_sub(ldk<K>(s, n, i), mp_mul(omega, ldk<K>(tv, n, i))));
    }
}

// rr = (r, r); breakdown when not finite or omega = 0; stop tests
template <int K>
__global__ __launch_bounds__(256) void k_bi_rr(const mpn<K> *__restrict__ part, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rr = pair_tree(part, m, P);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (!k_finite(rr) || st->omega.c[0] == 0.0) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        if (k_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// ---------------------------------------------------------------------------
// BiCG (A^T explicit; the shadow system preconditioned by the same Jacobi M)
// ---------------------------------------------------------------------------

// sigma = (p~, q): breakdown when 0 or not finite; alpha = rho / sigma
template <int K>
__global__ __launch_bounds__(256) void k_bicg_alpha(const mpn<K> *__restrict__ ppq, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> pq = pair_tree(ppq, m, P);
    if (threadIdx.x == 0) {
        st->pq = pq;
        if (pq.c[0] == 0.0 || !k_finite(pq))
            st->done = BROKE_DOWN;
        else
            st->alpha = k_div(st->rho, pq);
    }
}

// x += alpha p; r -= alpha q; r~ -= alpha q~; z = M^-1 r; z~ = M^-1 r~
template <int K>
__global__ __launch_bounds__(256) void k_bicg_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ z, const double *__restrict__ p,
                                                     const double *__restrict__ q, double *__restrict__ rt,
                                                     double *__restrict__ zt, const double *__restrict__ qt,
                                                     const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), mp_mul(alpha, ldk<K>(p, n, i))));
        const mpn<K> ri = k_sub(ldk<K>(r, n, i), mp_mul(alpha, ldk<K>(q, n, i)));
        const mpn<K> rti = k_sub(ldk<K>(rt, n, i), mp_mul(alpha, ldk<K>(qt, n, i)));
        stk<K>(r, n, i, ri);
        stk<K>(rt, n, i, rti);
        stk<K>(z, n, i, minv ? mp_mul_d(ri, minv[i]) : ri);
        stk<K>(zt, n, i, minv ? mp_mul_d(rti, minv[i]) : rti);
    }
}

// rho' = (r~, z), rr = (r, r): one step counted; breakdown when not finite or when
// rho' = 0 short of the tolerance; beta = rho' / rho; stop tests
template <int K>
__global__ __launch_bounds__(256) void k_bicg_beta(const mpn<K> *__restrict__ prz, const mpn<K> *__restrict__ prr,
                                                   int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rz = pair_tree(prz, m, P);
    const mpn<K> rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = rr;
        if (!k_finite(rr) || !k_finite(rz) || (rz.c[0] == 0.0 && !k_le(rr, st->tol2))) {
            st->done = BROKE_DOWN;
            return;
        }
        st->beta = k_div(rz, st->rho);
        st->rho = rz;
        if (k_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// p = z + beta p; p~ = z~ + beta p~
template <int K>
__global__ __launch_bounds__(256) void k_bicg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                                const double *__restrict__ zt, double *__restrict__ pt,
                                                const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        stk<K>(p, n, i, mp_add(ldk<K>(z, n, i), mp_mul(beta, ldk<K>(p, n, i))));
        stk<K>(pt, n, i, mp_add(ldk<K>(zt, n, i), mp_mul(beta, ldk<K>(pt, n, i))));
    }
}

// ---------------------------------------------------------------------------
// CGS (right Jacobi preconditioning)
// ---------------------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(256) void k_cgs_rho(const mpn<K> *__restrict__ prho, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rho = pair_tree(prho, m, P);
    if (threadIdx.x == 0) {
        if (rho.c[0] == 0.0 || !k_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho = rho;
        if (!st->fresh) st->beta = k_div(rho, st->rho_old);
    }
}

// fresh: u = p = r; else u = r + beta q, p = u + beta (q + beta p); p^ = M^-1 p
template <int K>
__global__ __launch_bounds__(256) void k_cgs_up(int64_t n, const double *__restrict__ r, const double *__restrict__ q,
                                                double *__restrict__ u, double *__restrict__ p,
                                                double *__restrict__ ph, const double *__restrict__ minv,
                                                const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> ri = ldk<K>(r, n, i);
        mpn<K> pi;
        if (fresh) {
            stk<K>(u, n, i, ri);
            pi = ri;
        } else {
            const mpn<K> qi = ldk<K>(q, n, i);
            const mpn<K> ui = mp_add(ri, mp_mul(beta, qi));
            const mpn<K> w = mp_add(qi, mp_mul(beta, ldk<K>(p, n, i)));
            stk<K>(u, n, i, ui);
            pi = mp_add(ui, mp_mul(beta, w));
        }
        stk<K>(p, n, i, pi);
        stk<K>(ph, n, i, minv ? mp_mul_d(pi, minv[i]) : pi);
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_cgs_alpha(const mpn<K> *__restrict__ psig, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> sigma = pair_tree(psig, m, P);
    if (threadIdx.x == 0) {
        st->fresh = 0;
        st->pq = sigma;
        if (sigma.c[0] == 0.0 || !k_finite(sigma))
            st->done = BROKE_DOWN;
        else
            st->alpha = k_div(st->rho, sigma);
    }
}

// q = u - alpha v; u^ = M^-1 (u + q); x += alpha u^
template <int K>
__global__ __launch_bounds__(256) void k_cgs_q(int64_t n, const double *__restrict__ u, const double *__restrict__ v,
                                               double *__restrict__ q, double *__restrict__ uh, double *__restrict__ x,
                                               const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> ui = ldk<K>(u, n, i);
        const mpn<K> qi = k_sub(ui, mp_mul(alpha, ldk<K>(v, n, i)));
        const mpn<K> sm = mp_add(ui, qi);
        const mpn<K> uhi = minv ? mp_mul_d(sm, minv[i]) : sm;
        stk<K>(q, n, i, qi);
        stk<K>(uh, n, i, uhi);
        stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), mp_mul(alpha, uhi)));
    }
}

// r -= alpha t
template <int K>
__global__ __launch_bounds__(256) void k_cgs_r(int64_t n, double *__restrict__ r, const double *__restrict__ t,
                                               const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const mpn<K> alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        stk<K>(r, n, i, k_sub(ldk<K>(r, n, i), mp_mul(alpha, ldk<K>(t, n, i))));
}

// rr = (r, r): one step counted; breakdown when not finite; stop tests
template <int K>
__global__ __launch_bounds__(256) void k_cgs_rr(const mpn<K> *__restrict__ prr, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->rr = rr;
        if (!k_finite(rr)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        if (k_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

// ---------------------------------------------------------------------------
// GPBiCG (right Jacobi preconditioning)
// ---------------------------------------------------------------------------

template <int K>
__global__ __launch_bounds__(256) void k_gp_rho(const mpn<K> *__restrict__ prho, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rho = pair_tree(prho, m, P);
    if (threadIdx.x == 0) {
        if (rho.c[0] == 0.0 || !k_finite(rho)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho = rho;
        if (!st->fresh) st->beta = mp_mul(k_div(st->alpha, st->omega), k_div(rho, st->rho_old));
    }
}

// fresh: p = r; else p = r + beta (p - u), w = c + beta q; tmp = M p
template <int K>
__global__ __launch_bounds__(256) void k_gp_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                                              const double *__restrict__ u, const double *__restrict__ c,
                                              const double *__restrict__ q, double *__restrict__ w,
                                              double *__restrict__ tmp, const double *__restrict__ minv,
                                              const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> beta = st->beta;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> ri = ldk<K>(r, n, i);
        mpn<K> pi;
        if (fresh) {
            pi = ri;
        } else {
            pi = mp_add(ri, mp_mul(beta, k_sub(ldk<K>(p, n, i), ldk<K>(u, n, i))));
            stk<K>(w, n, i, mp_add(ldk<K>(c, n, i), mp_mul(beta, ldk<K>(q, n, i))));
        }
        stk<K>(p, n, i, pi);
        stk<K>(tmp, n, i, minv ? mp_mul_d(pi, minv[i]) : pi);
    }
}

// sigma = (r~, q): breakdown when 0 or not finite; alpha = rho / sigma (the step's
// first-step flag stays set until the step ends)
template <int K>
__global__ __launch_bounds__(256) void k_gp_alpha(const mpn<K> *__restrict__ psig, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> sigma = pair_tree(psig, m, P);
    if (threadIdx.x == 0) {
        st->pq = sigma;
        if (sigma.c[0] == 0.0 || !k_finite(sigma))
            st->done = BROKE_DOWN;
        else
            st->alpha = k_div(st->rho, sigma);
    }
}

// t = r - alpha q; later steps y = (t' - t) - alpha w; tmp = M t
template <int K>
__global__ __launch_bounds__(256) void k_gp_t(int64_t n, const double *__restrict__ r, const double *__restrict__ q,
                                              const double *__restrict__ tp, const double *__restrict__ w,
                                              double *__restrict__ t, double *__restrict__ y, double *__restrict__ tmp,
                                              const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> ti = k_sub(ldk<K>(r, n, i), mp_mul(alpha, ldk<K>(q, n, i)));
        stk<K>(t, n, i, ti);
        if (!fresh) stk<K>(y, n, i, k_sub(k_sub(ldk<K>(tp, n, i), ti), mp_mul(alpha, ldk<K>(w, n, i))));
        stk<K>(tmp, n, i, minv ? mp_mul_d(ti, minv[i]) : ti);
    }
}

// half step met the tolerance: x += M (alpha p); r = t
template <int K>
__global__ __launch_bounds__(256) void k_gp_half(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ p, const double *__restrict__ t,
                                                 const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN || !st->half) return;
    const mpn<K> alpha = st->alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> d = mp_mul(alpha, ldk<K>(p, n, i));
        stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), minv ? mp_mul_d(d, minv[i]) : d));
        stk<K>(r, n, i, ldk<K>(t, n, i));
    }
}

template <int K>
__global__ __launch_bounds__(64) void k_gp_half_final(State<K> *__restrict__ st)
{
    if (threadIdx.x != 0 || st->done != RUN || !st->half) return;
    st->rr = st->ss;
    st->rho_old = st->rho;
    st->fresh = 1;
    st->half = 0;
    st->done = RECURRENCE_MET;
}

// zeta (kept in omega) and eta (kept in ts): first step zeta = (c,t)/(c,c), eta = 0;
// later steps from d = (c,c)(y,y) - (y,c)^2
template <int K>
__global__ __launch_bounds__(256) void k_gp_zeta(const mpn<K> *__restrict__ pcc, const mpn<K> *__restrict__ pct,
                                                 const mpn<K> *__restrict__ pyy, const mpn<K> *__restrict__ pyc,
                                                 const mpn<K> *__restrict__ pyt, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> cc = pair_tree(pcc, m, P);
    const mpn<K> ct = pair_tree(pct, m, P);
    mpn<K> yy = mp_zero<K>(), yc = mp_zero<K>(), yt = mp_zero<K>();
    if (!fresh) {
        yy = pair_tree(pyy, m, P);
        yc = pair_tree(pyc, m, P);
        yt = pair_tree(pyt, m, P);
    }
    if (threadIdx.x == 0) {
        mpn<K> zeta, eta;
        if (fresh) {
            if (cc.c[0] == 0.0 || !k_finite(cc)) {
                st->done = BROKE_DOWN;
                return;
            }
            zeta = k_div(ct, cc);
            eta = mp_zero<K>();
        } else {
            const mpn<K> den = k_sub(mp_mul(cc, yy), mp_mul(yc, yc));
            if (den.c[0] == 0.0 || !k_finite(den)) {
                st->done = BROKE_DOWN;
                return;
            }
            zeta = k_div(k_sub(mp_mul(yy, ct), mp_mul(yt, yc)), den);
            eta = k_div(k_sub(mp_mul(cc, yt), mp_mul(yc, ct)), den);
        }
        if (zeta.c[0] == 0.0 || !k_finite(zeta) || !k_finite(eta)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->omega = zeta;
        st->ts = eta;
    }
}

// u, z, x, r and t' of a full step (see the header for the forms)
template <int K>
__global__ __launch_bounds__(256) void k_gp_update(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   const double *__restrict__ t, const double *__restrict__ cv,
                                                   const double *__restrict__ y, double *__restrict__ u,
                                                   double *__restrict__ z, double *__restrict__ tp,
                                                   const double *__restrict__ minv, const State<K> *__restrict__ st)
{
    if (st->done != RUN) return;
    const bool fresh = st->fresh != 0;
    const mpn<K> alpha = st->alpha, beta = st->beta, zeta = st->omega, eta = st->ts;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const mpn<K> ri = ldk<K>(r, n, i), ti = ldk<K>(t, n, i), qi = ldk<K>(q, n, i), ci = ldk<K>(cv, n, i);
        mpn<K> ui, zi, rn;
        if (fresh) {
            ui = mp_mul(zeta, qi);
            zi = k_sub(mp_mul(zeta, ri), mp_mul(alpha, ui));
            rn = k_sub(ti, mp_mul(zeta, ci));
        } else {
            const mpn<K> g = mp_add(k_sub(ldk<K>(tp, n, i), ri), mp_mul(beta, ldk<K>(u, n, i)));
            ui = mp_add(mp_mul(zeta, qi), mp_mul(eta, g));
            zi = k_sub(mp_add(mp_mul(zeta, ri), mp_mul(eta, ldk<K>(z, n, i))), mp_mul(alpha, ui));
            rn = k_sub(k_sub(ti, mp_mul(eta, ldk<K>(y, n, i))), mp_mul(zeta, ci));
        }
        stk<K>(u, n, i, ui);
        stk<K>(z, n, i, zi);
        const mpn<K> d = mp_add(mp_mul(alpha, ldk<K>(p, n, i)), zi);
        stk<K>(x, n, i, mp_add(ldk<K>(x, n, i), minv ? mp_mul_d(d, minv[i]) : d));
        stk<K>(r, n, i, rn);
        stk<K>(tp, n, i, ti);
    }
}

// rr = (r, r): breakdown when not finite; the next step is not fresh; stop tests
template <int K>
__global__ __launch_bounds__(256) void k_gp_rr(const mpn<K> *__restrict__ prr, int m, State<K> *__restrict__ st)
{
    __shared__ mpn<K> P[kMaxChunks];
    if (st->done != RUN) return;
    const mpn<K> rr = pair_tree(prr, m, P);
    if (threadIdx.x == 0) {
        st->rr = rr;
        if (!k_finite(rr)) {
            st->done = BROKE_DOWN;
            return;
        }
        st->rho_old = st->rho;
        st->fresh = 0;
        if (k_le(rr, st->tol2))
            st->done = RECURRENCE_MET;
        else if (st->iters >= st->max_iter)
            st->done = ITER_LIMIT;
    }
}

#undef KMP_FOR

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int kVecs = 12;   // K-component work vectors (GPBiCG uses all of them)
constexpr int kParts = 6;   // chunk-sum arrays

template <int K>
size_t ws_bytes(int64_t n)
{
    return 2 * al256(sizeof(State<K>)) + al256(sizeof(double) * (size_t)n) +
           kVecs * al256(sizeof(double) * K * (size_t)n) + kParts * al256(sizeof(mpn<K>) * kMaxChunks) +
           al256(sizeof(double) * K * (size_t)n);   // staged x of the planned SpMV
}

template <int K>
struct Solver {
    const mp_csr *A;
    const double *a;
    const mp_plan *plan;
    hipStream_t s;
    int64_t n;
    int m;
    unsigned vb;
    State<K> *st;
    State<K> *st2;   // second slot of the double-buffered CG state
    double *minv;
    double *v[kVecs];
    mpn<K> *part[kParts];
    double *xs;   // interleaved copy of x that the planned SpMV gathers from

    void carve(void *ws)
    {
        char *p = static_cast<char *>(ws);
        st = reinterpret_cast<State<K> *>(p);
        st2 = reinterpret_cast<State<K> *>(p + al256(sizeof(State<K>)));
        p += 2 * al256(sizeof(State<K>));
        minv = reinterpret_cast<double *>(p);
        p += al256(sizeof(double) * (size_t)n);
        for (int i = 0; i < kVecs; ++i) {
            v[i] = reinterpret_cast<double *>(p);
            p += al256(sizeof(double) * K * (size_t)n);
        }
        for (int i = 0; i < kParts; ++i) {
            part[i] = reinterpret_cast<mpn<K> *>(p);
            p += al256(sizeof(mpn<K>) * kMaxChunks);
        }
        xs = reinterpret_cast<double *>(p);
    }
    mp_status launched()
    {
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
    mp_status spmv(const double *x, double *y)
    {
        return spmv_dispatch(K, false, A, a, nullptr, x, nullptr, y, nullptr, plan, xs, s);
    }
    mp_status dot2(const double *x1, const double *y1, const double *x2, const double *y2, mpn<K> *p1, mpn<K> *p2,
                   const State<K> *guard)
    {
        hipLaunchKernelGGL(k_dot2<K>, dim3(m), dim3(kChunkThreads), 0, s, n, x1, y1, x2, y2, p1, p2, guard);
        return launched();
    }
    mp_status residual(const double *b, const double *x, double *q, double *r)
    {
        mp_status e = spmv(x, q);
        if (e != MP_OK) return e;
        hipLaunchKernelGGL(k_residual<K>, dim3(vb), dim3(256), 0, s, n, b, q, r);
        return launched();
    }
    mp_status read_state(State<K> *h)
    {
        MP_HIP_TRY(hipMemcpyAsync(h, st, sizeof(State<K>), hipMemcpyDeviceToHost, s));
        MP_HIP_TRY(hipStreamSynchronize(s));
        return MP_OK;
    }
    mp_status true_residual(const double *b, const double *x, double *q, double *r, bool confirm)
    {
        mp_status e = residual(b, x, q, r);
        if (e == MP_OK) e = dot2(r, r, nullptr, nullptr, part[0], nullptr, nullptr);
        if (e != MP_OK) return e;
        if (confirm)
            hipLaunchKernelGGL(k_confirm<K>, dim3(1), dim3(256), 0, s, part[0], m, st);
        else
            hipLaunchKernelGGL(k_exit_rr<K>, dim3(1), dim3(256), 0, s, part[0], m, st);
        return launched();
    }
    mp_status jacobi()
    {
        hipLaunchKernelGGL(k_jacobi_minv, dim3(vb), dim3(256), 0, s, n, A->row_ptr, A->col_idx, a, minv);
        return launched();
    }
};

template <int K>
void fill(const State<K> &h, int status, double secs, mp_solve_info *info)
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
}

template <int K>
int finish_status(const State<K> &h)
{
    return h.done == CONFIRMED ? MP_OK : (h.done == BROKE_DOWN ? MP_ERR_BREAKDOWN : MP_ERR_NOT_CONVERGED);
}

template <int K>
mp_status run_cg(Solver<K> &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info,
                 const char *name)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.v[0], *z = S.v[1], *p = S.v[2], *q = S.v[3];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int64_t len = (int64_t)K * n;
    mp_status st;
    State<K> h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.st, 0, sizeof(State<K>), S.s));
    if (minv && (st = S.jacobi()) != MP_OK) return st;
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_precond<K>, dim3(S.vb), dim3(256), 0, S.s, n, minv, r, z, nullptr);
    hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, z, p);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, z, S.part[0], S.part[1], nullptr)) != MP_OK) return st;
    if ((st = S.dot2(r, r, nullptr, nullptr, S.part[2], nullptr, nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cg_init<K>, dim3(1), dim3(256), 0, S.s, S.part[0], S.part[1], S.part[2], m, o->rtol * o->rtol,
                       o->max_iter, S.st);
    if ((st = S.launched()) != MP_OK) return st;
    // the step's state alternates between the two slots; a chunk of an even number of
    // steps ends with it in S.st, where the rest of the driver reads it
    State<K> *sb[2] = {S.st, S.st2};
    const int steps = (every + 1) & ~1;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < steps; ++it) {
                State<K> *sr = sb[it & 1], *sw = sb[(it + 1) & 1];
                if ((st = S.spmv(p, q)) != MP_OK) return st;
                if ((st = S.dot2(p, q, nullptr, nullptr, S.part[0], nullptr, sr)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cg_update<K>, dim3(m), dim3(kChunkThreads), 0, S.s, n, r, z, q, minv, S.part[0],
                                   m, S.part[1], S.part[2], sr);
                hipLaunchKernelGGL(k_cg_pstep<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, z, p, S.part[1], S.part[2], m,
                                   sr, sw);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, q, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_precond<K>, dim3(S.vb), dim3(256), 0, S.s, n, minv, r, z, nullptr);
            hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, z, p);
            if ((st = S.launched()) != MP_OK) return st;
            if ((st = S.dot2(r, z, nullptr, nullptr, S.part[1], nullptr, nullptr)) != MP_OK) return st;
            hipLaunchKernelGGL(k_cg_restart<K>, dim3(1), dim3(256), 0, S.s, S.part[1], m, S.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        break;
    }
    const int status = finish_status(h);
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    fill(h, status, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "%s: no convergence in %d iterations", name, h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "%s: breakdown at iteration %d", name, h.iters);
    return MP_OK;
}

template <int K>
mp_status run_bicgstab(Solver<K> &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info,
                       const char *name)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.v[0], *rh = S.v[1], *p = S.v[2], *v = S.v[3], *ph = S.v[4], *s = S.v[5];
    double *sh = S.v[6], *tv = S.v[7], *q = S.v[8];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int64_t len = (int64_t)K * n;
    mp_status st;
    State<K> h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.st, 0, sizeof(State<K>), S.s));
    if (minv && (st = S.jacobi()) != MP_OK) return st;
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
    MP_HIP_TRY(hipMemsetAsync(v, 0, sizeof(double) * (size_t)len, S.s));
    MP_HIP_TRY(hipMemsetAsync(p, 0, sizeof(double) * (size_t)len, S.s));
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, S.part[0], S.part[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_bi_init<K>, dim3(1), dim3(256), 0, S.s, S.part[0], S.part[1], m, o->rtol * o->rtol,
                       o->max_iter, S.st);
    if ((st = S.launched()) != MP_OK) return st;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, S.part[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_rho<K>, dim3(1), dim3(256), 0, S.s, S.part[0], m, S.st);
                hipLaunchKernelGGL(k_bi_p<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, p, v, ph, minv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(ph, v)) != MP_OK) return st;
                if ((st = S.dot2(rh, v, nullptr, nullptr, S.part[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_alpha<K>, dim3(1), dim3(256), 0, S.s, S.part[0], m, S.st);
                hipLaunchKernelGGL(k_bi_s<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, v, s, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(s, s, nullptr, nullptr, S.part[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_ss<K>, dim3(1), dim3(256), 0, S.s, S.part[0], m, S.st);
                hipLaunchKernelGGL(k_bi_half<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, r, ph, s, S.st);
                hipLaunchKernelGGL(k_bi_half_final<K>, dim3(1), dim3(64), 0, S.s, S.st);
                hipLaunchKernelGGL(k_precond<K>, dim3(S.vb), dim3(256), 0, S.s, n, minv, s, sh, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(sh, tv)) != MP_OK) return st;
                if ((st = S.dot2(tv, s, tv, tv, S.part[0], S.part[1], S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_omega<K>, dim3(1), dim3(256), 0, S.s, S.part[0], S.part[1], m, S.st);
                hipLaunchKernelGGL(k_bi_xr<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, r, ph, sh, s, tv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(r, r, nullptr, nullptr, S.part[2], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_rr<K>, dim3(1), dim3(256), 0, S.s, S.part[2], m, S.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, q, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
            hipLaunchKernelGGL(k_bi_restart<K>, dim3(1), dim3(64), 0, S.s, S.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        break;
    }
    const int status = finish_status(h);
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    fill(h, status, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "%s: no convergence in %d iterations", name, h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "%s: breakdown at iteration %d", name, h.iters);
    return MP_OK;
}


template <int K>
mp_status run_bicg(Solver<K> &S, const mp_csr *At, const double *at, const mp_plan *plan_t, const double *b,
                   double *x, const mp_solve_opts *o, mp_solve_info *info, const char *name)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.v[0], *z = S.v[1], *p = S.v[2], *q = S.v[3], *rt = S.v[4], *zt = S.v[5], *pt = S.v[6], *qt = S.v[7];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int64_t len = (int64_t)K * n;
    mp_status st;
    State<K> h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.st, 0, sizeof(State<K>), S.s));
    if (minv && (st = S.jacobi()) != MP_OK) return st;
    // shadow start r~ = r; z = M^-1 r; z~ = p = p~ = z
    auto reset = [&]() -> mp_status {
        hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rt);
        hipLaunchKernelGGL(k_precond<K>, dim3(S.vb), dim3(256), 0, S.s, n, minv, r, z, nullptr);
        hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, z, zt);
        hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, z, p);
        hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, z, pt);
        return S.launched();
    };
    if ((st = S.residual(b, x, q, r)) != MP_OK) return st;
    if ((st = reset()) != MP_OK) return st;
    if ((st = S.dot2(b, b, rt, z, S.part[0], S.part[1], nullptr)) != MP_OK) return st;
    if ((st = S.dot2(r, r, nullptr, nullptr, S.part[2], nullptr, nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_cg_init<K>, dim3(1), dim3(256), 0, S.s, S.part[0], S.part[1], S.part[2], m, o->rtol * o->rtol,
                       o->max_iter, S.st);
    if ((st = S.launched()) != MP_OK) return st;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.spmv(p, q)) != MP_OK) return st;
                if ((st = spmv_dispatch(K, false, At, at, nullptr, pt, nullptr, qt, nullptr, plan_t, S.xs, S.s)) != MP_OK)
                    return st;
                if ((st = S.dot2(pt, q, nullptr, nullptr, S.part[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bicg_alpha<K>, dim3(1), dim3(256), 0, S.s, S.part[0], m, S.st);
                hipLaunchKernelGGL(k_bicg_update<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, r, z, p, q, rt, zt, qt, minv,
                                   S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(rt, z, r, r, S.part[1], S.part[2], S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bicg_beta<K>, dim3(1), dim3(256), 0, S.s, S.part[1], S.part[2], m, S.st);
                hipLaunchKernelGGL(k_bicg_p<K>, dim3(S.vb), dim3(256), 0, S.s, n, z, p, zt, pt, S.st);
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
            if ((st = S.dot2(rt, z, nullptr, nullptr, S.part[1], nullptr, nullptr)) != MP_OK) return st;
            hipLaunchKernelGGL(k_cg_restart<K>, dim3(1), dim3(256), 0, S.s, S.part[1], m, S.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        break;
    }
    const int status = finish_status(h);
    if ((st = S.true_residual(b, x, q, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    fill(h, status, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "%s: no convergence in %d iterations", name, h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "%s: breakdown at iteration %d", name, h.iters);
    return MP_OK;
}

template <int K>
mp_status run_cgs(Solver<K> &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info,
                  const char *name)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.v[0], *rh = S.v[1], *u = S.v[2], *p = S.v[3], *q = S.v[4], *v = S.v[5];
    double *uh = S.v[6], *t = S.v[7], *ph = S.v[8];
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int64_t len = (int64_t)K * n;
    mp_status st;
    State<K> h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.st, 0, sizeof(State<K>), S.s));
    if (minv && (st = S.jacobi()) != MP_OK) return st;
    if ((st = S.residual(b, x, t, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, S.part[0], S.part[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_bi_init<K>, dim3(1), dim3(256), 0, S.s, S.part[0], S.part[1], m, o->rtol * o->rtol,
                       o->max_iter, S.st);
    if ((st = S.launched()) != MP_OK) return st;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, S.part[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_rho<K>, dim3(1), dim3(256), 0, S.s, S.part[0], m, S.st);
                hipLaunchKernelGGL(k_cgs_up<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, q, u, p, ph, minv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(ph, v)) != MP_OK) return st;
                if ((st = S.dot2(rh, v, nullptr, nullptr, S.part[1], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_alpha<K>, dim3(1), dim3(256), 0, S.s, S.part[1], m, S.st);
                hipLaunchKernelGGL(k_cgs_q<K>, dim3(S.vb), dim3(256), 0, S.s, n, u, v, q, uh, x, minv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(uh, t)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_r<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, t, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(r, r, nullptr, nullptr, S.part[2], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_cgs_rr<K>, dim3(1), dim3(256), 0, S.s, S.part[2], m, S.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, t, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
            hipLaunchKernelGGL(k_bi_restart<K>, dim3(1), dim3(64), 0, S.s, S.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        break;
    }
    const int status = finish_status(h);
    if ((st = S.true_residual(b, x, t, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    fill(h, status, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "%s: no convergence in %d iterations", name, h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "%s: breakdown at iteration %d", name, h.iters);
    return MP_OK;
}

template <int K>
mp_status run_gpbicg(Solver<K> &S, const double *b, double *x, const mp_solve_opts *o, mp_solve_info *info,
                     const char *name)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = S.n;
    const int m = S.m;
    double *r = S.v[0], *rh = S.v[1], *p = S.v[2], *q = S.v[3], *t = S.v[4], *c = S.v[5];
    double *y = S.v[6], *u = S.v[7], *z = S.v[8], *w = S.v[9], *tp = S.v[10], *tmp = S.v[11];
    mpn<K> **P = S.part;
    const double *minv = o->precond == MP_PRECOND_JACOBI ? S.minv : nullptr;
    const int every = o->check_every > 0 ? o->check_every : 32;
    const int64_t len = (int64_t)K * n;
    mp_status st;
    State<K> h;
    std::memset(&h, 0, sizeof(h));
    MP_HIP_TRY(hipMemsetAsync(S.st, 0, sizeof(State<K>), S.s));
    if (minv && (st = S.jacobi()) != MP_OK) return st;
    if ((st = S.residual(b, x, tmp, r)) != MP_OK) return st;
    hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
    if ((st = S.launched()) != MP_OK) return st;
    if ((st = S.dot2(b, b, r, r, P[0], P[1], nullptr)) != MP_OK) return st;
    hipLaunchKernelGGL(k_bi_init<K>, dim3(1), dim3(256), 0, S.s, P[0], P[1], m, o->rtol * o->rtol, o->max_iter, S.st);
    if ((st = S.launched()) != MP_OK) return st;
    for (;;) {
        if ((st = S.read_state(&h)) != MP_OK) return st;
        if (h.done == RUN) {
            for (int it = 0; it < every; ++it) {
                if ((st = S.dot2(rh, r, nullptr, nullptr, P[0], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_rho<K>, dim3(1), dim3(256), 0, S.s, P[0], m, S.st);
                hipLaunchKernelGGL(k_gp_p<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, p, u, c, q, w, tmp, minv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(tmp, q)) != MP_OK) return st;
                if ((st = S.dot2(rh, q, nullptr, nullptr, P[1], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_alpha<K>, dim3(1), dim3(256), 0, S.s, P[1], m, S.st);
                hipLaunchKernelGGL(k_gp_t<K>, dim3(S.vb), dim3(256), 0, S.s, n, r, q, tp, w, t, y, tmp, minv, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(t, t, nullptr, nullptr, P[2], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_bi_ss<K>, dim3(1), dim3(256), 0, S.s, P[2], m, S.st);
                hipLaunchKernelGGL(k_gp_half<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, r, p, t, minv, S.st);
                hipLaunchKernelGGL(k_gp_half_final<K>, dim3(1), dim3(64), 0, S.s, S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.spmv(tmp, c)) != MP_OK) return st;
                if ((st = S.dot2(c, c, c, t, P[0], P[1], S.st)) != MP_OK) return st;
                if ((st = S.dot2(y, y, y, c, P[2], P[3], S.st)) != MP_OK) return st;
                if ((st = S.dot2(y, t, nullptr, nullptr, P[4], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_zeta<K>, dim3(1), dim3(256), 0, S.s, P[0], P[1], P[2], P[3], P[4], m, S.st);
                hipLaunchKernelGGL(k_gp_update<K>, dim3(S.vb), dim3(256), 0, S.s, n, x, r, p, q, t, c, y, u, z, tp, minv,
                                   S.st);
                if ((st = S.launched()) != MP_OK) return st;
                if ((st = S.dot2(r, r, nullptr, nullptr, P[5], nullptr, S.st)) != MP_OK) return st;
                hipLaunchKernelGGL(k_gp_rr<K>, dim3(1), dim3(256), 0, S.s, P[5], m, S.st);
                if ((st = S.launched()) != MP_OK) return st;
            }
            continue;
        }
        if (h.done == RECURRENCE_MET) {
            if ((st = S.true_residual(b, x, tmp, r, true)) != MP_OK) return st;
            continue;
        }
        if (h.done == RESTART) {
            hipLaunchKernelGGL(k_copy, dim3(S.vb), dim3(256), 0, S.s, len, r, rh);
            hipLaunchKernelGGL(k_bi_restart<K>, dim3(1), dim3(64), 0, S.s, S.st);
            if ((st = S.launched()) != MP_OK) return st;
            continue;
        }
        break;
    }
    const int status = finish_status(h);
    if ((st = S.true_residual(b, x, tmp, r, false)) != MP_OK) return st;
    if ((st = S.read_state(&h)) != MP_OK) return st;
    fill(h, status, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), info);
    if (status == MP_ERR_NOT_CONVERGED) return fail(MP_ERR_NOT_CONVERGED, "%s: no convergence in %d iterations", name, h.iters);
    if (status == MP_ERR_BREAKDOWN) return fail(MP_ERR_BREAKDOWN, "%s: breakdown at iteration %d", name, h.iters);
    return MP_OK;
}

// kind 0 CG, 1 BiCGSTAB, 2 CGS, 3 GPBiCG, 4 BiCG (with At, at and plan_t)
template <int K>
mp_status entry(const char *name, int kind, const mp_csr *A, const double *a, const double *b, double *x,
                const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t wsb, mp_solve_info *info,
                void *stream, const mp_csr *At = nullptr, const double *at = nullptr, const mp_plan *plan_t = nullptr)
{
    clear_error();
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (!opts || !info) return fail(MP_ERR_INVALID_ARG, "%s: opts or info is NULL", name);
    if (A->n_rows != A->n_cols) return fail(MP_ERR_INVALID_ARG, "%s: matrix must be square", name);
    if (A->n_rows > 0 && (!b || !x || !ws)) return fail(MP_ERR_INVALID_ARG, "%s: b, x or workspace is NULL", name);
    if (A->nnz > 0 && !a) return fail(MP_ERR_INVALID_ARG, "%s: a is NULL", name);
    if ((int64_t)A->n_rows > (int64_t)kMaxChunks * kChunk)
        return fail(MP_ERR_UNSUPPORTED, "%s: n = %d exceeds the solver limit %d", name, A->n_rows, kMaxChunks * kChunk);
    const size_t need = ws_bytes<K>(A->n_rows);
    if (wsb < need) return fail(MP_ERR_NO_MEMORY, "%s: workspace of %zu bytes, %zu needed", name, wsb, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MP_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", name);
    if (opts->precond != MP_PRECOND_NONE && opts->precond != MP_PRECOND_JACOBI)
        return fail(MP_ERR_INVALID_ARG, "%s: preconditioner must be none or Jacobi (got %d)", name, opts->precond);
    if (!(opts->rtol >= 0.0)) return fail(MP_ERR_INVALID_ARG, "%s: rtol must be >= 0", name);
    if (plan && (plan->ncomp != K || plan->cplx || plan->n_rows != A->n_rows || plan->nnz != A->nnz))
        return fail(MP_ERR_INVALID_ARG, "%s: plan is not a %d-component real plan of this matrix", name, K);
    const size_t vb = sizeof(double) * K * (size_t)A->n_rows;
    if (overlaps(x, vb, b, vb) || overlaps(x, vb, a, sizeof(double) * K * (size_t)A->nnz) || overlaps(x, vb, ws, wsb) ||
        overlaps(b, vb, ws, wsb))
        return fail(MP_ERR_ALIAS, "%s: x overlaps b, a or the workspace", name);
    if (A->n_rows == 0) {
        std::memset(info, 0, sizeof(*info));
        return MP_OK;
    }
    if (kind == 4) {
        if ((st = check_csr(At)) != MP_OK) return st;
        if (At->n_rows != A->n_rows || At->n_cols != A->n_cols || At->nnz != A->nnz)
            return fail(MP_ERR_INVALID_ARG, "%s: At is not %d x %d with %lld elements", name, A->n_rows, A->n_cols,
                        (long long)A->nnz);
        if (A->nnz > 0 && !at) return fail(MP_ERR_INVALID_ARG, "%s: at is NULL", name);
        if (plan_t && (plan_t->ncomp != K || plan_t->cplx || plan_t->n_rows != At->n_rows || plan_t->nnz != At->nnz))
            return fail(MP_ERR_INVALID_ARG, "%s: plan_t is not a %d-component real plan of At", name, K);
        if (overlaps(x, vb, at, sizeof(double) * K * (size_t)A->nnz))
            return fail(MP_ERR_ALIAS, "%s: x overlaps at", name);
    }
    Solver<K> S;
    S.A = A;
    S.a = a;
    S.plan = plan;
    S.s = static_cast<hipStream_t>(stream);
    S.n = A->n_rows;
    S.m = (int)((S.n + kChunk - 1) / kChunk);
    const int64_t blocks = (S.n + 255) / 256;
    S.vb = (unsigned)(blocks < 8192 ? blocks : 8192);
    S.carve(ws);
    switch (kind) {
        case 0: return run_cg<K>(S, b, x, opts, info, name);
        case 1: return run_bicgstab<K>(S, b, x, opts, info, name);
        case 2: return run_cgs<K>(S, b, x, opts, info, name);
        case 3: return run_gpbicg<K>(S, b, x, opts, info, name);
        default: return run_bicg<K>(S, At, at, plan_t, b, x, opts, info, name);
    }
}

}  // namespace kmp
}  // namespace mpk

extern "C" {

mp_status mpkrylov_mp_workspace_bytes(const mp_csr *A, int32_t ncomp, size_t *bytes)
{
    mpk::clear_error();
    mp_status st = mpk::check_csr(A);
    if (st != MP_OK) return st;
    if (!bytes) return mpk::fail(MP_ERR_INVALID_ARG, "bytes is NULL");
    if (ncomp != 3 && ncomp != 4) return mpk::fail(MP_ERR_INVALID_ARG, "ncomp must be 3 or 4 (got %d)", ncomp);
    *bytes = ncomp == 3 ? mpk::kmp::ws_bytes<3>(A->n_rows) : mpk::kmp::ws_bytes<4>(A->n_rows);
    return MP_OK;
}

mp_status mpkrylov_cg_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                         const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<3>("mpkrylov_cg_td", 0, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_cg_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                         const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<4>("mpkrylov_cg_qd", 0, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_bicgstab_td(const mp_csr *A, const double *a, const double *b, double *x,
                               const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                               mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<3>("mpkrylov_bicgstab_td", 1, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_bicgstab_qd(const mp_csr *A, const double *a, const double *b, double *x,
                               const mp_solve_opts *opts, const mp_plan *plan, void *ws, size_t ws_bytes,
                               mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<4>("mpkrylov_bicgstab_qd", 1, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

}  // extern "C"

extern "C" {

mp_status mpkrylov_cgs_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                          const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<3>("mpkrylov_cgs_td", 2, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_cgs_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                          const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<4>("mpkrylov_cgs_qd", 2, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_gpbicg_td(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                             const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<3>("mpkrylov_gpbicg_td", 3, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_gpbicg_qd(const mp_csr *A, const double *a, const double *b, double *x, const mp_solve_opts *opts,
                             const mp_plan *plan, void *ws, size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<4>("mpkrylov_gpbicg_qd", 3, A, a, b, x, opts, plan, ws, ws_bytes, info, stream);
}

mp_status mpkrylov_bicg_td(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                           double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                           size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<3>("mpkrylov_bicg_td", 4, A, a, b, x, opts, plan, ws, ws_bytes, info, stream, At, at, plan_t);
}

mp_status mpkrylov_bicg_qd(const mp_csr *A, const double *a, const mp_csr *At, const double *at, const double *b,
                           double *x, const mp_solve_opts *opts, const mp_plan *plan, const mp_plan *plan_t, void *ws,
                           size_t ws_bytes, mp_solve_info *info, void *stream)
{
    return mpk::kmp::entry<4>("mpkrylov_bicg_qd", 4, A, a, b, x, opts, plan, ws, ws_bytes, info, stream, At, at, plan_t);
}

}  // extern "C"
