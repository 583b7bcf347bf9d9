// spmv.hip -- multi-component CSR SpMV kernels for gfx950 and their C entry points.
//
// y = A x in DD / TD / QD, real and complex (Kouya, arXiv 2412.17510, Sec. 3, Fig. 1
// and Eq. 3).  The paper's AVX2 kernel multiplies four gathered vector entries at a
// time and sums the lanes; here the lanes of a wave64 take that role.  Row i with
// lane width W = 2^log2w[i] is summed by W lanes: lane l accumulates the products of
// elements l, l+W, ... in order (accumulator = first product), the W partial sums are
// folded pairwise acc[l] += acc[l+off], off = W/2..1, through cross-lane shuffles
// (one wavefront) or LDS (rows wider than a wavefront).  This order is a function of
// W only, so every kernel below gives bitwise identical results for the same W.
//
// Memory layout (component-planar, Sec. 3): component c of value k at a[c*nnz + k],
// of x_j at x[c*n_cols + j], of y_i at y[c*n_rows + i].  Complex: separate re / im
// blocks over one pattern.  Every nnz reads 4 B of col_idx and 8K B per value block
// once (coalesced along a row's lanes) and gathers K (or 2K) doubles of x.
//
// Kernels
//   spmv_small_kernel  tiles of rows with W <= 64: 256/W rows per 256-thread group,
//                      each row inside one wavefront, fold by shuffles;
//   spmv_big_kernel    rows with W in 128..1024: one (or two, W = 128) rows per
//                      group, 256 lanes per thread-sweep, fold in-thread, then LDS,
//                      then shuffles;
//   spmv_rowwave_kernel no plan: one row per wavefront, canonical W chosen in-kernel.
// Block indices are remapped so that consecutive tiles land on the same XCD.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "mp_arith.hpp"
#include "plan.hpp"

namespace mpk {

struct SpmvArgs {
    const int32_t *__restrict__ row_ptr;
    const int32_t *__restrict__ col;
    const double *__restrict__ a_re;
    const double *__restrict__ a_im;
    const double *__restrict__ x_re;
    const double *__restrict__ x_im;
    double *__restrict__ y_re;
    double *__restrict__ y_im;
    int64_t nnz;
    int32_t n_rows;
    int32_t n_cols;
    const int32_t *__restrict__ perm;
    const mp_tile *__restrict__ tiles;
    int32_t n_tiles;
};

// ---------------------------------------------------------------------------
// accumulators: one K-component value (real) or the four sets of Eq. 3 (complex)
// ---------------------------------------------------------------------------

template <int K, bool CPLX>
struct Acc;

template <int K>
struct Acc<K, false> {
    mpn<K> v;
};

template <int K>
struct Acc<K, true> {
    mpn<K> rr, ii, ri, ir;
};

template <int K>
__device__ __forceinline__ mpn<K> load_mp(const double *__restrict__ base, int64_t stride, int64_t i)
{
    mpn<K> v;
#pragma unroll
    for (int c = 0; c < K; ++c) v.c[c] = base[c * stride + i];
    return v;
}

template <int K>
__device__ __forceinline__ void store_mp(double *__restrict__ base, int64_t stride, int64_t i, const mpn<K> &v)
{
#pragma unroll
    for (int c = 0; c < K; ++c) base[c * stride + i] = v.c[c];
}

template <int K>
__device__ __forceinline__ mpn<K> shfl_xor_mp(const mpn<K> &v, int mask)
{
    mpn<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) r.c[c] = __shfl_xor(v.c[c], mask);
    return r;
}

// products of element k (matrix operand first)
template <int K>
__device__ __forceinline__ void first_product(const SpmvArgs &A, int64_t k, Acc<K, false> &acc)
{
    const int32_t j = A.col[k];
    acc.v = mp_mul(load_mp<K>(A.a_re, A.nnz, k), load_mp<K>(A.x_re, A.n_cols, j));
}

template <int K>
__device__ __forceinline__ void add_product(const SpmvArgs &A, int64_t k, Acc<K, false> &acc)
{
    const int32_t j = A.col[k];
    acc.v = mp_add(acc.v, mp_mul(load_mp<K>(A.a_re, A.nnz, k), load_mp<K>(A.x_re, A.n_cols, j)));
}

template <int K>
__device__ __forceinline__ void first_product(const SpmvArgs &A, int64_t k, Acc<K, true> &acc)
{
    const int32_t j = A.col[k];
    const mpn<K> ar = load_mp<K>(A.a_re, A.nnz, k), ai = load_mp<K>(A.a_im, A.nnz, k);
    const mpn<K> xr = load_mp<K>(A.x_re, A.n_cols, j), xi = load_mp<K>(A.x_im, A.n_cols, j);
    acc.rr = mp_mul(ar, xr);
    acc.ii = mp_mul(ai, xi);
    acc.ri = mp_mul(ar, xi);
    acc.ir = mp_mul(ai, xr);
}

template <int K>
__device__ __forceinline__ void add_product(const SpmvArgs &A, int64_t k, Acc<K, true> &acc)
{
    const int32_t j = A.col[k];
    const mpn<K> ar = load_mp<K>(A.a_re, A.nnz, k), ai = load_mp<K>(A.a_im, A.nnz, k);
    const mpn<K> xr = load_mp<K>(A.x_re, A.n_cols, j), xi = load_mp<K>(A.x_im, A.n_cols, j);
    acc.rr = mp_add(acc.rr, mp_mul(ar, xr));
    acc.ii = mp_add(acc.ii, mp_mul(ai, xi));
    acc.ri = mp_add(acc.ri, mp_mul(ar, xi));
    acc.ir = mp_add(acc.ir, mp_mul(ai, xr));
}

template <int K>
__device__ __forceinline__ void acc_zero(Acc<K, false> &a) { a.v = mp_zero<K>(); }
template <int K>
__device__ __forceinline__ void acc_zero(Acc<K, true> &a)
{
    a.rr = a.ii = a.ri = a.ir = mp_zero<K>();
}

// acc = acc (+) partner, partner taken from lane (lane ^ mask)
template <int K>
__device__ __forceinline__ void acc_fold_xor(Acc<K, false> &a, int mask)
{
    a.v = mp_add(a.v, shfl_xor_mp(a.v, mask));
}
template <int K>
__device__ __forceinline__ void acc_fold_xor(Acc<K, true> &a, int mask)
{
    a.rr = mp_add(a.rr, shfl_xor_mp(a.rr, mask));
    a.ii = mp_add(a.ii, shfl_xor_mp(a.ii, mask));
    a.ri = mp_add(a.ri, shfl_xor_mp(a.ri, mask));
    a.ir = mp_add(a.ir, shfl_xor_mp(a.ir, mask));
}

template <int K>
__device__ __forceinline__ void acc_add(Acc<K, false> &a, const Acc<K, false> &b) { a.v = mp_add(a.v, b.v); }
template <int K>
__device__ __forceinline__ void acc_add(Acc<K, true> &a, const Acc<K, true> &b)
{
    a.rr = mp_add(a.rr, b.rr);
    a.ii = mp_add(a.ii, b.ii);
    a.ri = mp_add(a.ri, b.ri);
    a.ir = mp_add(a.ir, b.ir);
}

template <int K>
__device__ __forceinline__ void acc_store(const SpmvArgs &A, int32_t row, const Acc<K, false> &a, bool nonempty)
{
    store_mp<K>(A.y_re, A.n_rows, row, nonempty ? a.v : mp_zero<K>());
}
template <int K>
__device__ __forceinline__ void acc_store(const SpmvArgs &A, int32_t row, const Acc<K, true> &a, bool nonempty)
{
    // Eq. 3, combined at the end of the row: y_re = rr - ii, y_im = ri + ir
    const mpn<K> yr = nonempty ? mp_add(a.rr, mp_neg(a.ii)) : mp_zero<K>();
    const mpn<K> yi = nonempty ? mp_add(a.ri, a.ir) : mp_zero<K>();
    store_mp<K>(A.y_re, A.n_rows, row, yr);
    store_mp<K>(A.y_im, A.n_rows, row, yi);
}

// Fold the W lane sums of each W-lane group of a wavefront (W <= 64).  Lanes
// l < off receive their partner l + off (= l ^ off inside the group); the other
// lanes' results are never read again.
template <int K, bool CPLX, int W>
__device__ __forceinline__ void wave_fold(Acc<K, CPLX> &acc)
{
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) acc_fold_xor(acc, off);
}

// Block index -> tile index such that each XCD (blocks are dealt round-robin to the
// 8 XCDs) gets one contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int xcd = b & 7;
    const int idx = b >> 3;
    const int per = nblocks >> 3;
    const int rem = nblocks & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// ---------------------------------------------------------------------------
// small tiles: W <= 64
// ---------------------------------------------------------------------------

template <int K, bool CPLX, int LW>
__device__ __forceinline__ void small_tile(const SpmvArgs &A, int first, int nrows)
{
    constexpr int W = 1 << LW;
    const int t = threadIdx.x;
    const int g = t >> LW;
    const int l = t & (W - 1);
    const bool active = g < nrows;
    int32_t row = 0, beg = 0, end = 0;
    if (active) {
        row = A.perm[first + g];
        beg = A.row_ptr[row];
        end = A.row_ptr[row + 1];
    }
    Acc<K, CPLX> acc;
    acc_zero(acc);
    if (beg + l < end) {
        first_product(A, beg + l, acc);
        for (int64_t k = (int64_t)beg + l + W; k < end; k += W) add_product(A, k, acc);
    }
    wave_fold<K, CPLX, W>(acc);
    if (active && l == 0) acc_store(A, row, acc, end > beg);
}

template <int K, bool CPLX>
__global__ __launch_bounds__(256) void spmv_small_kernel(SpmvArgs A)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const mp_tile d = A.tiles[tile];
    const int lw = d.lw_count >> 16;
    const int nrows = d.lw_count & 0xffff;
    switch (lw) {
        case 0: small_tile<K, CPLX, 0>(A, d.first, nrows); break;
        case 1: small_tile<K, CPLX, 1>(A, d.first, nrows); break;
        case 2: small_tile<K, CPLX, 2>(A, d.first, nrows); break;
        case 3: small_tile<K, CPLX, 3>(A, d.first, nrows); break;
        case 4: small_tile<K, CPLX, 4>(A, d.first, nrows); break;
        case 5: small_tile<K, CPLX, 5>(A, d.first, nrows); break;
        default: small_tile<K, CPLX, 6>(A, d.first, nrows); break;
    }
}

// ---------------------------------------------------------------------------
// big tiles: W = 128..1024
// ---------------------------------------------------------------------------

template <int K, bool CPLX, int LW>
__device__ __forceinline__ void big_tile(const SpmvArgs &A, int first, int nrows, Acc<K, CPLX> *lds)
{
    constexpr int W = 1 << LW;
    constexpr int J = W > 256 ? W / 256 : 1;        // lanes per thread
    constexpr int SPAN = W >= 256 ? 256 : W;        // threads per row
    const int t = threadIdx.x;
    const int g = t / SPAN;
    const int l0 = t % SPAN;
    const bool active = g < nrows;
    int32_t row = 0, beg = 0, end = 0;
    if (active) {
        row = A.perm[first + g];
        beg = A.row_ptr[row];
        end = A.row_ptr[row + 1];
    }
    Acc<K, CPLX> acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        acc_zero(acc[j]);
        const int l = l0 + 256 * j;
        if (beg + l < end) {
            first_product(A, beg + l, acc[j]);
            for (int64_t k = (int64_t)beg + l + W; k < end; k += W) add_product(A, k, acc[j]);
        }
    }
    // fold steps whose partner lane lives in the same thread (off >= 256)
#pragma unroll
    for (int off = W / 2; off >= 256; off >>= 1) {
#pragma unroll
        for (int j = 0; j < off / 256; ++j) acc_add(acc[j], acc[j + off / 256]);
    }
    // steps across wavefronts (off = 128, 64) through LDS
#pragma unroll
    for (int off = SPAN / 2; off >= 64; off >>= 1) {
        __syncthreads();
        lds[t] = acc[0];
        __syncthreads();
        if (l0 < off) acc_add(acc[0], lds[t + off]);
    }
    // steps inside a wavefront
    wave_fold<K, CPLX, 64>(acc[0]);
    if (active && l0 == 0) acc_store(A, row, acc[0], end > beg);
}

template <int K, bool CPLX>
__global__ __launch_bounds__(256) void spmv_big_kernel(SpmvArgs A)
{
    __shared__ Acc<K, CPLX> lds[256];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const mp_tile d = A.tiles[tile];
    const int lw = d.lw_count >> 16;
    const int nrows = d.lw_count & 0xffff;
    switch (lw) {
        case 7: big_tile<K, CPLX, 7>(A, d.first, nrows, lds); break;
        case 8: big_tile<K, CPLX, 8>(A, d.first, nrows, lds); break;
        case 9: big_tile<K, CPLX, 9>(A, d.first, nrows, lds); break;
        default: big_tile<K, CPLX, 10>(A, d.first, nrows, lds); break;
    }
}

// ---------------------------------------------------------------------------
// no plan: one row per wavefront, canonical W = largest power of two <= min(len, 64)
// ---------------------------------------------------------------------------

template <int K, bool CPLX>
__global__ __launch_bounds__(256) void spmv_rowwave_kernel(SpmvArgs A)
{
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= A.n_rows) return;   // uniform per wavefront
    const int32_t row = (int32_t)wave;
    const int32_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
    const int32_t len = end - beg;
    int W = 1;
    while (W < 64 && 2 * W <= len) W *= 2;
    Acc<K, CPLX> acc;
    acc_zero(acc);
    if (lane < W && lane < len) {
        first_product(A, beg + lane, acc);
        for (int64_t k = (int64_t)beg + lane + W; k < end; k += W) add_product(A, k, acc);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        if (off < W) acc_fold_xor(acc, off);
    if (lane == 0) acc_store(A, row, acc, len > 0);
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------

template <int K, bool CPLX>
mp_status launch_spmv(const mp_csr *Acsr, const double *a_re, const double *a_im, const double *x_re,
                      const double *x_im, double *y_re, double *y_im, const mp_plan *plan, hipStream_t s)
{
    SpmvArgs A;
    A.row_ptr = Acsr->row_ptr;
    A.col = Acsr->col_idx;
    A.a_re = a_re;
    A.a_im = a_im;
    A.x_re = x_re;
    A.x_im = x_im;
    A.y_re = y_re;
    A.y_im = y_im;
    A.nnz = Acsr->nnz;
    A.n_rows = Acsr->n_rows;
    A.n_cols = Acsr->n_cols;
    A.perm = nullptr;
    A.tiles = nullptr;
    A.n_tiles = 0;
    if (Acsr->n_rows == 0) return MP_OK;
    if (!plan) {
        const int64_t blocks = ((int64_t)Acsr->n_rows + 3) / 4;
        if (blocks > INT32_MAX) return fail(MP_ERR_INVALID_ARG, "too many rows for the plan-free kernel");
        hipLaunchKernelGGL((spmv_rowwave_kernel<K, CPLX>), dim3((unsigned)blocks), dim3(256), 0, s, A);
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
    A.perm = plan->d_perm;
    if (plan->n_small > 0) {
        A.tiles = plan->d_small;
        A.n_tiles = plan->n_small;
        hipLaunchKernelGGL((spmv_small_kernel<K, CPLX>), dim3(plan->n_small), dim3(256), 0, s, A);
        MP_HIP_TRY(hipGetLastError());
    }
    if (plan->n_big > 0) {
        A.tiles = plan->d_big;
        A.n_tiles = plan->n_big;
        hipLaunchKernelGGL((spmv_big_kernel<K, CPLX>), dim3(plan->n_big), dim3(256), 0, s, A);
        MP_HIP_TRY(hipGetLastError());
    }
    return MP_OK;
}

template <int K, bool CPLX>
mp_status spmv_entry(const char *name, const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                     const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *stream)
{
    clear_error();
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (A->n_rows > 0 && (!y_re || (CPLX && !y_im))) return fail(MP_ERR_INVALID_ARG, "%s: y is NULL", name);
    if (A->nnz > 0 && (!a_re || !x_re || (CPLX && (!a_im || !x_im))))
        return fail(MP_ERR_INVALID_ARG, "%s: a or x is NULL", name);
    if (plan && (plan->n_rows != A->n_rows || plan->nnz != A->nnz))
        return fail(MP_ERR_INVALID_ARG, "%s: plan was built for n_rows=%d nnz=%lld, matrix has n_rows=%d nnz=%lld",
                    name, plan->n_rows, (long long)plan->nnz, A->n_rows, (long long)A->nnz);
    const size_t yb = sizeof(double) * K * (size_t)A->n_rows;
    const size_t ab = sizeof(double) * K * (size_t)A->nnz;
    const size_t xb = sizeof(double) * K * (size_t)A->n_cols;
    const double *ins[4] = {a_re, a_im, x_re, x_im};
    const size_t insz[4] = {ab, CPLX ? ab : 0, xb, CPLX ? xb : 0};
    double *outs[2] = {y_re, CPLX ? y_im : nullptr};
    for (int o = 0; o < 2; ++o) {
        for (int i = 0; i < 4; ++i)
            if (overlaps(outs[o], outs[o] ? yb : 0, ins[i], insz[i]))
                return fail(MP_ERR_ALIAS, "%s: an output overlaps an input", name);
    }
    if (CPLX && overlaps(y_re, yb, y_im, yb)) return fail(MP_ERR_ALIAS, "%s: y_re overlaps y_im", name);
    return launch_spmv<K, CPLX>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, static_cast<hipStream_t>(stream));
}

// used by the autotuner
mp_status spmv_dispatch(int K, bool cplx, const mp_csr *A, const double *a_re, const double *a_im,
                        const double *x_re, const double *x_im, double *y_re, double *y_im, const mp_plan *plan,
                        hipStream_t s)
{
    switch (K * 2 + (cplx ? 1 : 0)) {
        case 4: return launch_spmv<2, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        case 5: return launch_spmv<2, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        case 6: return launch_spmv<3, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        case 7: return launch_spmv<3, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        case 8: return launch_spmv<4, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        case 9: return launch_spmv<4, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, s);
        default: return fail(MP_ERR_INVALID_ARG, "ncomp must be 2, 3 or 4 (got %d)", K);
    }
}

}  // namespace mpk

extern "C" {

mp_status mpspmv_csr_dd(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                        void *stream)
{
    return mpk::spmv_entry<2, false>("mpspmv_csr_dd", A, a, nullptr, x, nullptr, y, nullptr, plan, stream);
}

mp_status mpspmv_csr_td(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                        void *stream)
{
    return mpk::spmv_entry<3, false>("mpspmv_csr_td", A, a, nullptr, x, nullptr, y, nullptr, plan, stream);
}

mp_status mpspmv_csr_qd(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                        void *stream)
{
    return mpk::spmv_entry<4, false>("mpspmv_csr_qd", A, a, nullptr, x, nullptr, y, nullptr, plan, stream);
}

mp_status mpspmv_csr_dd_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *stream)
{
    return mpk::spmv_entry<2, true>("mpspmv_csr_dd_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, stream);
}

mp_status mpspmv_csr_td_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *stream)
{
    return mpk::spmv_entry<3, true>("mpspmv_csr_td_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, stream);
}

mp_status mpspmv_csr_qd_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                                const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *stream)
{
    return mpk::spmv_entry<4, true>("mpspmv_csr_qd_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, stream);
}

}  // extern "C"
