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
//   spmv_stream_kernel  planned path.  SHORT tiles (a contiguous range of rows with at
//                       most C = tile_nnz elements): phase 1 streams the tile's
//                       col_idx / value runs coalesced, gathers x and writes every
//                       product to LDS (all threads busy, many loads in flight);
//                       phase 2 runs the lane/fold order of each row out of LDS.
//                       LONG tiles (one row longer than C, W <= 256): the same two
//                       phases per chunk of C elements, lane sums carried in registers.
//   spmv_wide_kernel    rows longer than C with W = 512 or 1024: lanes strided over
//                       the row in registers, folded in-thread, through LDS, then by
//                       shuffles.
//   spmv_rowpack_kernel no plan: eight rows per wavefront, canonical W chosen in-kernel;
//                       rows with W <= 8 on their own group of eight lanes, wider
//                       rows afterwards with the whole wavefront.
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
    const double *__restrict__ xs;   // interleaved copy of x (planned path)
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
// DM: the matrix holds one binary64 value per element and the product is the
// K-component x times that value (Algs 3-5)
template <int K, bool DM>
__device__ __forceinline__ mpn<K> elem_product(const SpmvArgs &A, int64_t k)
{
    const int32_t j = A.col[k];
    if constexpr (DM)
        return mp_mul_d(load_mp<K>(A.x_re, A.n_cols, j), A.a_re[k]);
    else
        return mp_mul(load_mp<K>(A.a_re, A.nnz, k), load_mp<K>(A.x_re, A.n_cols, j));
}

template <int K, bool DM>
__device__ __forceinline__ void first_product(const SpmvArgs &A, int64_t k, Acc<K, false> &acc)
{
    acc.v = elem_product<K, DM>(A, k);
}

template <int K, bool DM>
__device__ __forceinline__ void add_product(const SpmvArgs &A, int64_t k, Acc<K, false> &acc)
{
    acc.v = mp_add(acc.v, elem_product<K, DM>(A, k));
}

// the four products of Eq. 3 for element k; DM: binary64 matrix parts, each product
// the K-component x part times the matrix part (Algs 3-5)
template <int K, bool DM>
__device__ __forceinline__ Acc<K, true> elem_products_c(const SpmvArgs &A, int64_t k)
{
    const int32_t j = A.col[k];
    const mpn<K> xr = load_mp<K>(A.x_re, A.n_cols, j), xi = load_mp<K>(A.x_im, A.n_cols, j);
    Acc<K, true> p;
    if constexpr (DM) {
        const double ar = A.a_re[k], ai = A.a_im[k];
        p.rr = mp_mul_d(xr, ar);
        p.ii = mp_mul_d(xi, ai);
        p.ri = mp_mul_d(xi, ar);
        p.ir = mp_mul_d(xr, ai);
    } else {
        const mpn<K> ar = load_mp<K>(A.a_re, A.nnz, k), ai = load_mp<K>(A.a_im, A.nnz, k);
        p.rr = mp_mul(ar, xr);
        p.ii = mp_mul(ai, xi);
        p.ri = mp_mul(ar, xi);
        p.ir = mp_mul(ai, xr);
    }
    return p;
}

template <int K, bool DM>
__device__ __forceinline__ void first_product(const SpmvArgs &A, int64_t k, Acc<K, true> &acc)
{
    acc = elem_products_c<K, DM>(A, k);
}

template <int K, bool DM>
__device__ __forceinline__ void add_product(const SpmvArgs &A, int64_t k, Acc<K, true> &acc)
{
    const Acc<K, true> p = elem_products_c<K, DM>(A, k);
    acc.rr = mp_add(acc.rr, p.rr);
    acc.ii = mp_add(acc.ii, p.ii);
    acc.ri = mp_add(acc.ri, p.ri);
    acc.ir = mp_add(acc.ir, p.ir);
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

// Complex products in two passes (H = 1, 2), each with two of Eq. 3's accumulator
// sets: pass 1 sums rr and ii and stores y_re = rr + (-ii), pass 2 sums ri and ir and
// stores y_im = ri + ir.  Every set is summed in the same order as in the one-pass form
// (H = 0), so the results are the same bits; a pass stages half the products in LDS.
template <int K>
struct Acc2 {
    mpn<K> s0, s1;
};

template <int K, bool CPLX, int H>
struct AccSel {
    using type = Acc<K, CPLX>;
};
template <int K, bool CPLX>
struct AccSel<K, CPLX, 1> {
    using type = Acc2<K>;
};
template <int K, bool CPLX>
struct AccSel<K, CPLX, 2> {
    using type = Acc2<K>;
};
template <int K, bool CPLX, int H>
using AccT = typename AccSel<K, CPLX, H>::type;

template <int K>
__device__ __forceinline__ void acc_zero(Acc2<K> &a) { a.s0 = a.s1 = mp_zero<K>(); }
template <int K>
__device__ __forceinline__ void acc_fold_xor(Acc2<K> &a, int mask)
{
    a.s0 = mp_add(a.s0, shfl_xor_mp(a.s0, mask));
    a.s1 = mp_add(a.s1, shfl_xor_mp(a.s1, mask));
}
template <int K>
__device__ __forceinline__ void acc_add(Acc2<K> &a, const Acc2<K> &b)
{
    a.s0 = mp_add(a.s0, b.s0);
    a.s1 = mp_add(a.s1, b.s1);
}

template <int H, int K, bool CPLX>
__device__ __forceinline__ void acc_store_h(const SpmvArgs &A, int32_t row, const Acc<K, CPLX> &a, bool nonempty)
{
    acc_store(A, row, a, nonempty);
}
template <int H, int K>
__device__ __forceinline__ void acc_store_h(const SpmvArgs &A, int32_t row, const Acc2<K> &a, bool nonempty)
{
    if constexpr (H == 1)
        store_mp<K>(A.y_re, A.n_rows, row, nonempty ? mp_add(a.s0, mp_neg(a.s1)) : mp_zero<K>());
    else
        store_mp<K>(A.y_im, A.n_rows, row, nonempty ? mp_add(a.s0, a.s1) : mp_zero<K>());
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
// stream tiles (planned path)
// ---------------------------------------------------------------------------

// Exclusive prefix sum of one int per thread over a 256-thread block.
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wave)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    int pre = 0;
    for (int w = 0; w < wid; ++w) pre += s_wave[w];
    return pre + x - v;
}

// Interleaved copy of x: column j holds its K real components, then (complex) its K
// imaginary ones, so one gather brings every component of x_j.
template <int K, bool CPLX>
__global__ __launch_bounds__(256) void k_stage_x(const double *__restrict__ x_re, const double *__restrict__ x_im,
                                                 int32_t n_cols, double *__restrict__ xs)
{
    constexpr int D = K * (CPLX ? 2 : 1);
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_cols; j += (int64_t)gridDim.x * 256) {
        double v[D];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            v[c] = x_re[c * (int64_t)n_cols + j];
            if constexpr (CPLX) v[K + c] = x_im[c * (int64_t)n_cols + j];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) xs[j * D + c] = v[c];
    }
}

// matrix operands of one element, loaded with the non-temporal hint (streamed once)
template <int K, bool CPLX>
struct AElem {
    int32_t col;
    mpn<K> re;
    mpn<K> im;
};

template <int K, bool CPLX, bool DM>
__device__ __forceinline__ void load_aelem(const SpmvArgs &A, int64_t k, AElem<K, CPLX> &e)
{
    e.col = __builtin_nontemporal_load(A.col + k);
    if constexpr (DM) {
        e.re.c[0] = __builtin_nontemporal_load(A.a_re + k);
        if constexpr (CPLX) e.im.c[0] = __builtin_nontemporal_load(A.a_im + k);
        return;
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
        e.re.c[c] = __builtin_nontemporal_load(A.a_re + c * A.nnz + k);
        if constexpr (CPLX) e.im.c[c] = __builtin_nontemporal_load(A.a_im + c * A.nnz + k);
    }
}

// every component of x_j from the staged copy (one gather)
template <int K, bool CPLX>
struct XVal {
    mpn<K> re;
    mpn<K> im;
};

template <int K, bool CPLX>
__device__ __forceinline__ XVal<K, CPLX> load_x(const SpmvArgs &A, int32_t col)
{
    constexpr int D = K * (CPLX ? 2 : 1);
    const double *xp = A.xs + (int64_t)col * D;
    XVal<K, CPLX> x;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        x.re.c[c] = xp[c];
        if constexpr (CPLX) x.im.c[c] = xp[K + c];
    }
    return x;
}

// product(s) of one element with its x (matrix operand first)
template <int K, bool CPLX, bool DM>
__device__ __forceinline__ Acc<K, CPLX> elem_times_x(const AElem<K, CPLX> &e, const XVal<K, CPLX> &x)
{
    Acc<K, CPLX> p;
    if constexpr (CPLX && DM) {
        p.rr = mp_mul_d(x.re, e.re.c[0]);
        p.ii = mp_mul_d(x.im, e.im.c[0]);
        p.ri = mp_mul_d(x.im, e.re.c[0]);
        p.ir = mp_mul_d(x.re, e.im.c[0]);
    } else if constexpr (CPLX) {
        p.rr = mp_mul(e.re, x.re);
        p.ii = mp_mul(e.im, x.im);
        p.ri = mp_mul(e.re, x.im);
        p.ir = mp_mul(e.im, x.re);
    } else if constexpr (DM) {
        p.v = mp_mul_d(x.re, e.re.c[0]);
    } else {
        p.v = mp_mul(e.re, x.re);
    }
    return p;
}

template <int K, bool CPLX, bool DM>
__device__ __forceinline__ Acc<K, CPLX> staged_product(const SpmvArgs &A, const AElem<K, CPLX> &e)
{
    return elem_times_x<K, CPLX, DM>(e, load_x<K, CPLX>(A, e.col));
}

// the product(s) one pass stages: H = 0 all sets; H = 1 (rr, ii); H = 2 (ri, ir)
template <int K, bool CPLX, bool DM, int H>
__device__ __forceinline__ AccT<K, CPLX, H> elem_times_x_h(const AElem<K, CPLX> &e, const XVal<K, CPLX> &x)
{
    if constexpr (H == 0) {
        return elem_times_x<K, CPLX, DM>(e, x);
    } else {
        Acc2<K> p;
        if constexpr (DM) {
            p.s0 = H == 1 ? mp_mul_d(x.re, e.re.c[0]) : mp_mul_d(x.im, e.re.c[0]);
            p.s1 = H == 1 ? mp_mul_d(x.im, e.im.c[0]) : mp_mul_d(x.re, e.im.c[0]);
        } else {
            p.s0 = H == 1 ? mp_mul(e.re, x.re) : mp_mul(e.re, x.im);
            p.s1 = H == 1 ? mp_mul(e.im, x.im) : mp_mul(e.im, x.re);
        }
        return p;
    }
}

template <int K, bool CPLX, bool DM, int H>
__device__ __forceinline__ AccT<K, CPLX, H> staged_product_h(const SpmvArgs &A, const AElem<K, CPLX> &e)
{
    return elem_times_x_h<K, CPLX, DM, H>(e, load_x<K, CPLX>(A, e.col));
}

// The fold of the short tiles runs over a compact list of (row, lane) pairs for TD
// (fewer wave-wide TD additions with idle lanes; measured +4-5 % real and complex),
// and lane by lane for DD and QD, where the list's bookkeeping costs what it saves.
template <int K>
constexpr bool compact_fold()
{
    return K == 3;
}

// LDS of one stream-tile workgroup staging C elements
template <int K, bool CPLX, int C, int H = 0>
struct StreamLds {
    static constexpr int kFoldRows = compact_fold<K>() ? C : 1;
    AccT<K, CPLX, H> prod[C];  // staged products, later lane sums
    int32_t beg[C + 1];        // row starts relative to the tile's first element
    int32_t off[C + 1];        // first lane of each row
    uint16_t lane_row[C];      // row of each lane
    int32_t wave_tmp[4];
    uint16_t rows_by_w[kFoldRows];   // compact fold: rows with W >= 2, widest first
    int32_t wcnt[16];                // compact fold: rows per log2 W
    int32_t wstart[16];              // compact fold: rows with a larger log2 W
};

// SHORT tile: rows [r0, r0+nr), ne <= C elements starting at e0, at most C rows.
// The element loads are issued first (their addresses need only the descriptor), the
// row bookkeeping overlaps them, then every gather of x is issued before the first
// product is formed, and the products go to LDS.  Loads and gathers are branch-free
// (a thread past the tile's end re-reads the tile's first element and discards it),
// so a thread keeps all of its gathers in flight at once.
template <int K, bool CPLX, int J, bool DM, int H>
__device__ __forceinline__ void short_tile(const SpmvArgs &A, const uint8_t *__restrict__ log2w,
                                           const mp_stream_tile &T, StreamLds<K, CPLX, 256 * J, H> &L)
{
    const int t = threadIdx.x;
    const int r0 = T.row_start;
    const int nr = T.row_count;
    const int32_t e0 = T.elem_start;
    const int ne = T.info >> 8;
    if constexpr (compact_fold<K>())
        if (t < 16) L.wcnt[t] = 0;
    // phase 1a: matrix operands of elements t, t+256, ...
    AElem<K, CPLX> el[J];
    if (ne > 0) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int p = t + 256 * j;
            load_aelem<K, CPLX, DM>(A, (int64_t)e0 + (p < ne ? p : 0), el[j]);
        }
    }
    // rows t*J .. t*J+J-1: starts, lane counts (W, or 0 for an empty row)
    int wl[J];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int i = t * J + q;
        wl[q] = 0;
        if (i < nr) {
            const int32_t b = A.row_ptr[r0 + i], e = A.row_ptr[r0 + i + 1];
            L.beg[i] = b - e0;
            wl[q] = e > b ? (1 << log2w[r0 + i]) : 0;
            sum += wl[q];
        }
    }
    if (t == 0) L.beg[nr] = ne;
    // phase 1b: gather x (all gathers first), products into LDS
    if (ne > 0) {
        XVal<K, CPLX> xv[J];
#pragma unroll
        for (int j = 0; j < J; ++j) xv[j] = load_x<K, CPLX>(A, el[j].col);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int p = t + 256 * j;
            if (p < ne) L.prod[p] = elem_times_x_h<K, CPLX, DM, H>(el[j], xv[j]);
        }
    }
    int run = block_exclusive_scan(sum, L.wave_tmp);
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int i = t * J + q;
        if (i < nr) L.off[i] = run;
        run += wl[q];
    }
    if (t == 255) L.off[nr] = run;
    __syncthreads();
    // lane -> row map
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int i = t * J + q;
        if (i < nr) {
            const int o = L.off[i];
            for (int l = 0; l < wl[q]; ++l) L.lane_row[o + l] = (uint16_t)i;
        }
    }
    if constexpr (compact_fold<K>()) {
        // counting sort of the rows with W >= 2 by log2 W, widest first (the order
        // inside a width class is immaterial: every row folds on its own)
#pragma unroll
        for (int q = 0; q < J; ++q)
            if (wl[q] >= 2) atomicAdd(&L.wcnt[31 - __clz(wl[q])], 1);
        __syncthreads();
        if (t == 0) {
            int acc = 0;
            for (int k = 15; k >= 0; --k) {
                L.wstart[k] = acc;
                acc += L.wcnt[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < J; ++q) {
            if (wl[q] >= 2) {
                const int k = 31 - __clz(wl[q]);
                L.rows_by_w[L.wstart[k] + atomicSub(&L.wcnt[k], 1) - 1] = (uint16_t)(t * J + q);
            }
        }
    }
    __syncthreads();
    // phase 2: lane l of row i sums its products l, l+W, ... and leaves the sum in the
    // slot of its first product (a slot no other lane reads)
    const int nl = L.off[nr];
    int li[J], ll[J], lw[J], lb[J];
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int lane = t + 256 * q;
        li[q] = -1;
        if (lane < nl) {
            const int i = L.lane_row[lane];
            const int o = L.off[i];
            li[q] = i;
            ll[q] = lane - o;
            lw[q] = L.off[i + 1] - o;
            lb[q] = L.beg[i];
            const int e = L.beg[i + 1];
            AccT<K, CPLX, H> acc = L.prod[lb[q] + ll[q]];
            for (int p = lb[q] + ll[q] + lw[q]; p < e; p += lw[q]) acc_add(acc, L.prod[p]);
            L.prod[lb[q] + ll[q]] = acc;
        }
    }
    __syncthreads();
    // fold: acc[l] += acc[l + off] for off = W/2 .. 1
    if constexpr (compact_fold<K>()) {
        // the rows with W > off = 2^k are the first wstart[k] entries of rows_by_w, and
        // each has off pairs: pair p is row rows_by_w[p >> k], lane p mod off
        for (int k = (T.info & 15) - 1; k >= 0; --k) {
            const int pairs = L.wstart[k] << k;
            for (int p = t; p < pairs; p += 256) {
                const int b = L.beg[L.rows_by_w[p >> k]] + (p & ((1 << k) - 1));
                AccT<K, CPLX, H> v = L.prod[b];
                acc_add(v, L.prod[b + (1 << k)]);
                L.prod[b] = v;
            }
            __syncthreads();
        }
    } else {
        for (int off = (1 << (T.info & 15)) >> 1; off >= 1; off >>= 1) {
#pragma unroll
            for (int q = 0; q < J; ++q) {
                if (li[q] >= 0 && ll[q] < off && off < lw[q]) {
                    AccT<K, CPLX, H> v = L.prod[lb[q] + ll[q]];
                    acc_add(v, L.prod[lb[q] + ll[q] + off]);
                    L.prod[lb[q] + ll[q]] = v;
                }
            }
            __syncthreads();
        }
    }
    for (int i = t; i < nr; i += 256) {
        const int b = L.beg[i];
        const bool nonempty = L.beg[i + 1] > b;
        AccT<K, CPLX, H> v;
        if (nonempty) v = L.prod[b];
        else acc_zero(v);
        acc_store_h<H>(A, r0 + i, v, nonempty);
    }
}

// LONG tile: one row of len > C with W <= 256 lanes (lane l on thread l).
//
// Register form: lane l reads its own elements l, l+W, ... straight from memory
// (consecutive lanes read consecutive elements, so every load is coalesced), a batch
// of them issued together (DD four, DD complex and TD / QD two, QD complex one: the
// register budget of the short tiles), and adds their products in order in
// registers.  The fold steps whose partner lies in another wavefront (off >= 64) go
// through LDS, the rest through cross-lane shuffles.
template <int K, bool CPLX>
constexpr int long_batch()
{
    return K == 2 ? (CPLX ? 2 : 4) : (CPLX ? 1 : 2);
}

template <int K, bool CPLX, int J, bool DM, int H>
__device__ __forceinline__ void long_tile_lanes(const SpmvArgs &A, const uint8_t *__restrict__ log2w,
                                                const mp_stream_tile &T, StreamLds<K, CPLX, 256 * J, H> &L)
{
    const int t = threadIdx.x;
    const int row = T.row_start;
    const int32_t b0 = A.row_ptr[row], end = A.row_ptr[row + 1];
    const int W = 1 << log2w[row];
    constexpr int kLongBatch = long_batch<K, CPLX>();
    AccT<K, CPLX, H> acc;
    acc_zero(acc);
    if (t < W) {
        // W <= len, so every lane owns at least one element and starts from its first product
        bool first = true;
        for (int64_t k0 = (int64_t)b0 + t; k0 < end; k0 += (int64_t)kLongBatch * W) {
            // branch-free batch: an element past the row's end re-reads the lane's first one
            AElem<K, CPLX> el[kLongBatch];
#pragma unroll
            for (int q = 0; q < kLongBatch; ++q) {
                const int64_t k = k0 + (int64_t)q * W;
                load_aelem<K, CPLX, DM>(A, k < end ? k : k0, el[q]);
            }
            XVal<K, CPLX> xv[kLongBatch];
#pragma unroll
            for (int q = 0; q < kLongBatch; ++q) xv[q] = load_x<K, CPLX>(A, el[q].col);
#pragma unroll
            for (int q = 0; q < kLongBatch; ++q) {
                if (k0 + (int64_t)q * W < end) {
                    const AccT<K, CPLX, H> p = elem_times_x_h<K, CPLX, DM, H>(el[q], xv[q]);
                    if (first)
                        acc = p;
                    else
                        acc_add(acc, p);
                    first = false;
                }
            }
        }
    }
    // fold acc[l] += acc[l + off], off = W/2 .. 1
    for (int off = W >> 1; off >= 64; off >>= 1) {
        if (t >= off && t < 2 * off) L.prod[t] = acc;
        __syncthreads();
        if (t < off) acc_add(acc, L.prod[t + off]);
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        if (off < W) acc_fold_xor(acc, off);
    if (t == 0) acc_store_h<H>(A, row, acc, true);
}

// LONG tile, staged form (rows whose lanes own many elements): the row's elements pass
// through LDS in chunks of C products, lane l (thread l) carrying its running sum in
// registers.
template <int K, bool CPLX, int J, bool DM, int H>
__device__ __forceinline__ void long_tile_staged(const SpmvArgs &A, const uint8_t *__restrict__ log2w,
                                          const mp_stream_tile &T, StreamLds<K, CPLX, 256 * J, H> &L)
{
    constexpr int C = 256 * J;
    const int t = threadIdx.x;
    const int row = T.row_start;
    const int32_t b0 = A.row_ptr[row], end = A.row_ptr[row + 1];
    const int W = 1 << log2w[row];
    AccT<K, CPLX, H> acc;
    acc_zero(acc);
    for (int32_t c0 = b0; c0 < end; c0 += C) {
        const int cl = (end - c0) < C ? (end - c0) : C;
        AElem<K, CPLX> el[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int p = t + 256 * j;
            if (p < cl) load_aelem<K, CPLX, DM>(A, (int64_t)c0 + p, el[j]);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int p = t + 256 * j;
            if (p < cl) L.prod[p] = staged_product_h<K, CPLX, DM, H>(A, el[j]);
        }
        __syncthreads();
        if (t < W) {
            // first local index p with (c0 - b0 + p) == t (mod W)
            const int rel = (c0 - b0) & (W - 1);
            int p = (t - rel) & (W - 1);
            if (c0 == b0) {
                acc = L.prod[p];   // the lane's first product (p = t < W <= C)
                p += W;
            }
            for (; p < cl; p += W) acc_add(acc, L.prod[p]);
        }
        __syncthreads();
    }
    if (t < W) L.prod[t] = acc;
    __syncthreads();
    for (int off = W >> 1; off >= 1; off >>= 1) {
        if (t < off) {
            AccT<K, CPLX, H> v = L.prod[t];
            acc_add(v, L.prod[t + off]);
            L.prod[t] = v;
        }
        __syncthreads();
    }
    if (t == 0) acc_store_h<H>(A, row, L.prod[0], true);
}

// Complex variants whose tiles run as two passes of two accumulator sets (H = 1, 2):
// QD, whose four staged sets of a 256-element tile fill 32 KiB of LDS and leave room
// for four workgroups per CU, and TD (24 KiB; measured 1.57 -> 1.38 ms on the 1e6-row
// power-law matrix); each pass stages half of that.
template <int K, bool CPLX, bool DM>
constexpr bool two_pass()
{
    return CPLX && K >= 3 && !DM;
}

// workgroups per CU asked of a two-pass tile kernel
template <int K, int J>
constexpr int two_pass_min_blocks()
{
    return J == 1 ? 6 : 1;
}

// A long row runs in register lanes when each lane owns at most kLaneElems elements
// (its chain of dependent batches stays short), else in the staged form, whose chunks
// keep all 256 threads loading.  Both sum in the same order.  TD complex keeps the
// staged form only (measured: its lanes form costs more in occupancy than it saves).
constexpr int kLaneElems = 16;

template <int K, bool CPLX>
constexpr bool lanes_form()
{
    return !(K == 3 && CPLX);
}

__device__ __forceinline__ bool long_in_lanes(const SpmvArgs &A, const uint8_t *__restrict__ log2w, int row)
{
    const int64_t len = (int64_t)A.row_ptr[row + 1] - A.row_ptr[row];
    return len <= ((int64_t)kLaneElems << log2w[row]);
}

// Workgroups per CU the register allocation must leave room for, where LDS admits more
// than the compiler's own register count would: TD complex with one element per thread
// 5 (100 -> 96 registers, +10-12 %), DD complex with one 8 (74 -> 64, +3-5 %), TD real
// with two 8 (68 -> 64, +2-5 %), QD real with two 7 (76 -> 70, +3-4 %).  Elsewhere the
// compiler's allocation stands.
template <int K, bool CPLX, int J, int H = 0>
constexpr int stream_min_blocks()
{
    if (H != 0) return two_pass_min_blocks<K, J>();
    if (K == 3 && CPLX && J == 1) return 5;
    if (K == 2 && CPLX && J == 1) return 8;
    if (K == 3 && !CPLX && J == 2) return 8;
    if (K == 4 && !CPLX && J == 2) return 7;
    return 1;
}

template <int K, bool CPLX, int J, bool DM, int H = 0>
__global__ __launch_bounds__(256, (stream_min_blocks<K, CPLX, J, H>())) void spmv_stream_kernel(
    SpmvArgs A, const mp_stream_tile *__restrict__ tiles, const uint8_t *__restrict__ log2w)
{
    __shared__ StreamLds<K, CPLX, 256 * J, H> L;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const mp_stream_tile T = tiles[tile];
    if (((T.info >> 4) & 15) == 0)
        short_tile<K, CPLX, J, DM, H>(A, log2w, T, L);
    else if (lanes_form<K, CPLX>() && long_in_lanes(A, log2w, T.row_start))
        long_tile_lanes<K, CPLX, J, DM, H>(A, log2w, T, L);
    else
        long_tile_staged<K, CPLX, J, DM, H>(A, log2w, T, L);
}

// ---------------------------------------------------------------------------
// row groups (plans built with row_groups): rows with W <= 64
// ---------------------------------------------------------------------------

// One wavefront per row group: up to 64 / W rows of one lane width W, row r of the group
// on lanes r*W .. r*W + W - 1.  Lane l reads elements l, l+W, ... of its row straight
// from memory (a batch at a time, branch-free), adds their products in order in
// registers starting from its first product, and the W lane sums fold acc[l] +=
// acc[l + off], off = W/2 .. 1, by shuffles inside the lane group: the tile kernels'
// order, with no LDS and no barrier.  Consecutive workgroups of an XCD take consecutive
// groups (a block of neighbouring rows).
template <int K, bool CPLX, bool DM>
__global__ __launch_bounds__(256) void spmv_rowgroup_kernel(SpmvArgs A, const mp_rg_wave *__restrict__ groups,
                                                            const int32_t *__restrict__ rows, int32_t n_groups)
{
    const int g = xcd_tile(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6);
    if (g >= n_groups) return;   // uniform per wavefront
    const mp_rg_wave G = groups[g];
    const int lw = G.info & 15;
    const int nr = G.info >> 8;
    const int W = 1 << lw;
    const int lane = threadIdx.x & 63;
    const int r = lane >> lw;
    const int l = lane & (W - 1);
    constexpr int kBatch = long_batch<K, CPLX>();
    Acc<K, CPLX> acc;
    acc_zero(acc);
    int32_t row = 0;
    bool nonempty = false;
    if (r < nr) {
        row = rows[G.first + r];
        const int32_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
        nonempty = end > beg;
        // W <= len for a non-empty row, so every lane owns at least one element
        bool first = true;
        for (int64_t k0 = (int64_t)beg + l; k0 < end; k0 += (int64_t)kBatch * W) {
            AElem<K, CPLX> el[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t k = k0 + (int64_t)q * W;
                load_aelem<K, CPLX, DM>(A, k < end ? k : k0, el[q]);
            }
            XVal<K, CPLX> xv[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) xv[q] = load_x<K, CPLX>(A, el[q].col);
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                if (k0 + (int64_t)q * W < end) {
                    const Acc<K, CPLX> p = elem_times_x<K, CPLX, DM>(el[q], xv[q]);
                    if (first)
                        acc = p;
                    else
                        acc_add(acc, p);
                    first = false;
                }
            }
        }
    }
    for (int off = W >> 1; off >= 1; off >>= 1) acc_fold_xor(acc, off);
    if (r < nr && l == 0) acc_store(A, row, acc, nonempty);
}

// ---------------------------------------------------------------------------
// wide rows: W = 512 or 1024 (one row per workgroup, lanes in registers)
// ---------------------------------------------------------------------------

template <int K, bool CPLX, int LW, bool DM>
__device__ __forceinline__ void wide_row(const SpmvArgs &A, int first, Acc<K, CPLX> *lds)
{
    constexpr int W = 1 << LW;
    constexpr int J = W / 256;   // lanes per thread
    const int t = threadIdx.x;
    const int32_t row = A.perm[first];
    const int32_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
    Acc<K, CPLX> acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        acc_zero(acc[j]);
        const int l = t + 256 * j;
        if (beg + l < end) {
            first_product<K, DM>(A, beg + l, acc[j]);
            for (int64_t k = (int64_t)beg + l + W; k < end; k += W) add_product<K, DM>(A, k, acc[j]);
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
    for (int off = 128; off >= 64; off >>= 1) {
        __syncthreads();
        lds[t] = acc[0];
        __syncthreads();
        if (t < off) acc_add(acc[0], lds[t + off]);
    }
    // steps inside a wavefront
    wave_fold<K, CPLX, 64>(acc[0]);
    if (t == 0) acc_store(A, row, acc[0], end > beg);
}

template <int K, bool CPLX, bool DM>
__global__ __launch_bounds__(256) void spmv_wide_kernel(SpmvArgs A)
{
    __shared__ Acc<K, CPLX> lds[256];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const mp_tile d = A.tiles[tile];
    if ((d.lw_count >> 16) == 9)
        wide_row<K, CPLX, 9, DM>(A, d.first, lds);
    else
        wide_row<K, CPLX, 10, DM>(A, d.first, lds);
}

// ---------------------------------------------------------------------------
// no plan: canonical W = largest power of two <= min(len, 64)
// ---------------------------------------------------------------------------

template <int K>
__device__ __forceinline__ void acc_fold_xor_if(Acc<K, false> &a, int mask, bool apply)
{
    const mpn<K> o = shfl_xor_mp(a.v, mask);
    if (apply) a.v = mp_add(a.v, o);
}
template <int K>
__device__ __forceinline__ void acc_fold_xor_if(Acc<K, true> &a, int mask, bool apply)
{
    const mpn<K> orr = shfl_xor_mp(a.rr, mask), oii = shfl_xor_mp(a.ii, mask);
    const mpn<K> ori = shfl_xor_mp(a.ri, mask), oir = shfl_xor_mp(a.ir, mask);
    if (apply) {
        a.rr = mp_add(a.rr, orr);
        a.ii = mp_add(a.ii, oii);
        a.ri = mp_add(a.ri, ori);
        a.ir = mp_add(a.ir, oir);
    }
}

__device__ __forceinline__ int canonical_w(int32_t len)
{
    int W = 1;
    while (W < 64 && 2 * W <= len) W *= 2;
    return W;
}

// Eight consecutive rows per wavefront.  A row with W <= 8 runs on its own group of
// eight lanes (lane l of the group: elements l, l+W, ...; folds by shuffles inside the
// group, steps off < W only), so short rows fill the wavefront; the rows with W > 8 then
// run one at a time on the whole wavefront.  The order of every row is the canonical one.
template <int K, bool CPLX, bool DM>
__global__ __launch_bounds__(256) void spmv_rowpack_kernel(SpmvArgs A)
{
    constexpr int kRows = 8;
    const int64_t r0 = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * kRows;
    const int lane = threadIdx.x & 63;
    if (r0 >= A.n_rows) return;   // uniform per wavefront
    const int64_t row = r0 + (lane >> 3);
    const int l = lane & 7;
    int32_t beg = 0, len = 0;
    if (row < A.n_rows) {
        beg = A.row_ptr[row];
        len = A.row_ptr[row + 1] - beg;
    }
    const int W = canonical_w(len);
    const bool packed = row < A.n_rows && W <= 8;
    Acc<K, CPLX> acc;
    acc_zero(acc);
    if (packed && l < W && l < len) {
        first_product<K, DM>(A, beg + l, acc);
        for (int64_t k = (int64_t)beg + l + W; k < beg + len; k += W) add_product<K, DM>(A, k, acc);
    }
#pragma unroll
    for (int off = 4; off >= 1; off >>= 1) acc_fold_xor_if(acc, off, off < W);
    if (packed && l == 0) acc_store(A, (int32_t)row, acc, len > 0);
    // rows with W > 8: the whole wavefront, one row at a time
    for (int j = 0; j < kRows && r0 + j < A.n_rows; ++j) {
        const int32_t rj = (int32_t)(r0 + j);
        const int32_t b = A.row_ptr[rj], e = A.row_ptr[rj + 1];
        const int Wj = canonical_w(e - b);
        if (Wj <= 8) continue;   // uniform per wavefront
        Acc<K, CPLX> a;
        acc_zero(a);
        if (lane < Wj) {
            first_product<K, DM>(A, b + lane, a);
            for (int64_t k = (int64_t)b + lane + Wj; k < e; k += Wj) add_product<K, DM>(A, k, a);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            if (off < Wj) acc_fold_xor(a, off);
        if (lane == 0) acc_store(A, rj, a, true);
    }
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------

template <int K, bool CPLX, int J, bool DM>
mp_status launch_stream(const SpmvArgs &A, const mp_plan *plan, hipStream_t s)
{
    if constexpr (sizeof(StreamLds<K, CPLX, 256 * J>) > 65536) {
        return fail(MP_ERR_UNSUPPORTED, "tile size %d exceeds the LDS budget of this variant", 256 * J);
    } else if constexpr (two_pass<K, CPLX, DM>()) {
        hipLaunchKernelGGL((spmv_stream_kernel<K, CPLX, J, DM, 1>), dim3(plan->n_stream), dim3(256), 0, s, A,
                           plan->d_stream, plan->d_log2w);
        hipLaunchKernelGGL((spmv_stream_kernel<K, CPLX, J, DM, 2>), dim3(plan->n_stream), dim3(256), 0, s, A,
                           plan->d_stream, plan->d_log2w);
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    } else {
        hipLaunchKernelGGL((spmv_stream_kernel<K, CPLX, J, DM>), dim3(plan->n_stream), dim3(256), 0, s, A,
                           plan->d_stream, plan->d_log2w);
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
}

// xs: the interleaved copy of x the tile kernel gathers from (caller memory of at least
// plan_stage_bytes(plan) bytes); stage = false: the caller has already written it
template <int K, bool CPLX, bool DM = false>
mp_status launch_spmv(const mp_csr *Acsr, const double *a_re, const double *a_im, const double *x_re,
                      const double *x_im, double *y_re, double *y_im, const mp_plan *plan, const double *xs,
                      hipStream_t s, bool stage = true)
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
    A.xs = nullptr;
    if (Acsr->n_rows == 0) return MP_OK;
    if (!plan) {
        const int64_t blocks = ((int64_t)Acsr->n_rows + 31) / 32;   // 8 rows per wavefront, 4 per workgroup
        hipLaunchKernelGGL((spmv_rowpack_kernel<K, CPLX, DM>), dim3((unsigned)blocks), dim3(256), 0, s, A);
        MP_HIP_TRY(hipGetLastError());
        return MP_OK;
    }
    if (plan->n_stream > 0 || plan->n_rg > 0) {
        if (plan->n_cols != Acsr->n_cols)
            return fail(MP_ERR_INVALID_ARG, "plan was built for n_cols=%d, matrix has %d", plan->n_cols, Acsr->n_cols);
        if (Acsr->n_cols > 0 && !xs) return fail(MP_ERR_INVALID_ARG, "a planned SpMV needs its staging workspace");
        A.xs = xs;
        if (stage && Acsr->n_cols > 0) {
            const int64_t sb = ((int64_t)Acsr->n_cols + 255) / 256;
            hipLaunchKernelGGL((k_stage_x<K, CPLX>), dim3((unsigned)(sb < 4096 ? sb : 4096)), dim3(256), 0, s, x_re,
                               x_im, Acsr->n_cols, const_cast<double *>(xs));
            MP_HIP_TRY(hipGetLastError());
        }
    }
    if (plan->n_rg > 0) {
        const int64_t blocks = ((int64_t)plan->n_rg + 3) / 4;
        hipLaunchKernelGGL((spmv_rowgroup_kernel<K, CPLX, DM>), dim3((unsigned)blocks), dim3(256), 0, s, A,
                           plan->d_rg, plan->d_rg_rows, plan->n_rg);
        MP_HIP_TRY(hipGetLastError());
    }
    if (plan->n_stream > 0) {
        mp_status st;
        switch (plan->tile_nnz) {
            case 256: st = launch_stream<K, CPLX, 1, DM>(A, plan, s); break;
            case 512: st = launch_stream<K, CPLX, 2, DM>(A, plan, s); break;
            case 1024: st = launch_stream<K, CPLX, 4, DM>(A, plan, s); break;
            case 2048: st = launch_stream<K, CPLX, 8, DM>(A, plan, s); break;
            default: st = fail(MP_ERR_INVALID_ARG, "plan has an invalid tile size %d", plan->tile_nnz);
        }
        if (st != MP_OK) return st;
    }
    if (plan->n_wide > 0) {
        A.perm = plan->d_wide_rows;
        A.tiles = plan->d_wide;
        A.n_tiles = plan->n_wide;
        hipLaunchKernelGGL((spmv_wide_kernel<K, CPLX, DM>), dim3(plan->n_wide), dim3(256), 0, s, A);
        MP_HIP_TRY(hipGetLastError());
    }
    return MP_OK;
}

size_t plan_stage_bytes(const mp_plan *plan)
{
    if (!plan || (plan->n_stream == 0 && plan->n_rg == 0) || plan->n_cols <= 0) return 0;
    return sizeof(double) * (size_t)xstage_doubles(plan->ncomp, plan->cplx != 0) * (size_t)plan->n_cols;
}

// the O(1) argument checks every SpMV entry point runs (the workspace is checked by
// the caller)
template <int K, bool CPLX, bool DM>
mp_status spmv_check(const char *name, const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                     const double *x_im, const double *y_re, const double *y_im, const mp_plan *plan)
{
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (A->n_rows > 0 && (!y_re || (CPLX && !y_im))) return fail(MP_ERR_INVALID_ARG, "%s: y is NULL", name);
    if (A->nnz > 0 && (!a_re || !x_re || (CPLX && (!a_im || !x_im))))
        return fail(MP_ERR_INVALID_ARG, "%s: a or x is NULL", name);
    if (plan && (plan->n_rows != A->n_rows || plan->nnz != A->nnz))
        return fail(MP_ERR_INVALID_ARG, "%s: plan was built for n_rows=%d nnz=%lld, matrix has n_rows=%d nnz=%lld",
                    name, plan->n_rows, (long long)plan->nnz, A->n_rows, (long long)A->nnz);
    if (plan && (plan->ncomp != K || plan->cplx != (CPLX ? 1 : 0)))
        return fail(MP_ERR_INVALID_ARG, "%s: plan was built for ncomp=%d is_complex=%d", name, plan->ncomp,
                    plan->cplx);
    if (plan && (plan->n_stream > 0 || plan->n_rg > 0) && plan->n_cols != A->n_cols)
        return fail(MP_ERR_INVALID_ARG, "%s: plan was built for n_cols=%d, matrix has %d", name, plan->n_cols,
                    A->n_cols);
    const size_t yb = sizeof(double) * K * (size_t)A->n_rows;
    const size_t ab = sizeof(double) * (DM ? 1 : K) * (size_t)A->nnz;
    const size_t xb = sizeof(double) * K * (size_t)A->n_cols;
    const double *ins[4] = {a_re, a_im, x_re, x_im};
    const size_t insz[4] = {ab, CPLX ? ab : 0, xb, CPLX ? xb : 0};
    const double *outs[2] = {y_re, CPLX ? y_im : nullptr};
    for (int o = 0; o < 2; ++o) {
        for (int i = 0; i < 4; ++i)
            if (overlaps(outs[o], outs[o] ? yb : 0, ins[i], insz[i]))
                return fail(MP_ERR_ALIAS, "%s: an output overlaps an input", name);
    }
    if (CPLX && overlaps(y_re, yb, y_im, yb)) return fail(MP_ERR_ALIAS, "%s: y_re overlaps y_im", name);
    return MP_OK;
}

// the staging workspace must not overlap an operand (it is written before the
// operands are read)
template <int K, bool CPLX, bool DM>
bool ws_overlaps(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re, const double *x_im,
                 const double *y_re, const double *y_im, const void *ws, size_t wb)
{
    const size_t yb = sizeof(double) * K * (size_t)A->n_rows;
    const size_t ab = sizeof(double) * (DM ? 1 : K) * (size_t)A->nnz;
    const size_t xb = sizeof(double) * K * (size_t)A->n_cols;
    return overlaps(ws, wb, a_re, ab) || (CPLX && overlaps(ws, wb, a_im, ab)) || overlaps(ws, wb, x_re, xb) ||
           (CPLX && overlaps(ws, wb, x_im, xb)) || overlaps(ws, wb, y_re, yb) || (CPLX && overlaps(ws, wb, y_im, yb)) ||
           overlaps(ws, wb, A->row_ptr, sizeof(int32_t) * ((size_t)A->n_rows + 1)) ||
           overlaps(ws, wb, A->col_idx, sizeof(int32_t) * (size_t)A->nnz);
}

template <int K, bool CPLX, bool DM = false>
mp_status spmv_entry(const char *name, const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
                     const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
                     void *stream)
{
    clear_error();
    mp_status st = spmv_check<K, CPLX, DM>(name, A, a_re, a_im, x_re, x_im, y_re, y_im, plan);
    if (st != MP_OK) return st;
    const size_t need = plan_stage_bytes(plan);
    if (need > 0) {
        if (!ws) return fail(MP_ERR_INVALID_ARG, "%s: the plan needs %zu bytes of workspace and ws is NULL", name, need);
        if (ws_bytes < need)
            return fail(MP_ERR_NO_MEMORY, "%s: workspace of %zu bytes, %zu needed", name, ws_bytes, need);
        if (reinterpret_cast<uintptr_t>(ws) & 255)
            return fail(MP_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", name);
        if (ws_overlaps<K, CPLX, DM>(A, a_re, a_im, x_re, x_im, y_re, y_im, ws, need))
            return fail(MP_ERR_ALIAS, "%s: the workspace overlaps an operand", name);
    }
    return launch_spmv<K, CPLX, DM>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, static_cast<double *>(ws),
                                    static_cast<hipStream_t>(stream));
}

mp_status spmv_check_dd(const char *name, const mp_csr *A, const double *a, const double *x, const double *y,
                        const mp_plan *plan)
{
    return spmv_check<2, false, false>(name, A, a, nullptr, x, nullptr, y, nullptr, plan);
}

mp_status spmv_stage_x(int K, bool cplx, const mp_csr *A, const double *x_re, const double *x_im,
                       const mp_plan *plan, double *xs, hipStream_t s)
{
    if (plan_stage_bytes(plan) == 0) return MP_OK;
    if (K != 2 || cplx) return fail(MP_ERR_UNSUPPORTED, "staging is only exported for the DD real variant");
    if (!xs) return fail(MP_ERR_INVALID_ARG, "staging workspace is NULL");
    const int64_t sb = ((int64_t)A->n_cols + 255) / 256;
    hipLaunchKernelGGL((k_stage_x<2, false>), dim3((unsigned)(sb < 4096 ? sb : 4096)), dim3(256), 0, s, x_re, x_im,
                       A->n_cols, xs);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

mp_status spmv_dd_prestaged(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                            const double *xs, hipStream_t s)
{
    return launch_spmv<2, false>(A, a, nullptr, x, nullptr, y, nullptr, plan, xs, s, false);
}

mp_status spmv_dispatch(int K, bool cplx, const mp_csr *A, const double *a_re, const double *a_im,
                        const double *x_re, const double *x_im, double *y_re, double *y_im, const mp_plan *plan,
                        double *xs, hipStream_t s)
{
    switch (K * 2 + (cplx ? 1 : 0)) {
        case 4: return launch_spmv<2, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        case 5: return launch_spmv<2, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        case 6: return launch_spmv<3, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        case 7: return launch_spmv<3, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        case 8: return launch_spmv<4, false>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        case 9: return launch_spmv<4, true>(A, a_re, a_im, x_re, x_im, y_re, y_im, plan, xs, s);
        default: return fail(MP_ERR_INVALID_ARG, "ncomp must be 2, 3 or 4 (got %d)", K);
    }
}

}  // namespace mpk

extern "C" {

mp_status mpspmv_workspace_bytes(const mp_plan *plan, size_t *bytes)
{
    mpk::clear_error();
    if (!bytes) return mpk::fail(MP_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = mpk::plan_stage_bytes(plan);
    return MP_OK;
}

mp_status mpspmv_csr_dd(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<2, false>("mpspmv_csr_dd", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_td(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<3, false>("mpspmv_csr_td", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_qd(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<4, false>("mpspmv_csr_qd", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_dd_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<2, true>("mpspmv_csr_dd_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

mp_status mpspmv_csr_td_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<3, true>("mpspmv_csr_td_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

mp_status mpspmv_csr_qd_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<4, true>("mpspmv_csr_qd_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

mp_status mpspmv_csr_dd_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<2, false, true>("mpspmv_csr_dd_d", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_td_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<3, false, true>("mpspmv_csr_td_d", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_qd_d(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan, void *ws,
        size_t ws_bytes, void *stream)
{
    return mpk::spmv_entry<4, false, true>("mpspmv_csr_qd_d", A, a, nullptr, x, nullptr, y, nullptr, plan, ws, ws_bytes, stream);
}

mp_status mpspmv_csr_dd_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<2, true, true>("mpspmv_csr_dd_d_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

mp_status mpspmv_csr_td_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<3, true, true>("mpspmv_csr_td_d_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

mp_status mpspmv_csr_qd_d_complex(const mp_csr *A, const double *a_re, const double *a_im, const double *x_re,
        const double *x_im, double *y_re, double *y_im, const mp_plan *plan, void *ws, size_t ws_bytes,
        void *stream)
{
    return mpk::spmv_entry<4, true, true>("mpspmv_csr_qd_d_complex", A, a_re, a_im, x_re, x_im, y_re, y_im, plan, ws, ws_bytes,
        stream);
}

}  // extern "C"
