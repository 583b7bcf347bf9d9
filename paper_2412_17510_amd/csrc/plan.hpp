// plan.hpp -- the execution plan of a CSR pattern (library-internal layout).
//
// A plan fixes, for one variant (K components, real or complex):
//   * the summation order of every row, i.e. its lane width W = 2^log2w (host and
//     device copies);
//   * the tiles one SpMV launch walks, in row order:
//       SHORT  a contiguous range of rows holding at most tile_nnz elements (and at
//              most tile_nnz rows): the workgroup stages all their products in LDS,
//              then applies the lane/fold order from LDS;
//       LONG   one row longer than tile_nnz with W <= 256: processed in chunks of
//              tile_nnz staged products, W lane accumulators carried in registers;
//   * rows longer than tile_nnz with W >= 512 go to a separate list handled by the
//     register-only wide-row kernel (one row per workgroup);
// A planned SpMV first writes an interleaved copy of x (the K components of x_j, and
// for complex data then the K imaginary ones, side by side) into caller workspace so
// that one gather fetches all components of x_j; the plan itself holds no buffer that
// an SpMV writes, so it is read-only after creation and may serve several streams.
// Tiles are in ascending row order, so the XCD-aware block mapping hands each XCD a
// contiguous range of rows (its L2 then holds the banded part of x those rows gather).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mpsparse.h"

struct mp_stream_tile {
    int32_t row_start;
    int32_t row_count;
    int32_t elem_start;  // first element (row_ptr[row_start])
    int32_t info;        // max_log2w | kind << 4 | elem_count << 8 (SHORT tiles; 0 count for LONG)
};

inline int32_t tile_info(int max_log2w, int kind, int elem_count)
{
    return max_log2w | (kind << 4) | (elem_count << 8);
}

// row-group wavefront: up to 64 / W rows of one lane width W = 2^(info & 15), listed at
// rows[first ..], (info >> 8) of them
struct mp_rg_wave {
    int32_t first;
    int32_t info;
};

// wide-row tile: position in the wide-row permutation and (log2w << 16) | row count
struct mp_tile {
    int32_t first;
    int32_t lw_count;
};

struct mp_plan {
    int32_t n_rows = 0;
    int64_t nnz = 0;
    int32_t ncomp = 2;
    int32_t cplx = 0;
    int32_t tile_nnz = 1024;
    int32_t n_stream = 0;
    int32_t n_wide = 0;
    mp_stream_tile *d_stream = nullptr;   // device, n_stream
    int32_t n_cols = 0;
    uint8_t *d_log2w = nullptr;           // device, n_rows
    int32_t *d_wide_rows = nullptr;       // device, n_wide
    mp_tile *d_wide = nullptr;            // device, n_wide
    int32_t n_rg = 0;                     // row-group wavefronts
    mp_rg_wave *d_rg = nullptr;           // device, n_rg
    int32_t *d_rg_rows = nullptr;         // device: the rows of the row groups, wavefront by wavefront
    std::vector<uint8_t> log2w;           // host copy of the order
    mp_plan_opts opts{0, 6, 0, 0};
    bool explicit_order = false;
};

namespace mpk {

constexpr int kMaxLog2W = 10;
constexpr int kMaxLongLog2W = 8;   // LONG tiles: W <= 256
constexpr int kRgMaxLog2W = 6;     // row groups: W <= 64 (one wavefront)
constexpr int kRgLaneElems = 16;   // row_groups = 1: at most this many elements per lane
constexpr int kRgBlockRows = 2048; // row groups are formed inside blocks of this many rows

// doubles per staged product: K, times 4 accumulator sets for complex
inline int prod_doubles(int K, bool cplx) { return K * (cplx ? 4 : 1); }

// doubles per column of the interleaved x copy
inline int xstage_doubles(int K, bool cplx) { return K * (cplx ? 2 : 1); }

// LDS bytes of a SHORT/LONG tile kernel staging C elements
inline int64_t stream_lds_bytes(int K, bool cplx, int C)
{
    // products, row starts, lane offsets, lane rows, scan scratch; TD adds the fold's
    // row list and width counters
    return (int64_t)C * (8 * prod_doubles(K, cplx) + 4 + 4 + 2) + 16 + (K == 3 ? 2 * (int64_t)C + 128 : 4 + 128);
}

// largest tile size (power of two in 256..2048) that fits 64 KiB of LDS
inline int max_tile_nnz(int K, bool cplx)
{
    int c = 2048;
    while (c > 256 && stream_lds_bytes(K, cplx, c) > 65536) c >>= 1;
    return c;
}

inline int default_tile_nnz(int K, bool cplx)
{
    const int m = max_tile_nnz(K, cplx);
    return m < 1024 ? m : 1024;
}

// lane-width exponent of a row of `len` elements under the plan options
inline int policy_log2w(int64_t len, int shift, int max_log2w)
{
    if (len <= 0) return 0;
    int fl = 0;
    while (fl < 62 && ((int64_t)2 << fl) <= len) ++fl;
    int w = fl - shift;
    if (w < 0) w = 0;
    if (w > max_log2w) w = max_log2w;
    return w;
}

// Build a plan from host row_ptr and per-row log2w (validated by the caller).
mp_status plan_build(const std::vector<int32_t> &row_ptr_host, std::vector<uint8_t> &&log2w, int64_t nnz,
                     int32_t n_cols, int K, bool cplx, int tile_nnz, int row_groups, hipStream_t stream,
                     mp_plan **out);

void plan_free(mp_plan *p);

// bytes of the interleaved copy of x that a planned SpMV writes before its tile kernel
// gathers from it (0 when the plan has no tile kernel, or for a NULL plan)
size_t plan_stage_bytes(const mp_plan *plan);

// the O(1) argument checks of mpspmv_csr_dd (pattern, operands, plan, aliasing; not the
// workspace)
mp_status spmv_check_dd(const char *name, const mp_csr *A, const double *a, const double *x, const double *y,
                        const mp_plan *plan);

// write x into the interleaved copy xs (no-op when the plan needs none); DD real only
mp_status spmv_stage_x(int K, bool cplx, const mp_csr *A, const double *x_re, const double *x_im,
                       const mp_plan *plan, double *xs, hipStream_t s);

// DD real SpMV whose x has already been staged into xs (same x planar: the wide-row
// kernel reads it)
mp_status spmv_dd_prestaged(const mp_csr *A, const double *a, const double *x, double *y, const mp_plan *plan,
                            const double *xs, hipStream_t s);

// launch one SpMV of variant (K, cplx) with an optional plan; xs: staging buffer of at
// least plan_stage_bytes(plan) bytes (may be NULL when that is 0)
mp_status spmv_dispatch(int K, bool cplx, const mp_csr *A, const double *a_re, const double *a_im,
                        const double *x_re, const double *x_im, double *y_re, double *y_im, const mp_plan *plan,
                        double *xs, hipStream_t s);

}  // namespace mpk
