// plan.hpp -- the execution plan of a CSR pattern (library-internal layout).
//
// A plan fixes the summation order of every row (its lane width W = 2^log2w) and
// the work decomposition of one SpMV:
//   * rows are binned by log2w (stable, so each bin keeps ascending row order) into
//     a permutation `perm`;
//   * each bin is cut into workgroup tiles of 256 lanes: a tile of bin w holds
//     256 >> w rows for w <= 8 and one row for w >= 8;
//   * "small" tiles (w <= 6: whole rows inside one wavefront) and "big" tiles (w >= 7:
//     rows spanning several wavefronts) go to two kernels;
//   * inside each list tiles are ordered by their first row, so the XCD-aware
//     block mapping hands each XCD a contiguous range of rows (its L2 then holds the
//     banded part of x those rows gather).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mpsparse.h"

// A tile: first position in perm, and (log2w << 16) | number of rows.
struct mp_tile {
    int32_t first;
    int32_t lw_count;
};

struct mp_plan {
    int32_t n_rows = 0;
    int64_t nnz = 0;
    int32_t n_small = 0;          // tiles with log2w <= 6
    int32_t n_big = 0;            // tiles with log2w >= 7
    int32_t max_log2w = 0;
    int32_t *d_perm = nullptr;    // device, n_rows
    mp_tile *d_small = nullptr;   // device, n_small
    mp_tile *d_big = nullptr;     // device, n_big
    std::vector<uint8_t> log2w;   // host copy of the order
    mp_width_policy policy{0, 6};
    bool explicit_order = false;
};

namespace mpk {

constexpr int kTileLanes = 256;
constexpr int kMaxLog2W = 10;

// lane-width exponent of a row of `len` elements under a width policy
inline int policy_log2w(int64_t len, const mp_width_policy &p)
{
    if (len <= 0) return 0;
    int fl = 0;
    while (fl < 62 && ((int64_t)2 << fl) <= len) ++fl;
    int w = fl - p.shift;
    if (w < 0) w = 0;
    if (w > p.max_log2w) w = p.max_log2w;
    return w;
}

// Build a plan from host row lengths and per-row log2w (validated by the caller).
mp_status plan_build(const std::vector<int32_t> &row_ptr_host, std::vector<uint8_t> &&log2w, int64_t nnz,
                     hipStream_t stream, mp_plan **out);

}  // namespace mpk
