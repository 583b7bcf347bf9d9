// plan.cpp -- plan construction (row tiling), explicit orders and the autotuner.
// Host C++; the per-row work is O(n) integer bookkeeping done once per pattern and
// variant, after which SpMV calls only read the uploaded tile list and lane widths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace mpk {

void plan_free(mp_plan *p)
{
    if (!p) return;
    if (p->d_stream) (void)hipFree(p->d_stream);
    if (p->d_log2w) (void)hipFree(p->d_log2w);
    if (p->d_wide_rows) (void)hipFree(p->d_wide_rows);
    if (p->d_wide) (void)hipFree(p->d_wide);
    if (p->d_rg) (void)hipFree(p->d_rg);
    if (p->d_rg_rows) (void)hipFree(p->d_rg_rows);
    delete p;
}

namespace {

template <typename T>
mp_status upload(const std::vector<T> &h, T **d, hipStream_t s)
{
    *d = nullptr;
    if (h.empty()) return MP_OK;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(d), h.size() * sizeof(T)));
    MP_HIP_TRY(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return MP_OK;
}

mp_status read_row_ptr(const mp_csr *A, hipStream_t s, std::vector<int32_t> &h)
{
    h.resize((size_t)A->n_rows + 1);
    MP_HIP_TRY(hipMemcpyAsync(h.data(), A->row_ptr, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MP_HIP_TRY(hipStreamSynchronize(s));
    if (h[0] != 0 || (int64_t)h[A->n_rows] != A->nnz)
        return fail(MP_ERR_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n_rows] must equal nnz");
    for (int32_t i = 0; i < A->n_rows; ++i)
        if (h[i + 1] < h[i]) return fail(MP_ERR_INVALID_ARG, "row_ptr decreases at row %d", i);
    return MP_OK;
}

mp_status check_variant(int32_t ncomp, int32_t is_complex)
{
    if (ncomp < 2 || ncomp > 4) return fail(MP_ERR_INVALID_ARG, "ncomp must be 2, 3 or 4 (got %d)", ncomp);
    if (is_complex != 0 && is_complex != 1) return fail(MP_ERR_INVALID_ARG, "is_complex must be 0 or 1");
    return MP_OK;
}

mp_status resolve_tile(int32_t ncomp, int32_t is_complex, int32_t requested, int *tile)
{
    const int mx = max_tile_nnz(ncomp, is_complex != 0);
    if (requested == 0) {
        *tile = default_tile_nnz(ncomp, is_complex != 0);
        return MP_OK;
    }
    if (requested < 256 || requested > 2048 || (requested & (requested - 1)))
        return fail(MP_ERR_INVALID_ARG, "tile_nnz must be 0 or a power of two in 256..2048 (got %d)", requested);
    if (requested > mx)
        return fail(MP_ERR_UNSUPPORTED, "tile_nnz %d exceeds the LDS budget of this variant (max %d)", requested, mx);
    *tile = requested;
    return MP_OK;
}

}  // namespace

mp_status plan_build(const std::vector<int32_t> &rp, std::vector<uint8_t> &&log2w, int64_t nnz, int32_t n_cols,
                     int K, bool cplx, int C, int row_groups, hipStream_t s, mp_plan **out)
{
    const int32_t n = (int32_t)rp.size() - 1;
    mp_plan *p = new (std::nothrow) mp_plan;
    if (!p) return fail(MP_ERR_NO_MEMORY, "plan allocation failed");
    p->n_rows = n;
    p->nnz = nnz;
    p->ncomp = K;
    p->cplx = cplx ? 1 : 0;
    p->tile_nnz = C;
    p->n_cols = n_cols;
    p->log2w = std::move(log2w);
    std::vector<mp_stream_tile> tiles;
    std::vector<int32_t> wide_rows;
    std::vector<mp_tile> wide;
    tiles.reserve((size_t)(nnz / C + 16));
    std::vector<mp_rg_wave> rg;
    std::vector<int32_t> rg_rows;
    if (row_groups) {
        // rows with W <= 64 (and, for row_groups = 1, at most kRgLaneElems elements per
        // lane), block by block of kRgBlockRows rows (so that a stretch of wavefronts covers
        // neighbouring rows), grouped by W inside a block, by decreasing length inside a
        // group; every other row is a LONG tile (W <= 256) or a wide row
        std::vector<int32_t> by_w[kRgMaxLog2W + 1];
        for (int32_t b0 = 0; b0 < n; b0 += kRgBlockRows) {
            const int32_t b1 = n - b0 < kRgBlockRows ? n : b0 + kRgBlockRows;
            for (auto &v : by_w) v.clear();
            for (int32_t r = b0; r < b1; ++r) {
                const int64_t len = (int64_t)rp[r + 1] - rp[r];
                const int lw = p->log2w[r];
                if (lw <= kRgMaxLog2W && (row_groups == 2 || len <= ((int64_t)kRgLaneElems << lw))) {
                    by_w[lw].push_back(r);
                } else if (lw > kMaxLongLog2W) {
                    wide.push_back(mp_tile{(int32_t)wide_rows.size(), (int32_t)((lw << 16) | 1)});
                    wide_rows.push_back(r);
                } else {
                    tiles.push_back(mp_stream_tile{r, 1, rp[r], tile_info(lw, 1, 0)});
                }
            }
            for (int lw = 0; lw <= kRgMaxLog2W; ++lw) {
                const int per = 64 >> lw;
                // longest rows first inside a width class: the rows of one wavefront then
                // have similar lengths, so its lanes finish together
                std::vector<int32_t> &v = by_w[lw];
                std::stable_sort(v.begin(), v.end(), [&rp](int32_t x, int32_t y) {
                    return rp[x + 1] - rp[x] > rp[y + 1] - rp[y];
                });
                for (size_t k = 0; k < v.size(); k += (size_t)per) {
                    const int cnt = v.size() - k < (size_t)per ? (int)(v.size() - k) : per;
                    rg.push_back(mp_rg_wave{(int32_t)rg_rows.size(), lw | (cnt << 8)});
                    rg_rows.insert(rg_rows.end(), v.begin() + (long)k, v.begin() + (long)k + cnt);
                }
            }
        }
    }
    int32_t i = row_groups ? n : 0;
    while (i < n) {
        const int64_t len = (int64_t)rp[i + 1] - rp[i];
        if (len > C) {
            const int lw = p->log2w[i];
            if (lw > kMaxLongLog2W) {
                wide.push_back(mp_tile{(int32_t)wide_rows.size(), (int32_t)((lw << 16) | 1)});
                wide_rows.push_back(i);
            } else {
                tiles.push_back(mp_stream_tile{i, 1, rp[i], tile_info(lw, 1, 0)});
            }
            ++i;
            continue;
        }
        const int32_t start = i;
        int64_t acc = 0;
        int32_t cnt = 0;
        int maxlw = 0;
        while (i < n && cnt < C) {
            const int64_t l = (int64_t)rp[i + 1] - rp[i];
            if (l > C || acc + l > C) break;
            acc += l;
            if (l > 0 && p->log2w[i] > maxlw) maxlw = p->log2w[i];
            ++cnt;
            ++i;
        }
        tiles.push_back(mp_stream_tile{start, cnt, rp[start], tile_info(maxlw, 0, (int)acc)});
    }
    p->n_stream = (int32_t)tiles.size();
    p->n_wide = (int32_t)wide.size();
    p->n_rg = (int32_t)rg.size();
    mp_status st = upload(tiles, &p->d_stream, s);
    if (st == MP_OK) st = upload(rg, &p->d_rg, s);
    if (st == MP_OK) st = upload(rg_rows, &p->d_rg_rows, s);
    if (st == MP_OK) st = upload(p->log2w, &p->d_log2w, s);
    if (st == MP_OK) st = upload(wide_rows, &p->d_wide_rows, s);
    if (st == MP_OK) st = upload(wide, &p->d_wide, s);
    if (st == MP_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st != MP_OK) {
        plan_free(p);
        return st;
    }
    *out = p;
    return MP_OK;
}

namespace {

mp_status create_with_opts(const mp_csr *A, int K, bool cplx, const mp_plan_opts &o, int C, hipStream_t s,
                           const std::vector<int32_t> &rp, mp_plan **out)
{
    std::vector<uint8_t> lw((size_t)A->n_rows);
    for (int32_t i = 0; i < A->n_rows; ++i)
        lw[i] = (uint8_t)policy_log2w((int64_t)rp[i + 1] - rp[i], o.shift, o.max_log2w);
    mp_status st = plan_build(rp, std::move(lw), A->nnz, A->n_cols, K, cplx, C, o.row_groups, s, out);
    if (st == MP_OK) {
        (*out)->opts = o;
        (*out)->opts.tile_nnz = C;
        (*out)->explicit_order = false;
    }
    return st;
}

mp_status check_opts(const mp_plan_opts &o)
{
    if (o.shift < 0 || o.shift > 12 || o.max_log2w < 0 || o.max_log2w > kMaxLog2W || o.row_groups < 0 ||
        o.row_groups > 2)
        return fail(MP_ERR_INVALID_ARG, "plan options out of range (shift=%d max_log2w=%d row_groups=%d)", o.shift,
                    o.max_log2w, o.row_groups);
    return MP_OK;
}

}  // namespace

}  // namespace mpk

extern "C" {

mp_status mp_plan_create(const mp_csr *A, int32_t ncomp, int32_t is_complex, const mp_plan_opts *opts, void *stream,
                         mp_plan **out)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
    if (st == MP_OK) st = mpk::check_variant(ncomp, is_complex);
    if (st != MP_OK) return st;
    const mp_plan_opts o = opts ? *opts : mp_plan_opts{0, 6, 0, 0};
    st = mpk::check_opts(o);
    int C = 0;
    if (st == MP_OK) st = mpk::resolve_tile(ncomp, is_complex, o.tile_nnz, &C);
    if (st != MP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> rp;
    st = mpk::read_row_ptr(A, s, rp);
    if (st != MP_OK) return st;
    return mpk::create_with_opts(A, ncomp, is_complex != 0, o, C, s, rp, out);
}

mp_status mp_plan_create_explicit(const mp_csr *A, int32_t ncomp, int32_t is_complex, const uint8_t *log2w_host,
                                  int32_t tile_nnz, void *stream, mp_plan **out)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
    if (st == MP_OK) st = mpk::check_variant(ncomp, is_complex);
    int C = 0;
    if (st == MP_OK) st = mpk::resolve_tile(ncomp, is_complex, tile_nnz, &C);
    if (st != MP_OK) return st;
    if (A->n_rows > 0 && !log2w_host) return mpk::fail(MP_ERR_INVALID_ARG, "log2w is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> rp;
    st = mpk::read_row_ptr(A, s, rp);
    if (st != MP_OK) return st;
    std::vector<uint8_t> lw(log2w_host, log2w_host + A->n_rows);
    for (int32_t i = 0; i < A->n_rows; ++i) {
        const int64_t len = (int64_t)rp[i + 1] - rp[i];
        if (lw[i] > mpk::kMaxLog2W || (len > 0 && ((int64_t)1 << lw[i]) > len) || (len == 0 && lw[i] != 0))
            return mpk::fail(MP_ERR_INVALID_ARG, "log2w[%d] = %d is not valid for a row of %lld elements", i,
                             (int)lw[i], (long long)len);
    }
    st = mpk::plan_build(rp, std::move(lw), A->nnz, A->n_cols, ncomp, is_complex != 0, C, 0, s, out);
    if (st == MP_OK) {
        (*out)->explicit_order = true;
        (*out)->opts.tile_nnz = C;
    }
    return st;
}

mp_status mp_plan_destroy(mp_plan *plan)
{
    mpk::clear_error();
    mpk::plan_free(plan);
    return MP_OK;
}

mp_status mp_plan_row_log2w(const mp_plan *plan, uint8_t *log2w_host)
{
    mpk::clear_error();
    if (!plan || (plan->n_rows > 0 && !log2w_host)) return mpk::fail(MP_ERR_INVALID_ARG, "NULL argument");
    if (plan->n_rows > 0) std::memcpy(log2w_host, plan->log2w.data(), (size_t)plan->n_rows);
    return MP_OK;
}

mp_status mp_plan_info(const mp_plan *plan, int32_t *n_rows, int32_t *n_tiles, int32_t *tile_nnz, int32_t *ncomp,
                       int32_t *is_complex)
{
    mpk::clear_error();
    if (!plan) return mpk::fail(MP_ERR_INVALID_ARG, "plan is NULL");
    if (n_rows) *n_rows = plan->n_rows;
    if (n_tiles) *n_tiles = plan->n_stream + plan->n_wide + plan->n_rg;
    if (tile_nnz) *tile_nnz = plan->tile_nnz;
    if (ncomp) *ncomp = plan->ncomp;
    if (is_complex) *is_complex = plan->cplx;
    return MP_OK;
}

mp_status mp_plan_autotune(const mp_csr *A, int32_t ncomp, int32_t is_complex, const double *a_re,
                           const double *a_im, const double *x_re, const double *x_im, double *y_re, double *y_im,
                           int32_t reps, void *stream, mp_plan **out, mp_plan_opts *chosen)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
    if (st == MP_OK) st = mpk::check_variant(ncomp, is_complex);
    if (st != MP_OK) return st;
    if (A->nnz > 0 && (!a_re || !x_re || !y_re || (is_complex && (!a_im || !x_im || !y_im))))
        return mpk::fail(MP_ERR_INVALID_ARG, "operand is NULL");
    if (reps < 1) reps = 1;
    const bool cplx = is_complex != 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> rp;
    st = mpk::read_row_ptr(A, s, rp);
    if (st != MP_OK) return st;
    // one staging buffer serves every trial plan (the calls run in order on s)
    double *xs = nullptr;
    if (A->n_cols > 0)
        MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&xs),
                             sizeof(double) * (size_t)mpk::xstage_doubles(ncomp, cplx) * (size_t)A->n_cols));
    hipEvent_t e0, e1;
    hipError_t ee = hipEventCreate(&e0);
    if (ee == hipSuccess) {
        ee = hipEventCreate(&e1);
        if (ee != hipSuccess) (void)hipEventDestroy(e0);
    }
    if (ee != hipSuccess) {
        if (xs) (void)hipFree(xs);
        return mpk::hip_fail(ee, "hipEventCreate");
    }
    // the three fastest plans so far (by their trial time), fastest first
    constexpr int kTop = 3;
    mp_plan *top[kTop] = {nullptr, nullptr, nullptr};
    float top_ms[kTop] = {0.f, 0.f, 0.f};
    auto time_plan = [&](mp_plan *p, float *ms) -> mp_status {
        mp_status t = mpk::spmv_dispatch(ncomp, cplx, A, a_re, a_im, x_re, x_im, y_re, y_im, p, xs, s);
        hipError_t err = hipSuccess;
        if (t == MP_OK) err = hipEventRecord(e0, s);
        for (int r = 0; t == MP_OK && err == hipSuccess && r < reps; ++r)
            t = mpk::spmv_dispatch(ncomp, cplx, A, a_re, a_im, x_re, x_im, y_re, y_im, p, xs, s);
        if (t == MP_OK && err == hipSuccess) err = hipEventRecord(e1, s);
        if (t == MP_OK && err == hipSuccess) err = hipEventSynchronize(e1);
        if (t == MP_OK && err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
        if (t == MP_OK && err != hipSuccess) t = mpk::hip_fail(err, "autotune timing");
        return t;
    };
    auto trial = [&](const mp_plan_opts &o) -> mp_status {
        int C = 0;
        mp_status t = mpk::resolve_tile(ncomp, is_complex, o.tile_nnz, &C);
        if (t != MP_OK) return t;
        mp_plan *p = nullptr;
        t = mpk::create_with_opts(A, ncomp, cplx, o, C, s, rp, &p);
        if (t != MP_OK) return t;
        float ms = 0.f;
        t = time_plan(p, &ms);
        if (t != MP_OK) {
            mpk::plan_free(p);
            return t;
        }
        int k = kTop;
        while (k > 0 && (!top[k - 1] || ms < top_ms[k - 1])) --k;
        if (k == kTop) {
            mpk::plan_free(p);
            return MP_OK;
        }
        mpk::plan_free(top[kTop - 1]);
        for (int j = kTop - 1; j > k; --j) {
            top[j] = top[j - 1];
            top_ms[j] = top_ms[j - 1];
        }
        top[k] = p;
        top_ms[k] = ms;
        return MP_OK;
    };
    // stage 1: tile sizes under a middle-of-the-road order; stage 2: lane-width policies;
    // stage 3: the same policies (W <= 64 only) with row groups, short rows or every row
    const int mx = mpk::max_tile_nnz(ncomp, cplx);
    for (int C = 256; st == MP_OK && C <= mx; C <<= 1) st = trial(mp_plan_opts{1, 6, C, 0});
    const int bestC = top[0] ? top[0]->tile_nnz : mpk::default_tile_nnz(ncomp, cplx);
    static const int pols[][2] = {{0, 6}, {1, 6}, {2, 6}, {3, 6}, {0, 5}, {1, 5}, {2, 5}, {0, 4}, {1, 4},
                                  {2, 4}, {1, 3}, {0, 8}, {1, 8}, {2, 8}};
    for (const auto &pp : pols) {
        if (st != MP_OK) break;
        if (pp[0] != 1 || pp[1] != 6) st = trial(mp_plan_opts{pp[0], pp[1], bestC, 0});
    }
    for (int rg = 1; rg <= 2; ++rg) {
        for (const auto &pp : pols) {
            if (st != MP_OK) break;
            if (pp[1] <= mpk::kRgMaxLog2W) st = trial(mp_plan_opts{pp[0], pp[1], bestC, rg});
        }
    }
    // runoff: the three fastest re-timed twice more, in turn; the lowest total wins
    // (one trial's timing alone can rank near-ties by noise)
    float total[kTop] = {0.f, 0.f, 0.f};
    for (int round = 0; st == MP_OK && round < 2; ++round) {
        for (int k = 0; st == MP_OK && k < kTop; ++k) {
            if (!top[k]) continue;
            float ms = 0.f;
            st = time_plan(top[k], &ms);
            total[k] += ms;
        }
    }
    int win = 0;
    for (int k = 1; k < kTop; ++k)
        if (top[k] && total[k] < total[win]) win = k;
    mp_plan *best = top[win];
    for (int k = 0; k < kTop; ++k)
        if (k != win) mpk::plan_free(top[k]);
    const mp_plan_opts best_o = best ? best->opts : mp_plan_opts{0, 6, 0, 0};
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == MP_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = mpk::hip_fail(e, "hipStreamSynchronize");
    }
    if (xs) (void)hipFree(xs);
    if (st != MP_OK) {
        mpk::plan_free(best);
        return st;
    }
    *out = best;
    if (chosen) *chosen = best_o;
    return MP_OK;
}

}  // extern "C"
