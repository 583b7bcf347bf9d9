// plan.cpp -- plan construction (row binning by lane width), explicit orders and the
// autotuner.  Host C++; the per-row work is O(n) integer bookkeeping done once per
// pattern, after which SpMV calls only read the uploaded permutation and tile lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "plan.hpp"

namespace mpk {

mp_status spmv_dispatch(int K, bool cplx, const mp_csr *A, const double *a_re, const double *a_im,
                        const double *x_re, const double *x_im, double *y_re, double *y_im, const mp_plan *plan,
                        hipStream_t s);

namespace {

void free_plan(mp_plan *p)
{
    if (!p) return;
    if (p->d_perm) (void)hipFree(p->d_perm);
    if (p->d_small) (void)hipFree(p->d_small);
    if (p->d_big) (void)hipFree(p->d_big);
    delete p;
}

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

}  // namespace

mp_status plan_build(const std::vector<int32_t> &rp, std::vector<uint8_t> &&log2w, int64_t nnz, hipStream_t s,
                     mp_plan **out)
{
    const int32_t n = (int32_t)rp.size() - 1;
    mp_plan *p = new (std::nothrow) mp_plan;
    if (!p) return fail(MP_ERR_NO_MEMORY, "plan allocation failed");
    p->n_rows = n;
    p->nnz = nnz;
    p->log2w = std::move(log2w);
    // stable counting sort of the rows by lane width
    int64_t count[kMaxLog2W + 2] = {0};
    for (int32_t i = 0; i < n; ++i) count[p->log2w[i] + 1]++;
    for (int w = 0; w <= kMaxLog2W; ++w) count[w + 1] += count[w];
    std::vector<int32_t> perm((size_t)n);
    {
        int64_t pos[kMaxLog2W + 1];
        for (int w = 0; w <= kMaxLog2W; ++w) pos[w] = count[w];
        for (int32_t i = 0; i < n; ++i) perm[(size_t)pos[p->log2w[i]]++] = i;
    }
    std::vector<mp_tile> small, big;
    int maxw = 0;
    for (int w = 0; w <= kMaxLog2W; ++w) {
        const int64_t b = count[w], e = count[w + 1];
        if (e > b) maxw = w;
        const int64_t per = w <= 8 ? (kTileLanes >> w) : 1;
        for (int64_t f = b; f < e; f += per) {
            const int64_t cnt = std::min<int64_t>(per, e - f);
            mp_tile t{(int32_t)f, (int32_t)((w << 16) | (int32_t)cnt)};
            (w <= 6 ? small : big).push_back(t);
        }
    }
    auto by_first_row = [&](const mp_tile &a, const mp_tile &b) { return perm[a.first] < perm[b.first]; };
    std::stable_sort(small.begin(), small.end(), by_first_row);
    std::stable_sort(big.begin(), big.end(), by_first_row);
    p->n_small = (int32_t)small.size();
    p->n_big = (int32_t)big.size();
    p->max_log2w = maxw;
    mp_status st = upload(perm, &p->d_perm, s);
    if (st == MP_OK) st = upload(small, &p->d_small, s);
    if (st == MP_OK) st = upload(big, &p->d_big, s);
    if (st == MP_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    if (st != MP_OK) {
        free_plan(p);
        return st;
    }
    *out = p;
    return MP_OK;
}

namespace {

mp_status create_with_policy(const mp_csr *A, const mp_width_policy &pol, hipStream_t s,
                             const std::vector<int32_t> &rp, mp_plan **out)
{
    std::vector<uint8_t> lw((size_t)A->n_rows);
    for (int32_t i = 0; i < A->n_rows; ++i) lw[i] = (uint8_t)policy_log2w((int64_t)rp[i + 1] - rp[i], pol);
    mp_status st = plan_build(rp, std::move(lw), A->nnz, s, out);
    if (st == MP_OK) {
        (*out)->policy = pol;
        (*out)->explicit_order = false;
    }
    return st;
}

mp_status check_policy(const mp_width_policy &pol)
{
    if (pol.shift < 0 || pol.shift > 12 || pol.max_log2w < 0 || pol.max_log2w > kMaxLog2W)
        return fail(MP_ERR_INVALID_ARG, "width policy out of range (shift=%d max_log2w=%d)", pol.shift, pol.max_log2w);
    return MP_OK;
}

}  // namespace

}  // namespace mpk

extern "C" {

mp_status mp_plan_create(const mp_csr *A, const mp_width_policy *policy, void *stream, mp_plan **out)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
    if (st != MP_OK) return st;
    const mp_width_policy pol = policy ? *policy : mp_width_policy{0, 6};
    st = mpk::check_policy(pol);
    if (st != MP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> rp;
    st = mpk::read_row_ptr(A, s, rp);
    if (st != MP_OK) return st;
    return mpk::create_with_policy(A, pol, s, rp, out);
}

mp_status mp_plan_create_explicit(const mp_csr *A, const uint8_t *log2w_host, void *stream, mp_plan **out)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
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
    st = mpk::plan_build(rp, std::move(lw), A->nnz, s, out);
    if (st == MP_OK) (*out)->explicit_order = true;
    return st;
}

mp_status mp_plan_destroy(mp_plan *plan)
{
    mpk::clear_error();
    mpk::free_plan(plan);
    return MP_OK;
}

mp_status mp_plan_row_log2w(const mp_plan *plan, uint8_t *log2w_host)
{
    mpk::clear_error();
    if (!plan || (plan->n_rows > 0 && !log2w_host)) return mpk::fail(MP_ERR_INVALID_ARG, "NULL argument");
    if (plan->n_rows > 0) std::memcpy(log2w_host, plan->log2w.data(), (size_t)plan->n_rows);
    return MP_OK;
}

mp_status mp_plan_info(const mp_plan *plan, int32_t *n_rows, int32_t *n_tiles)
{
    mpk::clear_error();
    if (!plan) return mpk::fail(MP_ERR_INVALID_ARG, "plan is NULL");
    if (n_rows) *n_rows = plan->n_rows;
    if (n_tiles) *n_tiles = plan->n_small + plan->n_big;
    return MP_OK;
}

mp_status mp_plan_autotune(const mp_csr *A, int32_t ncomp, int32_t is_complex, const double *a_re,
                           const double *a_im, const double *x_re, const double *x_im, double *y_re, double *y_im,
                           int32_t reps, void *stream, mp_plan **out, mp_width_policy *chosen)
{
    mpk::clear_error();
    if (!out) return mpk::fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = mpk::check_csr(A);
    if (st != MP_OK) return st;
    if (ncomp < 2 || ncomp > 4) return mpk::fail(MP_ERR_INVALID_ARG, "ncomp must be 2, 3 or 4");
    if (A->nnz > 0 && (!a_re || !x_re || !y_re || (is_complex && (!a_im || !x_im || !y_im))))
        return mpk::fail(MP_ERR_INVALID_ARG, "operand is NULL");
    if (reps < 1) reps = 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int32_t> rp;
    st = mpk::read_row_ptr(A, s, rp);
    if (st != MP_OK) return st;
    // candidate width policies: lane widths from "as wide as the row" (shift 0) to
    // "several elements per lane" (shift 3), capped at 16..1024 lanes
    static const mp_width_policy cands[] = {{0, 6}, {1, 6}, {2, 6}, {3, 6}, {0, 5}, {1, 5}, {2, 5}, {0, 4},
                                            {1, 4}, {2, 4}, {1, 3}, {0, 8}, {1, 8}, {0, 10}};
    hipEvent_t e0, e1;
    MP_HIP_TRY(hipEventCreate(&e0));
    MP_HIP_TRY(hipEventCreate(&e1));
    mp_plan *best = nullptr;
    float best_ms = 0.f;
    mp_width_policy best_pol{0, 6};
    for (const mp_width_policy &pol : cands) {
        mp_plan *p = nullptr;
        st = mpk::create_with_policy(A, pol, s, rp, &p);
        if (st != MP_OK) break;
        st = mpk::spmv_dispatch(ncomp, is_complex != 0, A, a_re, a_im, x_re, x_im, y_re, y_im, p, s);
        hipError_t err = hipSuccess;
        if (st == MP_OK) err = hipEventRecord(e0, s);
        for (int r = 0; st == MP_OK && err == hipSuccess && r < reps; ++r)
            st = mpk::spmv_dispatch(ncomp, is_complex != 0, A, a_re, a_im, x_re, x_im, y_re, y_im, p, s);
        if (st == MP_OK && err == hipSuccess) err = hipEventRecord(e1, s);
        if (st == MP_OK && err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (st == MP_OK && err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (st == MP_OK && err != hipSuccess) st = mpk::hip_fail(err, "autotune timing");
        if (st != MP_OK) {
            mpk::free_plan(p);
            break;
        }
        if (!best || ms < best_ms) {
            mpk::free_plan(best);
            best = p;
            best_ms = ms;
            best_pol = pol;
        } else {
            mpk::free_plan(p);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MP_OK) {
        mpk::free_plan(best);
        return st;
    }
    *out = best;
    if (chosen) *chosen = best_pol;
    return MP_OK;
}

}  // extern "C"
