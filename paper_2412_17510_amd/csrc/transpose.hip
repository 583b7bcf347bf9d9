// transpose.hip -- CSR transpose (for A^T v) and COO -> CSR conversion on the device
// (Sec. 3's storage formats).
//
// The paper forms A^T v by splitting A across threads and combining partial results
// in a critical section (its order depends on the thread schedule) and suggests
// transposing first.  Here the transpose is explicit and deterministic: row j of A^T
// lists column j of A in increasing row order (a stable sort of the elements by
// column), the values permuted with the pattern; A^T v is then an ordinary SpMV of
// A^T with its own plan.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>

#include "common.hpp"

namespace mpk {

__global__ __launch_bounds__(256) void k_t_rows(int32_t n, const int32_t *__restrict__ rp, int32_t *__restrict__ rows)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) rows[k] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_t_iota(int64_t nnz, int32_t *__restrict__ v)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256)
        v[k] = (int32_t)k;
}

// row_ptr_t[j] = first position p of the sorted columns with col >= j: element p
// writes the entries j in (col[p-1], col[p]]; the last one also the tail up to n_cols
__global__ __launch_bounds__(256) void k_t_bounds(int64_t nnz, int32_t n_cols, const int32_t *__restrict__ scol,
                                                  int32_t *__restrict__ rpt)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * 256) {
        // clamped to [0, n_cols] so that a column index outside the matrix cannot write out of bounds
        const int32_t cur = scol[p] < 0 ? 0 : (scol[p] > n_cols ? n_cols : scol[p]);
        int32_t prev = p == 0 ? -1 : scol[p - 1];
        prev = prev < -1 ? -1 : (prev > n_cols ? n_cols : prev);
        for (int32_t j = prev + 1; j <= cur; ++j) rpt[j] = (int32_t)p;
        if (p == nnz - 1)
            for (int32_t j = cur + 1; j <= n_cols; ++j) rpt[j] = (int32_t)nnz;
    }
}

__global__ __launch_bounds__(256) void k_t_empty(int32_t n_cols, int32_t *__restrict__ rpt)
{
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j <= n_cols; j += (int64_t)gridDim.x * 256) rpt[j] = 0;
}

// col_idx_t[p] = row of element perm[p]; values gathered the same way
__global__ __launch_bounds__(256) void k_t_gather(int64_t nnz, int ncomp, const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ rows, const double *__restrict__ a_re,
                                                  const double *__restrict__ a_im, int32_t *__restrict__ cit,
                                                  double *__restrict__ at_re, double *__restrict__ at_im)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * 256) {
        const int64_t k = perm[p];
        cit[p] = rows[k];
        for (int c = 0; c < ncomp; ++c) {
            at_re[c * nnz + p] = a_re[c * nnz + k];
            if (a_im) at_im[c * nnz + p] = a_im[c * nnz + k];
        }
    }
}

// COO coordinates: count those outside the matrix; sort key row * n_cols + col
__global__ __launch_bounds__(256) void k_c_keys(int64_t nnz, int32_t n_rows, int32_t n_cols,
                                                const int32_t *__restrict__ row, const int32_t *__restrict__ col,
                                                uint64_t *__restrict__ key, int32_t *__restrict__ vin,
                                                unsigned int *__restrict__ bad)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * 256) {
        const int32_t r = row[k], c = col[k];
        const bool ok = r >= 0 && r < n_rows && c >= 0 && c < n_cols;
        if (!ok) atomicAdd(bad, 1u);
        key[k] = ok ? (uint64_t)r * (uint64_t)n_cols + (uint64_t)c : 0;
        vin[k] = (int32_t)k;
    }
}

// sorted keys -> row of each element and its column
__global__ __launch_bounds__(256) void k_c_split(int64_t nnz, int32_t n_cols, const uint64_t *__restrict__ key,
                                                 int32_t *__restrict__ srow, int32_t *__restrict__ cout)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * 256) {
        const uint64_t q = key[p];
        srow[p] = (int32_t)(q / (uint64_t)n_cols);
        cout[p] = (int32_t)(q % (uint64_t)n_cols);
    }
}

// values in sorted order: a[c][p] = v[c][perm[p]]
__global__ __launch_bounds__(256) void k_c_gather(int64_t nnz, int ncomp, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ v_re, const double *__restrict__ v_im,
                                                  double *__restrict__ a_re, double *__restrict__ a_im)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * 256) {
        const int64_t k = perm[p];
        for (int c = 0; c < ncomp; ++c) {
            a_re[c * nnz + p] = v_re[c * nnz + k];
            if (v_im) a_im[c * nnz + p] = v_im[c * nnz + k];
        }
    }
}

inline unsigned tgrid(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b < 16384 ? b : 16384));
}

}  // namespace mpk

extern "C" mp_status mp_csr_transpose(const mp_csr *A, int32_t ncomp, const double *a_re, const double *a_im,
                                      int32_t *row_ptr_t, int32_t *col_idx_t, double *at_re, double *at_im,
                                      void *stream)
{
    using namespace mpk;
    clear_error();
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (ncomp < 1 || ncomp > 4) return fail(MP_ERR_INVALID_ARG, "mp_csr_transpose: ncomp must be 1..4 (got %d)", ncomp);
    if (!row_ptr_t) return fail(MP_ERR_INVALID_ARG, "mp_csr_transpose: row_ptr_t is NULL");
    if (A->nnz > 0 && (!a_re || !col_idx_t || !at_re))
        return fail(MP_ERR_INVALID_ARG, "mp_csr_transpose: a_re, col_idx_t or at_re is NULL");
    if ((a_im == nullptr) != (at_im == nullptr))
        return fail(MP_ERR_INVALID_ARG, "mp_csr_transpose: a_im and at_im must both be given or both NULL");
    if (A->nnz >= INT32_MAX) return fail(MP_ERR_UNSUPPORTED, "mp_csr_transpose: nnz must be below 2^31");
    const size_t vb = sizeof(double) * (size_t)ncomp * (size_t)A->nnz;
    const size_t pb = sizeof(int32_t) * ((size_t)A->n_cols + 1), cb = sizeof(int32_t) * (size_t)A->nnz;
    const void *ins[5] = {a_re, a_im, A->row_ptr, A->col_idx, nullptr};
    const size_t insz[5] = {vb, a_im ? vb : 0, sizeof(int32_t) * ((size_t)A->n_rows + 1), cb, 0};
    void *outs[4] = {row_ptr_t, col_idx_t, at_re, at_im};
    const size_t outsz[4] = {pb, cb, vb, at_im ? vb : 0};
    for (int o = 0; o < 4; ++o) {
        for (int i = 0; i < 4; ++i)
            if (overlaps(outs[o], outsz[o], ins[i], insz[i]))
                return fail(MP_ERR_ALIAS, "mp_csr_transpose: an output overlaps an input");
        for (int p = o + 1; p < 4; ++p)
            if (overlaps(outs[o], outsz[o], outs[p], outsz[p]))
                return fail(MP_ERR_ALIAS, "mp_csr_transpose: two outputs overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nnz = A->nnz;
    if (nnz == 0) {
        hipLaunchKernelGGL(k_t_empty, dim3(tgrid((int64_t)A->n_cols + 1)), dim3(256), 0, s, A->n_cols, row_ptr_t);
        MP_HIP_TRY(hipGetLastError());
        MP_HIP_TRY(hipStreamSynchronize(s));
        return MP_OK;
    }
    // temporaries: rows, keys out, values in/out, sort workspace
    int end_bit = 1;
    while (end_bit < 31 && ((int64_t)1 << end_bit) < (int64_t)A->n_cols) ++end_bit;
    size_t sort_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const int32_t *)nullptr, (int32_t *)nullptr,
                                                      (const int32_t *)nullptr, (int32_t *)nullptr, (int)nnz, 0,
                                                      end_bit, s);
    if (e != hipSuccess) return hip_fail(e, "mp_csr_transpose: sort size query");
    char *tmp = nullptr;
    const size_t n4 = ((size_t)nnz * sizeof(int32_t) + 255) & ~(size_t)255;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&tmp), 4 * n4 + sort_bytes));
    int32_t *rows = reinterpret_cast<int32_t *>(tmp);
    int32_t *scol = reinterpret_cast<int32_t *>(tmp + n4);
    int32_t *vin = reinterpret_cast<int32_t *>(tmp + 2 * n4);
    int32_t *perm = reinterpret_cast<int32_t *>(tmp + 3 * n4);
    void *sort_ws = tmp + 4 * n4;
    hipLaunchKernelGGL(k_t_rows, dim3(tgrid(A->n_rows)), dim3(256), 0, s, A->n_rows, A->row_ptr, rows);
    hipLaunchKernelGGL(k_t_iota, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, vin);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(sort_ws, sort_bytes, A->col_idx, scol, vin, perm, (int)nnz, 0, end_bit,
                                               s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_t_bounds, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, A->n_cols, scol, row_ptr_t);
        hipLaunchKernelGGL(k_t_gather, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, ncomp, perm, rows, a_re, a_im, col_idx_t,
                           at_re, at_im);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "mp_csr_transpose");
    return MP_OK;
}

extern "C" mp_status mp_coo_to_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row,
                                   const int32_t *col, int32_t ncomp, const double *v_re, const double *v_im,
                                   int32_t *row_ptr, int32_t *col_idx, double *a_re, double *a_im, void *stream)
{
    using namespace mpk;
    clear_error();
    if (n_rows < 0 || n_cols < 0 || nnz < 0)
        return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: negative size (n_rows=%d n_cols=%d nnz=%lld)", n_rows, n_cols,
                    (long long)nnz);
    if (nnz >= INT32_MAX) return fail(MP_ERR_UNSUPPORTED, "mp_coo_to_csr: nnz must be below 2^31");
    if (nnz > 0 && (n_rows == 0 || n_cols == 0))
        return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: %lld elements in an empty matrix", (long long)nnz);
    if (ncomp < 1 || ncomp > 4) return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: ncomp must be 1..4 (got %d)", ncomp);
    if (!row_ptr) return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: row_ptr is NULL");
    if (nnz > 0 && (!row || !col || !v_re || !col_idx || !a_re))
        return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: row, col, v_re, col_idx or a_re is NULL");
    if ((v_im == nullptr) != (a_im == nullptr))
        return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: v_im and a_im must both be given or both NULL");
    const size_t vb = sizeof(double) * (size_t)ncomp * (size_t)nnz, ib = sizeof(int32_t) * (size_t)nnz;
    const void *ins[4] = {row, col, v_re, v_im};
    const size_t insz[4] = {ib, ib, vb, v_im ? vb : 0};
    void *outs[4] = {row_ptr, col_idx, a_re, a_im};
    const size_t outsz[4] = {sizeof(int32_t) * ((size_t)n_rows + 1), ib, vb, a_im ? vb : 0};
    for (int o = 0; o < 4; ++o) {
        for (int i = 0; i < 4; ++i)
            if (overlaps(outs[o], outsz[o], ins[i], insz[i]))
                return fail(MP_ERR_ALIAS, "mp_coo_to_csr: an output overlaps an input");
        for (int p = o + 1; p < 4; ++p)
            if (overlaps(outs[o], outsz[o], outs[p], outsz[p]))
                return fail(MP_ERR_ALIAS, "mp_coo_to_csr: two outputs overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nnz == 0) {
        hipLaunchKernelGGL(k_t_empty, dim3(tgrid((int64_t)n_rows + 1)), dim3(256), 0, s, n_rows, row_ptr);
        MP_HIP_TRY(hipGetLastError());
        MP_HIP_TRY(hipStreamSynchronize(s));
        return MP_OK;
    }
    // key bits: enough for n_rows * n_cols - 1
    const uint64_t kmax = (uint64_t)n_rows * (uint64_t)n_cols;
    int end_bit = 1;
    while (end_bit < 64 && ((uint64_t)1 << end_bit) < kmax) ++end_bit;
    size_t sort_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (const uint64_t *)nullptr,
                                                      (uint64_t *)nullptr, (const int32_t *)nullptr, (int32_t *)nullptr,
                                                      (int)nnz, 0, end_bit, s);
    if (e != hipSuccess) return hip_fail(e, "mp_coo_to_csr: sort size query");
    const size_t n8 = ((size_t)nnz * sizeof(uint64_t) + 255) & ~(size_t)255;
    const size_t n4 = ((size_t)nnz * sizeof(int32_t) + 255) & ~(size_t)255;
    char *tmp = nullptr;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&tmp), 2 * n8 + 3 * n4 + 256 + sort_bytes));
    uint64_t *key = reinterpret_cast<uint64_t *>(tmp);
    uint64_t *skey = reinterpret_cast<uint64_t *>(tmp + n8);
    int32_t *vin = reinterpret_cast<int32_t *>(tmp + 2 * n8);
    int32_t *perm = reinterpret_cast<int32_t *>(tmp + 2 * n8 + n4);
    int32_t *srow = reinterpret_cast<int32_t *>(tmp + 2 * n8 + 2 * n4);
    unsigned int *bad = reinterpret_cast<unsigned int *>(tmp + 2 * n8 + 3 * n4);
    void *sort_ws = tmp + 2 * n8 + 3 * n4 + 256;
    unsigned int nbad = 0;
    e = hipMemsetAsync(bad, 0, sizeof(unsigned int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_c_keys, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, n_rows, n_cols, row, col, key, vin, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && nbad > 0) {
        (void)hipFree(tmp);
        return fail(MP_ERR_INVALID_ARG, "mp_coo_to_csr: %u coordinates outside the %d x %d matrix", nbad, n_rows,
                    n_cols);
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(sort_ws, sort_bytes, key, skey, vin, perm, (int)nnz, 0, end_bit, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_c_split, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, n_cols, skey, srow, col_idx);
        hipLaunchKernelGGL(k_t_bounds, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, n_rows, srow, row_ptr);
        hipLaunchKernelGGL(k_c_gather, dim3(tgrid(nnz)), dim3(256), 0, s, nnz, ncomp, perm, v_re, v_im, a_re, a_im);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "mp_coo_to_csr");
    return MP_OK;
}
