// common.cpp -- error state, version string, CSR descriptor checks and the
// O(nnz) structural validation kernel.
#include "common.hpp"

#include <cstdio>
#include <cstring>

namespace mpk {

namespace {
thread_local char g_last_error[512] = "";
}

mp_status fail(mp_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

mp_status hip_fail(hipError_t err, const char *what)
{
    return fail(MP_ERR_HIP, "%s failed: %s", what, hipGetErrorString(err));
}

void clear_error() { g_last_error[0] = '\0'; }

mp_status check_csr(const mp_csr *A)
{
    if (!A) return fail(MP_ERR_INVALID_ARG, "CSR descriptor is NULL");
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0)
        return fail(MP_ERR_INVALID_ARG, "negative CSR size (n_rows=%d n_cols=%d nnz=%lld)", A->n_rows, A->n_cols,
                    (long long)A->nnz);
    if (A->nnz > INT32_MAX) return fail(MP_ERR_INVALID_ARG, "nnz %lld exceeds int32 indexing", (long long)A->nnz);
    if (!A->row_ptr) return fail(MP_ERR_INVALID_ARG, "row_ptr is NULL");
    if (A->nnz > 0 && !A->col_idx) return fail(MP_ERR_INVALID_ARG, "col_idx is NULL");
    return MP_OK;
}

// Each thread checks one row (row_ptr monotone, in range) and one stretch of columns;
// the smallest offending index of each kind is kept with atomicMin (integer work, no
// ordering concerns).
__global__ void validate_kernel(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t *bad)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n_rows; i += nthr) {
        const int32_t b = row_ptr[i], e = row_ptr[i + 1];
        if (b > e || b < 0 || (int64_t)e > nnz) atomicMin(&bad[0], (int32_t)i);
    }
    if (tid == 0 && (row_ptr[0] != 0 || (int64_t)row_ptr[n_rows] != nnz)) atomicMin(&bad[0], -1);
    for (int64_t k = tid; k < nnz; k += nthr) {
        const int32_t c = col[k];
        if (c < 0 || c >= n_cols) atomicMin(&bad[1], (int32_t)k);
    }
}

}  // namespace mpk

extern "C" {

const char *mp_last_error(void) { return mpk::g_last_error; }

const char *mp_version(void) { return "mpsparse 0.1 (gfx950)"; }

mp_status mp_csr_validate(const mp_csr *A, void *stream)
{
    mpk::clear_error();
    mp_status st = mpk::check_csr(A);
    if (st != MP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *d_bad = nullptr;
    MP_HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&d_bad), 2 * sizeof(int32_t), s));
    const int32_t init[2] = {INT32_MAX, INT32_MAX};
    int32_t h_bad[2];
    hipError_t err = hipMemcpyAsync(d_bad, init, sizeof(init), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) {
        const int64_t work = A->nnz > A->n_rows ? A->nnz : A->n_rows;
        int64_t blocks = (work + 255) / 256;
        if (blocks < 1) blocks = 1;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(mpk::validate_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A->row_ptr, A->col_idx,
                           A->n_rows, A->n_cols, A->nnz, d_bad);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipMemcpyAsync(h_bad, d_bad, sizeof(h_bad), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    hipError_t ferr = hipFreeAsync(d_bad, s);
    if (err != hipSuccess) return mpk::hip_fail(err, "mp_csr_validate");
    if (ferr != hipSuccess) return mpk::hip_fail(ferr, "hipFreeAsync");
    if (h_bad[0] == -1) return mpk::fail(MP_ERR_INVALID_ARG, "row_ptr[0] != 0 or row_ptr[n_rows] != nnz");
    if (h_bad[0] != INT32_MAX) return mpk::fail(MP_ERR_INVALID_ARG, "row_ptr not monotone in range at row %d", h_bad[0]);
    if (h_bad[1] != INT32_MAX) return mpk::fail(MP_ERR_INVALID_ARG, "col_idx out of range at entry %d", h_bad[1]);
    return MP_OK;
}

}  // extern "C"
