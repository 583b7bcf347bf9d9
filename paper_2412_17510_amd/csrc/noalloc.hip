// noalloc.hip -- the DD SpMV for callers that cannot allocate device memory.
//
// mpspmv_csr_dd needs caller workspace for the interleaved copy of x that its tile
// kernel gathers from.  mpspmv_csr_dd_noalloc takes no workspace: it stages x in a
// fixed device array of this file (`scratch`, 16 MiB, so n_cols <= 1,048,576), which
// every GPU the library runs on holds from module load until the process ends.  The
// array's host-side name is not a device address; its address on each device comes
// from hipGetSymbolAddress, taken once per device (with that device current) at the
// first call there, and only that address reaches kernels.  Calls that overlap on one
// GPU share the array and race; nothing in it needs clearing (each call rewrites the
// staged columns before its tile kernel reads them).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "plan.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr size_t kScratchColumns = kScratchBytes / (2 * sizeof(double));   // DD columns
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
mp_status scratch_address(double **out)
{
    int dev = -1;
    MP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return mpk::fail(MP_ERR_UNSUPPORTED, "mpspmv_csr_dd_noalloc: device %d is beyond the %d the library tracks",
                         dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return mpk::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return mpk::fail(MP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MP_OK;
}

}  // namespace

extern "C" mp_status mpspmv_csr_dd_noalloc(const mp_csr *A, const double *a, const double *x, double *y,
                                           const mp_plan *plan, void *stream)
{
    mpk::clear_error();
    mp_status st = mpk::spmv_check_dd("mpspmv_csr_dd_noalloc", A, a, x, y, plan);
    if (st != MP_OK) return st;
    const size_t need = mpk::plan_stage_bytes(plan);
    double *xs = nullptr;
    if (need > 0) {
        if (need > kScratchBytes)
            return mpk::fail(MP_ERR_NO_MEMORY,
                             "mpspmv_csr_dd_noalloc: n_cols = %d needs %zu bytes of staging; the allocation-free call "
                             "holds %zu (n_cols <= %zu)",
                             A->n_cols, need, kScratchBytes, kScratchColumns);
        st = scratch_address(&xs);
        if (st != MP_OK) return st;
    }
    return mpk::spmv_dispatch(2, false, A, a, nullptr, x, nullptr, y, nullptr, plan, xs,
                              static_cast<hipStream_t>(stream));
}
