// measure.hip -- throughput probes that state measured ceilings beside the spec-sheet
// ones: the binary64 FMA rate of independent chains (the vector peak as the device
// delivers it) and the rate of the library's own K-component step "multiply, then
// add" (Sec. 2 operations, the inner step of every SpMV here) with two independent
// accumulators per thread.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "mp_arith.hpp"

namespace mpk {
namespace {

constexpr int kRateBlocks = 256 * 16;   // 16 workgroups per compute unit
constexpr int kRateThreads = 256;
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(256) void k_fma_rate(double *out, int iters, double b)
{
    const int tid = blockIdx.x * kRateThreads + threadIdx.x;
    double a[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) a[c] = tid * 1e-9 + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kFmaChains; ++c) a[c] = __builtin_fma(a[c], b, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) s += a[c];
    out[tid] = s;
}

// acc = add(acc, mul(v, w)) on two accumulators; v's leading component is scaled by
// one binary64 multiply per step so that the product cannot be hoisted out of the loop
template <int K>
__global__ __launch_bounds__(256) void k_muladd_rate(double *out, int iters, double b)
{
    const int tid = blockIdx.x * kRateThreads + threadIdx.x;
    mpn<K> v, w, acc[2];
    double scale = 1.0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        v.c[c] = 0.7 * (1.0 + tid * 1e-7) * scale;
        w.c[c] = b * (1.0 - tid * 3e-7) * scale;
        scale *= 0x1p-53;
    }
    acc[0] = mp_mul(v, w);
    acc[1] = mp_mul(w, v);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            acc[c] = mp_add(acc[c], mp_mul(v, w));
            v.c[0] = v.c[0] * 0.9999999;
        }
    }
    out[tid] = acc[0].c[0] + acc[1].c[K - 1];
}

}  // namespace
}  // namespace mpk

extern "C" mp_status mp_measure_rate(int32_t kind, double *per_second, void *stream)
{
    mpk::clear_error();
    if (!per_second) return mpk::fail(MP_ERR_INVALID_ARG, "per_second is NULL");
    if (kind != 0 && (kind < 2 || kind > 4)) return mpk::fail(MP_ERR_INVALID_ARG, "kind must be 0, 2, 3 or 4");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nthreads = (int64_t)mpk::kRateBlocks * mpk::kRateThreads;
    double *out = nullptr;
    MP_HIP_TRY(hipMalloc(reinterpret_cast<void **>(&out), sizeof(double) * (size_t)nthreads));
    const int iters = kind == 0 ? 2048 : (kind == 2 ? 1024 : 128);
    auto launch = [&]() {
        if (kind == 0)
            mpk::k_fma_rate<<<mpk::kRateBlocks, mpk::kRateThreads, 0, s>>>(out, iters, 0.999);
        else if (kind == 2)
            mpk::k_muladd_rate<2><<<mpk::kRateBlocks, mpk::kRateThreads, 0, s>>>(out, iters, 0.3);
        else if (kind == 3)
            mpk::k_muladd_rate<3><<<mpk::kRateBlocks, mpk::kRateThreads, 0, s>>>(out, iters, 0.3);
        else
            mpk::k_muladd_rate<4><<<mpk::kRateBlocks, mpk::kRateThreads, 0, s>>>(out, iters, 0.3);
        return hipGetLastError();
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    constexpr int kReps = 5;
    if (err == hipSuccess) err = launch();   // warm-up
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; err == hipSuccess && r < kReps; ++r) err = launch();
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const hipError_t ferr = hipFree(out);
    if (err == hipSuccess) err = ferr;
    if (err != hipSuccess) return mpk::hip_fail(err, "mp_measure_rate");
    const double per_call = kind == 0 ? (double)mpk::kFmaChains * iters * nthreads : 2.0 * iters * nthreads;
    *per_second = per_call * kReps / (ms * 1e-3);
    return MP_OK;
}
