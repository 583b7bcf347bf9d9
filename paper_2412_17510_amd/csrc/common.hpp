// common.hpp -- host-side helpers shared by the library's translation units:
// the thread-local error message, HIP error mapping, argument and aliasing checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>

#include "mpsparse.h"

namespace mpk {

// Record a formatted message as the calling thread's last error and return `code`.
mp_status fail(mp_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Map a HIP error to MP_ERR_HIP with the runtime's message.
mp_status hip_fail(hipError_t err, const char *what);

// Clear the calling thread's last error.
void clear_error();

// True if the byte ranges [p, p+pn) and [q, q+qn) overlap (either may be null/empty).
inline bool overlaps(const void *p, size_t pn, const void *q, size_t qn)
{
    if (!p || !q || pn == 0 || qn == 0) return false;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = reinterpret_cast<uintptr_t>(q);
    return a < b + qn && b < a + pn;
}

// O(1) checks of a CSR descriptor: non-null, non-negative sizes, int32-addressable.
mp_status check_csr(const mp_csr *A);

}  // namespace mpk

#define MP_HIP_TRY(call)                                      \
    do {                                                      \
        hipError_t mp_hip_err_ = (call);                      \
        if (mp_hip_err_ != hipSuccess)                        \
            return ::mpk::hip_fail(mp_hip_err_, #call);       \
    } while (0)
