// Internal helpers of the HIP library: error reporting, launch checks, a
// device-wide exclusive scan and small device utilities.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "bop.h"

namespace bop {

// Thread-local last-error message (see bop_last_error).
void set_error(const char *fmt, ...);

#define BOP_REQUIRE(cond, code, ...)            \
    do {                                        \
        if (!(cond)) {                          \
            ::bop::set_error(__VA_ARGS__);      \
            return (code);                      \
        }                                       \
    } while (0)

#define BOP_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ::bop::set_error("%s failed: %s", #call, hipGetErrorString(e_));   \
            return BOP_E_HIP;                                                  \
        }                                                                      \
    } while (0)

#define BOP_LAUNCHED()                                                         \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) {                                                \
            ::bop::set_error("kernel launch failed: %s", hipGetErrorString(e_)); \
            return BOP_E_HIP;                                                  \
        }                                                                      \
    } while (0)

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bytes of scratch an exclusive scan of n ints needs.
size_t scan_scratch_bytes(long n);
// out[0..n] = exclusive prefix sum of in[0..n-1] (out[n] = total), int32.
// `in` and `out` may alias only if equal.  Enqueued on `stream`.
int exclusive_scan(const int *in, int *out, long n, void *scratch, hipStream_t stream);

// Reduction scratch inside a bop_energy workspace (partials for at least
// ceil(n_rows/256)+1 blocks, two doubles each, and a zeroed counter).
void energy_ws_scratch(void *ws, long n_rows, int n_exp, double **part, unsigned **counter);

// Number of compute units of the current device (cached per device).
int device_cus();

// Small device helpers -------------------------------------------------------
__device__ inline int atomic_load_agent(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void atomic_store_agent(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> __device__ inline T wave_uniform(T v);
template <> __device__ inline int wave_uniform<int>(int v) { return __builtin_amdgcn_readfirstlane(v); }

}  // namespace bop
