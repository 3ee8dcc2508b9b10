// Internal helpers of the HIP library: error reporting, launch checks, a
// device-wide exclusive scan and small device utilities.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cmath>
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

// Packed d-d bond block (FP64/FP32): entry (a, b) of the symmetric 5 x 5
// block, upper triangle row-major; BOP_D_PACKED values per block, the last 0.
__host__ __device__ constexpr int d_packed_index(int a, int b)
{
    return a <= b ? a * 5 - a * (a - 1) / 2 + (b - a) : b * 5 - b * (b - 1) / 2 + (a - b);
}

// Bytes of scratch an exclusive scan of n ints needs.
size_t scan_scratch_bytes(long n);
// out[0..n] = exclusive prefix sum of in[0..n-1] (out[n] = total), int32.
// `in` and `out` may alias only if equal.  Enqueued on `stream`.
int exclusive_scan(const int *in, int *out, long n, void *scratch, hipStream_t stream);

// Reduction scratch inside a bop_energy workspace (partials for at least
// ceil(n_rows/256)+1 blocks, two doubles each, and a zeroed counter).
double *energy_ws_scratch(void *ws, long n_rows, int n_exp);   // block-partial scratch

// Number of compute units of the current device (cached per device).
int device_cus();
// Largest LDS allocation of one workgroup on the current device (cached).
int device_lds_per_block();

// Small device helpers -------------------------------------------------------
// Combination of per-block partials part[q * stride + off], q < n, by all
// threads of one block in a fixed order (thread t takes q = t, t + blockDim.x,
// ...; then a fixed tree over the block), so the result does not depend on
// scheduling.  op 0: sum, 1: min, 2: max.  Valid in thread 0.  Every thread of
// the block must call it; s_red holds blockDim.x / 64 doubles.
__device__ inline double block_combine(double v, int op, double *s_red)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o);
        v = op == 0 ? v + u : (op == 1 ? fmin(v, u) : fmax(v, u));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    double t = v;
    if (threadIdx.x == 0) {
        t = s_red[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
            t = op == 0 ? t + s_red[q] : (op == 1 ? fmin(t, s_red[q]) : fmax(t, s_red[q]));
    }
    __syncthreads();
    return t;
}

__device__ inline double partials_combine(const double *part, unsigned n, size_t stride, size_t off, int op,
                                          double *s_red)
{
    double v = op == 0 ? 0.0 : (op == 1 ? INFINITY : -INFINITY);
    for (unsigned q = threadIdx.x; q < n; q += blockDim.x) {
        const double x = __hip_atomic_load(&part[q * stride + off], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = op == 0 ? v + x : (op == 1 ? fmin(v, x) : fmax(v, x));
    }
    return block_combine(v, op, s_red);
}

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
