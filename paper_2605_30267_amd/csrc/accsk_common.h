// Internal helpers shared by the HIP translation units of libaccsk (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "accsk.h"

namespace accsk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;

// Every grid barrier spins at most this many sleep rounds (about two seconds)
// before it gives up and reports ACCSK_HIP_ERROR, so a kernel always drains.
constexpr long kBarrierSpinLimit = 1L << 25;

// FP64 transcendentals used off the streaming loops.  Kept out of line so
// the polynomial constants are not hoisted into registers for the whole
// persistent kernel.
__device__ __attribute__((noinline)) inline double dlog2(double x) { return log2(x); }
__device__ __attribute__((noinline)) inline double dexp2(double x) { return exp2(x); }
__device__ __attribute__((noinline)) inline double dsqrt(double x) { return sqrt(x); }

// Empty asm barriers that make a value opaque to the optimizer (no code emitted).
template <typename T>
__device__ __forceinline__ void opaque_ptr(T *&p) {
    asm volatile("" : "+s"(p));
}
__device__ __forceinline__ void opaque_int(int &v) { asm volatile("" : "+v"(v)); }

// Deterministic wave-level reductions (fixed xor butterfly, 64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Grid-wide barrier for a cooperative launch.  `bar` is a zeroed 64-bit
// counter; `gen` counts the barriers this block has passed (uniform).
// Returns false if the wait exceeded kBarrierSpinLimit.
__device__ __forceinline__ bool grid_sync(unsigned long long *bar, unsigned long long &gen,
                                          int *lds_flag) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    gen += 1;
    if (threadIdx.x == 0) {
        const unsigned long long target = gen * (unsigned long long)gridDim.x;
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long spins = 0;
        int ok = 1;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kBarrierSpinLimit) {
                ok = 0;
                break;
            }
        }
        *lds_flag = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *lds_flag != 0;
}

// Device-side result record copied back to the host accsk_result.
struct DevResult {
    long long iters;
    long long steps;
    long long fallback;
    double err;
    double eot;
    double fval;
    double cost;
    int converged;
    int status;
};

}  // namespace accsk

#define ACCSK_HIP_TRY(expr)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return ACCSK_HIP_ERROR;        \
    } while (0)
