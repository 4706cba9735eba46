// Device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include <cstdint>

#include "kernels.h"

// Launch through hipExtLaunchKernel with the timing events of an open timed
// scope (first launch only), else a plain launch.
#define TPT_KLAUNCH(KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                                  \
    do {                                                                                                    \
        ::tpt::LaunchEvents& le_ = ::tpt::launch_events();                                                  \
        if (le_.start && !le_.used) {                                                                       \
            le_.used = true;                                                                                \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, le_.start, le_.stop, 0u, __VA_ARGS__);  \
        } else {                                                                                            \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                              \
        }                                                                                                   \
    } while (0)

namespace tpt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// 1/d from the hardware reciprocal and two Newton steps (about 1 ulp): the
// Thomas recurrence is a chain of dependent operations, so a short chain is
// what matters here (Thomas kernels).
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum (a, b) over the block in a fixed order; thread 0 gets the result.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            sa += red[2 * i];
            sb += red[2 * i + 1];
        }
        a = sa;
        b = sb;
    }
}

template <typename T>
__device__ __forceinline__ T load_as(const void* p, long long i, int dtype) {
    if (dtype == DT_F64) return (T)(((const double*)p)[i]);
    return (T)(((const float*)p)[i]);
}


// Round to nearest even to bf16 (inf / nan kept), and back.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_to_f(hi));
}
// The same split of two values at once by the hardware's packed conversion
// (round to nearest even, as bf16_rne for every finite value; a NaN or an
// infinity gives a NaN lo either way): element 0 in the low half of each word.
typedef float tpt_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 tpt_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
    const tpt_f32x2 v = {a, b};
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, tpt_bf16x2));
    const tpt_f32x2 r = {a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u)};
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, tpt_bf16x2));
}

// Blocks of one launch are dealt round-robin to the 8 XCDs, each with its own
// L2.  Renumbering block b of nb this way gives every XCD one contiguous range
// of logical blocks, so tiles that read the same operand rows (neighbouring
// logical blocks) share that XCD's L2 instead of fetching them once per XCD.
__device__ __forceinline__ long long xcd_block(long long b, long long nb) {
    const long long q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Upper bound on the grid of a persistent multi-problem launch.
constexpr long long PERSISTENT_BLOCKS = 2048;

}  // namespace tpt
