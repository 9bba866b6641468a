// Device helpers shared by the HIP kernels of libwfq.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wfq {

// Round a double to bfloat16 (nearest, ties to even) from its bits, so no intermediate float
// rounding can alter the result. Finite values in the normal range (or zero) only.
__device__ inline uint16_t bf16_rne(double v) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    uint64_t sign = b >> 63;
    int e = (int)((b >> 52) & 0x7ff);
    if (e == 0) return (uint16_t)(sign << 15);
    uint64_t mant = b & 0xfffffffffffffull;
    uint64_t keep = mant >> 45;
    uint64_t rest = mant & ((1ull << 45) - 1);
    const uint64_t half = 1ull << 44;
    uint32_t out = (uint32_t)(((uint64_t)(e - 1023 + 127) << 7) | keep);
    if (rest > half || (rest == half && (keep & 1))) out += 1;
    return (uint16_t)((sign << 15) | out);
}

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename E>
__device__ inline E cast_from_double(double v);
template <>
__device__ inline double cast_from_double<double>(double v) { return v; }
template <>
__device__ inline float cast_from_double<float>(double v) { return (float)v; }  // round to nearest even
template <>
__device__ inline uint16_t cast_from_double<uint16_t>(double v) { return bf16_rne(v); }

__device__ inline double widen(double v) { return v; }
__device__ inline double widen(float v) { return (double)v; }

// Sum over the 64 lanes of a wave; every lane receives the total. Fixed butterfly order, so the
// result does not depend on scheduling.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace wfq
