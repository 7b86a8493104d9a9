// Exact fixed-point sums of a document's TF-IDF weights (device helpers shared
// by the signing passes).
//
// For idf in [1, 32), idf = m * 2^(E-23) with an integer mantissa m < 2^24, so
// (tf * idf)^2 * 2^46 = (tf * m)^2 * 2^(2E) is an integer; a 128-bit sum of
// these is exact for documents up to 2^22 tokens, and |w_d| is the square
// root of that sum rounded once to float64. The result does not depend on the
// order of summation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrc_exact {

typedef unsigned __int128 u128;

// tf * idf^2 * 2^46 (the contribution of one occurrence of a term with count tf)
__device__ __forceinline__ u128 occ_sq_fixed(uint32_t tf, float idf) {
    const uint32_t b = __float_as_uint(idf);
    const int E = (int)(b >> 23) - 127;  // 0 <= E <= 4 for idf in [1, 32)
    const uint64_t m = (b & 0x7FFFFFu) | 0x800000u;
    return ((u128)(m * m) * tf) << (2 * E);
}

// (tf * idf)^2 * 2^46 (the contribution of a distinct term with count tf)
__device__ __forceinline__ u128 term_sq_fixed(uint32_t tf, float idf) {
    const uint32_t b = __float_as_uint(idf);
    const int E = (int)(b >> 23) - 127;
    const uint64_t m = (b & 0x7FFFFFu) | 0x800000u;
    const uint64_t a = (uint64_t)tf * m;
    return ((u128)a * a) << (2 * E);
}

// Correctly rounded u128 -> double: the leading 64 bits with a sticky bit for
// the rest (below the rounding position), converted once.
__device__ __forceinline__ double u128_to_double(u128 v) {
    const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    if (hi == 0) return (double)lo;
    const int lz = __clzll((long long)hi);
    const uint64_t top = lz ? (hi << lz) | (lo >> (64 - lz)) : hi;
    const uint64_t rest = lz ? (lo << lz) : lo;
    return ldexp((double)(top | (rest != 0 ? 1ull : 0ull)), 64 - lz);
}

__device__ __forceinline__ double norm_from_fixed(u128 s) { return sqrt(u128_to_double(s) * 0x1p-46); }

__device__ __forceinline__ u128 wave_sum_u128(u128 v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t lo = __shfl_xor((unsigned long long)(uint64_t)v, off, 64);
        const uint64_t hi = __shfl_xor((unsigned long long)(uint64_t)(v >> 64), off, 64);
        v += ((u128)hi << 64) | lo;
    }
    return v;
}

// mantissa(x) << exponent(x) for a float 1 <= x < 32: x * 2^23, an integer
// below 2^28.
__device__ __forceinline__ uint32_t idf_scaled(float x) {
    const uint32_t b = __float_as_uint(x);
    return ((b & 0x7FFFFFu) | 0x800000u) << ((b >> 23) - 127u);
}

}  // namespace mrc_exact
