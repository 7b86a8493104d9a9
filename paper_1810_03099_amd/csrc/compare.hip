// Signature comparison (Eq. 1 applied to two signatures; the similarity that
// Eq. 2 calls multi reference cosine).
//
//  * k_normalise: unit signatures u = sig / |sig| (float32), their bfloat16
//    codes, float8 e4m3fn codes with a per-row scale max|u|/448, and per-row
//    error norms |u - dequantised| used to bound low-precision scores.
//  * k_compare_f32: the plain path. Every pair i < j gets the score
//    acc = 0; acc = fmaf(u_ic, u_jc, acc), c = 0..k-1, on the vector ALUs,
//    register-tiled 8x8 per thread over a 128x128 tile, upper-triangle tiles
//    only; pairs with acc >= tau are appended to the output.
//  * k_score_pairs / k_rescore: the same chain for listed pairs.
#include "common.h"

using namespace mrc;

namespace {

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t c) { return __uint_as_float((uint32_t)c << 16); }

// float32 -> OCP float8 e4m3fn bits, round to nearest even. Magnitudes above
// 464 (which would round past 448) give NaN (0x7F), like a non-saturating
// conversion; the callers only pass |x| <= 448 * (1 + 2^-23).
__device__ __forceinline__ uint8_t e4m3fn_rne(float x) {
    const uint32_t sgn = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    uint32_t code;
    if (a < 0.015625f) {                        // below 2^-6: multiples of 2^-9
        code = (uint32_t)rintf(a * 512.0f);     // exact scaling, RNE; 8 -> 2^-6
    } else if (a > 464.0f) {
        code = 0x7Fu;
    } else {
        const uint32_t u = __float_as_uint(a);
        const uint32_t r = (u + 0x7FFFFu + ((u >> 20) & 1u)) >> 20;  // keep 3 mantissa bits
        code = r - ((127u - 7u) << 3);
        if (code > 0x7Eu) code = 0x7Eu;         // (448, 464] -> 448 unless tie-up to 480
        if (a == 464.0f) code = 0x7Eu;
    }
    return (uint8_t)(code | sgn);
}

__device__ __forceinline__ float e4m3fn_value(uint8_t c) {
    const uint32_t e = (c >> 3) & 15u, f = c & 7u;
    float mag = e == 0 ? (float)f * 0.001953125f : __uint_as_float(((e + 120u) << 23) | (f << 20));
    return (c & 0x80u) ? -mag : mag;
}

// One wavefront per row; k <= 64 * kMaxPerLane.
constexpr int kMaxPerLane = 16;

__global__ __launch_bounds__(256) void k_normalise(const float* __restrict__ sig, int64_t n, int k,
                                                   float* __restrict__ unit, uint16_t* __restrict__ bf16,
                                                   uint8_t* __restrict__ fp8, float* __restrict__ scale,
                                                   float* __restrict__ err) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float* x = sig + row * k;
    float v[kMaxPerLane];
    float s2 = 0.f;
#pragma unroll
    for (int r = 0; r < kMaxPerLane; ++r) {
        const int c = lane + 64 * r;
        v[r] = c < k ? x[c] : 0.f;
        s2 = fmaf(v[r], v[r], s2);
    }
    s2 = mrc_dev::wave_sum(s2);
    const float nrm = sqrtf(s2);
    float amax = 0.f;
#pragma unroll
    for (int r = 0; r < kMaxPerLane; ++r) {
        v[r] = nrm > 0.f ? v[r] / nrm : 0.f;
        amax = fmaxf(amax, fabsf(v[r]));
        const int c = lane + 64 * r;
        if (c < k && unit) unit[row * k + c] = v[r];
    }
    amax = mrc_dev::wave_max(amax);
    const float sc = amax / 448.0f;
    double eb = 0.0, e8 = 0.0;
#pragma unroll
    for (int r = 0; r < kMaxPerLane; ++r) {
        const int c = lane + 64 * r;
        if (c >= k) continue;
        const uint16_t b = bf16_rne(v[r]);
        const double db = (double)v[r] - (double)bf16_value(b);
        eb += db * db;
        if (bf16) bf16[row * k + c] = b;
        const uint8_t q = sc > 0.f ? e4m3fn_rne(v[r] / sc) : (uint8_t)0;
        const double d8 = (double)v[r] - (double)e4m3fn_value(q) * (double)sc;
        e8 += d8 * d8;
        if (fp8) fp8[row * k + c] = q;
    }
    eb = mrc_dev::wave_sum(eb);
    e8 = mrc_dev::wave_sum(e8);
    if (lane == 0) {
        if (scale) scale[row] = sc;
        if (err) {
            // round the float64 norms up to float so the stored value bounds the error
            float fb = (float)sqrt(eb), f8 = (float)sqrt(e8);
            err[row] = (double)fb < sqrt(eb) ? nextafterf(fb, INFINITY) : fb;
            err[n + row] = (double)f8 < sqrt(e8) ? nextafterf(f8, INFINITY) : f8;
        }
    }
}

// ---------------------------------------------------------------- FP32 plain path

constexpr int kT = 128;       // tile edge
constexpr int kKC = 32;       // k chunk staged in LDS
constexpr int kPad = 4;

__device__ __forceinline__ void tile_coords(int64_t t, int nb, int* bi, int* bj) {
    // Upper-triangle tiles (bi <= bj) in row-major order: row bi holds nb - bi tiles.
    // Invert t = bi*nb - bi*(bi-1)/2 + (bj - bi) with a float64 estimate and a fix-up.
    double a = 2.0 * nb + 1.0;
    int r = (int)((a - sqrt(a * a - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > nb - 1) r = nb - 1;
    auto start = [nb](int64_t row) { return row * nb - row * (row - 1) / 2; };
    while (r > 0 && start(r) > t) --r;
    while (r + 1 < nb && start(r + 1) <= t) ++r;
    *bi = r;
    *bj = r + (int)(t - start(r));
}

__global__ __launch_bounds__(256) void k_compare_f32(const float* __restrict__ u, int n, int k,
                                                     float tau, int nb, PairSink sink) {
    __shared__ float As[kKC][kT + kPad];
    __shared__ float Bs[kKC][kT + kPad];
    int bi, bj;
    tile_coords(blockIdx.x, nb, &bi, &bj);
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int row0 = bi * kT, col0 = bj * kT;
    float acc[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = 0.f;

    for (int c0 = 0; c0 < k; c0 += kKC) {
        // stage 128 rows x 32 columns of each operand, transposed to [c][row]
#pragma unroll
        for (int it = 0; it < (kT * kKC) / 256; ++it) {
            const int idx = it * 256 + tid;
            const int r = idx / kKC, c = idx % kKC;
            const int ga = row0 + r, gb = col0 + r, gc = c0 + c;
            As[c][r] = (ga < n && gc < k) ? u[(int64_t)ga * k + gc] : 0.f;
            Bs[c][r] = (gb < n && gc < k) ? u[(int64_t)gb * k + gc] : 0.f;
        }
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < kKC; ++c) {
            const float4 a0 = *(const float4*)&As[c][ty * 8];
            const float4 a1 = *(const float4*)&As[c][ty * 8 + 4];
            const float4 b0 = *(const float4*)&Bs[c][tx * 8];
            const float4 b1 = *(const float4*)&Bs[c][tx * 8 + 4];
            const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const float b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int x = 0; x < 8; ++x)
#pragma unroll
                for (int y = 0; y < 8; ++y) acc[x][y] = __builtin_fmaf(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
    // The zero padding past k adds fmaf(0, 0, acc) = acc steps: the chain is unchanged.
    int mine = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int i = row0 + ty * 8 + x;
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            const int j = col0 + tx * 8 + y;
            mine += (i < j && j < n && acc[x][y] >= tau) ? 1 : 0;
        }
    }
    int64_t idx = mrc_dev::wave_reserve(sink.counter, mine);
    if (mine == 0) return;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int i = row0 + ty * 8 + x;
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            const int j = col0 + tx * 8 + y;
            if (i < j && j < n && acc[x][y] >= tau) {
                if (idx < sink.capacity) sink.pairs[idx] = mrc_pair{i, j, acc[x][y], 0};
                ++idx;
            }
        }
    }
}

// Plain score of listed pairs (one thread per pair, same chain).
__global__ void k_score_pairs(const float* __restrict__ u, int k, const int32_t* __restrict__ ii,
                              const int32_t* __restrict__ jj, int64_t np, float* __restrict__ out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float* a = u + (int64_t)ii[p] * k;
    const float* b = u + (int64_t)jj[p] * k;
    float acc = 0.f;
    for (int c = 0; c < k; ++c) acc = __builtin_fmaf(a[c], b[c], acc);
    out[p] = acc;
}

}  // namespace

namespace mrc {

mrc_status launch_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit,
                            uint16_t* bf16, uint8_t* fp8, float* scale, float* err, hipStream_t s) {
    if (k > 64 * kMaxPerLane) return fail(MRC_E_INVAL, "k exceeds 1024");
    if (n == 0) return MRC_OK;
    ScopedTimer tm(ctx, "normalise", s);
    hipLaunchKernelGGL(k_normalise, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, s, sig, n, k, unit, bf16,
                       fp8, scale, err);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_compare_f32(mrc_ctx* ctx, const float* unit, int64_t n, int32_t k, float tau,
                              PairSink sink, hipStream_t s) {
    if (n < 2) return MRC_OK;
    const int nb = (int)ceil_div(n, kT);
    const int64_t tiles = (int64_t)nb * (nb + 1) / 2;
    if (tiles > 0x7FFFFFFFLL) return fail(MRC_E_INVAL, "too many tiles for one launch");
    ScopedTimer tm(ctx, "compare_f32", s);
    hipLaunchKernelGGL(k_compare_f32, dim3((unsigned)tiles), dim3(256), 0, s, unit, (int)n, k, tau, nb, sink);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_score_pairs(mrc_ctx* ctx, const float* unit, int32_t k, const int32_t* ii,
                              const int32_t* jj, int64_t n_pairs, float* out, hipStream_t s) {
    if (n_pairs == 0) return MRC_OK;
    hipLaunchKernelGGL(k_score_pairs, dim3((unsigned)ceil_div(n_pairs, 256)), dim3(256), 0, s, unit, k, ii, jj,
                       n_pairs, out);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
