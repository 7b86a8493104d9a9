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
#include <algorithm>

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

// Column position of component c in the matrix-core layout: inside each block
// of 16 components the 4x4 sub-blocks are transposed, so that lane group g
// loading 4 consecutive floats at 4g feeds MFMA step m with component 4m + g.
__device__ __forceinline__ int mfma_col(int c) { return (c & ~15) | ((c & 3) << 2) | ((c >> 2) & 3); }

__global__ __launch_bounds__(256) void k_normalise(const float* __restrict__ sig, int64_t n, int k,
                                                   float* __restrict__ unit, uint16_t* __restrict__ bf16,
                                                   uint8_t* __restrict__ fp8, float* __restrict__ scale,
                                                   float* __restrict__ err, float* __restrict__ umfma,
                                                   int64_t n_pad, int kp) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (umfma && row >= n && row < n_pad) {
        for (int c = lane; c < kp; c += 64) umfma[row * kp + c] = 0.f;
        return;
    }
    if (row >= n) return;
    if (umfma) {
        for (int c = k + lane; c < kp; c += 64) umfma[row * kp + mfma_col(c)] = 0.f;
    }
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
        if (c < k && umfma) umfma[row * kp + mfma_col(c)] = v[r];
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

typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// One wavefront per 64x64 tile of the upper triangle. v_mfma_f32_16x16x4_f32
// computes acc = fmaf(a3, b3, fmaf(a2, b2, fmaf(a1, b1, fmaf(a0, b0, acc))))
// over its 4 k-values in lane-group order, so with the transposed 16-blocks of
// `u` (kp columns, rows padded to 64) each output is exactly the plain chain
// acc = fmaf(u_ic, u_jc, acc) over c = 0..k-1 ascending (zero columns past k
// leave it unchanged).
constexpr int kWT = 64;

// Per-wavefront LDS staging of flagged pairs: a wavefront appends pairs to its
// own buffer and reserves global output space with one atomic per flush.
constexpr int kStage = 512;

struct PairStage {
    mrc_pair* buf;  // LDS, kStage entries of this wavefront
    int n;          // staged entries (wavefront-uniform)

    __device__ __forceinline__ void flush(const PairSink& sink) {
        if (n == 0) return;
        const int lane = __lane_id();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(sink.counter, (unsigned long long)n);
        base = __shfl(base, 0, 64);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (int e = lane; e < n; e += 64) {
            const int64_t dst = (int64_t)base + e;
            if (dst < sink.capacity) sink.pairs[dst] = buf[e];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        n = 0;
    }

    // Append the pairs of one output slot across the wavefront (flag per lane).
    // The pair indices are only formed on this (rare) path.
    template <class IJ>
    __device__ __forceinline__ void add(const PairSink& sink, bool flag, IJ ij, float s, int flags) {
        const unsigned long long m = __ballot(flag);
        if (m == 0) return;
        const int cnt = __popcll(m);
        if (n + cnt > kStage) flush(sink);
        if (flag) {
            const int lane = __lane_id();
            const int r = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            int i, j;
            ij(&i, &j);
            buf[n + r] = mrc_pair{i, j, s, flags};
        }
        n += cnt;
    }
};

// Persistent wavefronts: workgroup p runs on XCD p % 8 and its wavefronts walk
// that XCD's contiguous share of the band-ordered tiles. Each tile is 64x64;
// the 16-column chunks are fully unrolled (NC even) and the first chunk of
// the next tile is loaded before the epilogue of the current one.
template <int NC>
__global__ __launch_bounds__(256) void k_compare_f32(const float* __restrict__ u, int n, int kp, float tau,
                                                     TileOrder ord, PairSink sink) {
    static_assert(NC % 2 == 0, "even chunk count");
    __shared__ mrc_pair stage_buf[4][kStage];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    PairStage st{stage_buf[wave], 0};
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    const int64_t stride = per_xcd_blocks * 4;
    int64_t t = t_lo + bx * 4 + wave;
    if (t >= t_hi) return;
    int bi, bj;
    ord.tile_at(t, &bi, &bj);
    const float* pa = u + (int64_t)(bi * kWT + li) * kp + 4 * lg;
    const float* pb = u + (int64_t)(bj * kWT + li) * kp + 4 * lg;
    f32x4 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        a[0][x] = *(const f32x4*)(pa + (int64_t)16 * x * kp);
        b[0][x] = *(const f32x4*)(pb + (int64_t)16 * x * kp);
    }
    while (true) {
        f32x4 acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int row0 = bi * kWT, col0 = bj * kWT;
        const int64_t tn = t + stride;
        const bool more = tn < t_hi;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cur = c & 1, nxt = cur ^ 1;
            if (c + 1 < NC) {
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x] = *(const f32x4*)(pa + (int64_t)16 * x * kp + 16 * (c + 1));
                    b[nxt][x] = *(const f32x4*)(pb + (int64_t)16 * x * kp + 16 * (c + 1));
                }
            } else if (more) {
                // first chunk of the next tile (NC even: it goes to buffer 0)
                int ni, nj;
                ord.tile_at(tn, &ni, &nj);
                pa = u + (int64_t)(ni * kWT + li) * kp + 4 * lg;
                pb = u + (int64_t)(nj * kWT + li) * kp + 4 * lg;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x] = *(const f32x4*)(pa + (int64_t)16 * x * kp);
                    b[nxt][x] = *(const f32x4*)(pb + (int64_t)16 * x * kp);
                }
                bi = ni;
                bj = nj;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cur][x][m], b[cur][y][m], acc[x][y], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        // epilogue: lane holds rows row0 + 16x + 4lg + r, column col0 + 16y + li
        const bool interior = row0 + kWT <= col0 && col0 + kWT <= n;
        const int ib = row0 + 4 * lg, jb = col0 + li;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = acc[x][y][r];
                    bool f = v >= tau;
                    if (!interior) {
                        const int i = ib + 16 * x + r, j = jb + 16 * y;
                        f = f && i < j && j < n;
                    }
                    st.add(sink, f, [&](int* i, int* j) { *i = ib + 16 * x + r; *j = jb + 16 * y; }, v, 0);
                }
        if (!more) break;
        t = tn;
    }
    st.flush(sink);
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

int mfma_chunks(int k);

mrc_status launch_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit,
                            uint16_t* bf16, uint8_t* fp8, float* scale, float* err, hipStream_t s,
                            float* umfma) {
    if (k > 64 * kMaxPerLane) return fail(MRC_E_INVAL, "k exceeds 1024");
    const int64_t n_pad = umfma ? ceil_div(n, 64) * 64 : n;
    const int kp = 16 * mfma_chunks(k);
    if (n_pad == 0) return MRC_OK;
    ScopedTimer tm(ctx, "normalise", s);
    hipLaunchKernelGGL(k_normalise, dim3((unsigned)ceil_div(n_pad, 4)), dim3(256), 0, s, sig, n, k, unit, bf16,
                       fp8, scale, err, umfma, n_pad, kp);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

int mfma_chunks(int k) {
    const int nc = (int)ceil_div(k, 16);
    for (int c : {2, 4, 6, 8, 12, 16, 24, 32, 48, 64})
        if (nc <= c) return c;
    return -1;
}

mrc_status launch_compare_f32(mrc_ctx* ctx, const float* umfma, int64_t n, int32_t k, float tau,
                              PairSink sink, hipStream_t s) {
    if (n < 2) return MRC_OK;
    TileOrder ord;
    int64_t grid = 0;
    MRC_TRY(make_tile_order(ctx, (int)ceil_div(n, kWT), 4, &ord, &grid, s));
    const int nc = mfma_chunks(k);
    const int kp = 16 * nc;
    ScopedTimer tm(ctx, "compare_f32", s);
    switch (nc) {
#define MRC_NC(c)                                                                                        \
    case c: {                                                                                            \
        const int64_t pgrid = persistent_grid(ctx, (const void*)k_compare_f32<c>, 256, grid);            \
        hipLaunchKernelGGL(k_compare_f32<c>, dim3((unsigned)pgrid), dim3(256), 0, s, umfma, (int)n, kp, tau, \
                           ord, sink);                                                                   \
    } break;
        MRC_NC(2) MRC_NC(4) MRC_NC(6) MRC_NC(8) MRC_NC(12) MRC_NC(16) MRC_NC(24) MRC_NC(32)
        MRC_NC(48) MRC_NC(64)
#undef MRC_NC
        default: return fail(MRC_E_INVAL, "k exceeds 1024");
    }
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
