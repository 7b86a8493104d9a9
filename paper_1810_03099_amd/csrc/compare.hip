// Signature comparison (Eq. 1 applied to two signatures; the similarity that
// Eq. 2 calls multi reference cosine).
//
//  * k_normalise_vec (k a multiple of 4; k_normalise otherwise): unit
//    signatures u = sig / |sig| (float32), their bfloat16 codes, float8
//    e4m3fn codes with a per-row power-of-two scale (the smallest one >=
//    max|u|/448, so that the matrix cores can apply it as an E8M0 operand
//    scale), and per-row error norms |u - dequantised| used to bound
//    low-precision scores.
//  * the plain FP32 path (allpairs_f32.hip) and the candidate search over the
//    BF16 / FP8 codes (lds_allpairs.hip) consume these layouts;
//  * launch_compare_lowp: the candidate search over the BF16 / FP8 codes
//    (LDS-tiled kernels of lds_allpairs.hip), emitting the candidates that
//    k_rescore then decides with the plain chain.
//  * k_score_pairs / k_rescore: the same chain for listed pairs.
#include <algorithm>

#include "allpairs.h"
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

using mrc_dev::mfma_col;

// Output layouts of k_normalise (NormLayout): leading dimensions let the comparison
// kernels use zero-padded internal copies (rows padded to n_pad, columns to ld).
using NormOut = NormLayout;

__global__ __launch_bounds__(256) void k_normalise(const float* __restrict__ sig, int64_t n, int k, NormOut o) {
    if (blockIdx.x == 0 && (int)threadIdx.x < o.n_clear) o.clear[threadIdx.x] = 0;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= o.n_pad) return;
    if (row >= n) {  // padding rows: zeros everywhere
        if (o.unit) for (int c = lane; c < o.ld_unit; c += 64) o.unit[row * o.ld_unit + c] = 0.f;
        if (o.bf16) for (int c = lane; c < o.ld_bf16; c += 64) o.bf16[row * o.ld_bf16 + c] = 0;
        if (o.fp8) for (int c = lane; c < o.ld_fp8; c += 64) o.fp8[row * o.ld_fp8 + c] = 0;
        if (o.umfma)
            for (int c = lane; c < o.ld_mfma; c += 64)
                o.umfma[o.frag ? frag_offset(row, c, o.ld_mfma / 16) : row * o.ld_mfma + c] = 0.f;
        if (lane == 0) {
            if (o.scale) o.scale[row] = 0.f;
            if (o.err) o.err[row] = o.err[o.ld_err + row] = 0.f;
        }
        return;
    }
    if (o.unit) for (int c = k + lane; c < o.ld_unit; c += 64) o.unit[row * o.ld_unit + c] = 0.f;
    if (o.bf16) for (int c = k + lane; c < o.ld_bf16; c += 64) o.bf16[row * o.ld_bf16 + c] = 0;
    if (o.fp8) for (int c = k + lane; c < o.ld_fp8; c += 64) o.fp8[row * o.ld_fp8 + c] = 0;
    if (o.umfma)
        for (int c = k + lane; c < o.ld_mfma; c += 64)
            o.umfma[o.frag ? frag_offset(row, c, o.ld_mfma / 16) : row * o.ld_mfma + mfma_col(c)] = 0.f;
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
        if (c < k && o.unit) o.unit[row * o.ld_unit + c] = v[r];
        if (c < k && o.umfma)
            o.umfma[o.frag ? frag_offset(row, c, o.ld_mfma / 16) : row * o.ld_mfma + mfma_col(c)] = v[r];
    }
    amax = mrc_dev::wave_max(amax);
    // smallest power of two >= amax / 448 (amax / 448 is a normal float: a
    // unit vector of k <= 1024 components has amax >= 2^-5)
    float sc = amax / 448.0f;
    if (__float_as_uint(sc) & 0x007FFFFFu) sc = __uint_as_float((__float_as_uint(sc) & 0x7F800000u) + 0x00800000u);
    double eb = 0.0, e8 = 0.0;
#pragma unroll
    for (int r = 0; r < kMaxPerLane; ++r) {
        const int c = lane + 64 * r;
        if (c >= k) continue;
        const uint16_t b = bf16_rne(v[r]);
        if (o.errs & 1) {
            const double db = (double)v[r] - (double)bf16_value(b);
            eb += db * db;
        }
        if (o.bf16) o.bf16[row * o.ld_bf16 + c] = b;
        const uint8_t q = sc > 0.f ? e4m3fn_rne(v[r] / sc) : (uint8_t)0;
        if (o.errs & 2) {
            const double d8 = (double)v[r] - (double)e4m3fn_value(q) * (double)sc;
            e8 += d8 * d8;
        }
        if (o.fp8) o.fp8[row * o.ld_fp8 + c] = q;
    }
    eb = mrc_dev::wave_sum(eb);
    e8 = mrc_dev::wave_sum(e8);
    if (lane == 0) {
        if (o.scale) o.scale[row] = sc;
        if (o.err) {
            // round the float64 norms up to float so the stored value bounds the error
            float fb = (float)sqrt(eb), f8 = (float)sqrt(e8);
            o.err[row] = (double)fb < sqrt(eb) ? nextafterf(fb, INFINITY) : fb;
            o.err[o.ld_err + row] = (double)f8 < sqrt(e8) ? nextafterf(f8, INFINITY) : f8;
        }
    }
}

// The same quantities for k a multiple of 4, with 16-byte row accesses: LPR
// lanes per row (64 / LPR rows per wavefront), lane li holding the float4
// groups c = 4 (li + LPR q), q < VPL, of its row. The results depend on k
// alone (not on which accesses can be vector ones: bit b of `wide` says the
// input (b = 0), unit (1), bf16 (2) and fp8 (3) rows are 16-, 8- or 4-byte
// aligned accordingly); they are those of k_normalise up to the summation
// order of |sig|^2.
template <int LPR>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <int LPR>
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

template <int LPR, int VPL>
__global__ __launch_bounds__(256) void k_normalise_vec(const float* __restrict__ sig, int64_t n, int k, NormOut o,
                                                       int wide) {
    if (blockIdx.x == 0 && (int)threadIdx.x < o.n_clear) o.clear[threadIdx.x] = 0;
    constexpr int RPW = 64 / LPR;
    const int lane = threadIdx.x & 63, li = lane % LPR;
    const int64_t row = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW + lane / LPR;
    const bool live = row < n;
    if (row >= o.n_pad) return;  // (whole row groups: the shuffles below stay within a group)
    const int nc = o.ld_mfma / 16;
    auto put_mfma = [&](int c, float x) {
        o.umfma[o.frag ? frag_offset(row, c, nc) : row * o.ld_mfma + mfma_col(c)] = x;
    };
    // padding columns [k, ld) (all columns of padding rows)
    const int c_pad = live ? k : 0;
    if (o.unit)
        for (int c = c_pad + li; c < o.ld_unit; c += LPR) o.unit[row * o.ld_unit + c] = 0.f;
    if (o.bf16)
        for (int c = c_pad + li; c < o.ld_bf16; c += LPR) o.bf16[row * o.ld_bf16 + c] = 0;
    if (o.fp8)
        for (int c = c_pad + li; c < o.ld_fp8; c += LPR) o.fp8[row * o.ld_fp8 + c] = 0;
    if (o.umfma)
        for (int c = c_pad + li; c < o.ld_mfma; c += LPR) put_mfma(c, 0.f);
    if (!live) {
        if (li == 0) {
            if (o.scale) o.scale[row] = 0.f;
            if (o.err) o.err[row] = o.err[o.ld_err + row] = 0.f;
        }
        return;
    }
    const float* x = sig + row * k;
    float4 v[VPL];
    float s2 = 0.f;
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
        const int c = 4 * (li + LPR * q);
        if (c >= k) v[q] = float4{0.f, 0.f, 0.f, 0.f};
        else if (wide & 1) v[q] = *(const float4*)(x + c);
        else v[q] = float4{x[c], x[c + 1], x[c + 2], x[c + 3]};
        s2 = fmaf(v[q].x, v[q].x, s2);
        s2 = fmaf(v[q].y, v[q].y, s2);
        s2 = fmaf(v[q].z, v[q].z, s2);
        s2 = fmaf(v[q].w, v[q].w, s2);
    }
    const float nrm = sqrtf(group_sum<LPR>(s2));
    float amax = 0.f;
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
        const int c = 4 * (li + LPR * q);
        v[q].x = nrm > 0.f ? v[q].x / nrm : 0.f;
        v[q].y = nrm > 0.f ? v[q].y / nrm : 0.f;
        v[q].z = nrm > 0.f ? v[q].z / nrm : 0.f;
        v[q].w = nrm > 0.f ? v[q].w / nrm : 0.f;
        amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v[q].x), fabsf(v[q].y)), fmaxf(fabsf(v[q].z), fabsf(v[q].w))));
        if (c < k) {
            if (o.unit) {
                float* pu = o.unit + row * o.ld_unit + c;
                if (wide & 2) {
                    *(float4*)pu = v[q];
                } else {
                    pu[0] = v[q].x, pu[1] = v[q].y, pu[2] = v[q].z, pu[3] = v[q].w;
                }
            }
            if (o.umfma) {
                put_mfma(c, v[q].x);
                put_mfma(c + 1, v[q].y);
                put_mfma(c + 2, v[q].z);
                put_mfma(c + 3, v[q].w);
            }
        }
    }
    amax = group_max<LPR>(amax);
    // smallest power of two >= amax / 448 (see k_normalise); dividing by it is
    // multiplying by its exact reciprocal
    float sc = amax / 448.0f;
    if (__float_as_uint(sc) & 0x007FFFFFu) sc = __uint_as_float((__float_as_uint(sc) & 0x7F800000u) + 0x00800000u);
    const float inv_sc = sc > 0.f ? 1.0f / sc : 0.f;
    double eb = 0.0, e8 = 0.0;
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
        const int c = 4 * (li + LPR * q);
        if (c >= k) continue;
        const float u4[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
        uint16_t b[4];
        uint8_t f8[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b[j] = bf16_rne(u4[j]);
            if (o.errs & 1) {
                const double db = (double)u4[j] - (double)bf16_value(b[j]);
                eb += db * db;
            }
            f8[j] = (o.fp8 || (o.errs & 2)) && sc > 0.f ? e4m3fn_rne(u4[j] * inv_sc) : (uint8_t)0;
            if (o.errs & 2) {
                const double d8 = (double)u4[j] - (double)e4m3fn_value(f8[j]) * (double)sc;
                e8 += d8 * d8;
            }
        }
        if (o.bf16) {
            uint16_t* pb = o.bf16 + row * o.ld_bf16 + c;
            if (wide & 4)
                *(uint2*)pb = uint2{(uint32_t)b[0] | ((uint32_t)b[1] << 16), (uint32_t)b[2] | ((uint32_t)b[3] << 16)};
            else
                for (int j = 0; j < 4; ++j) pb[j] = b[j];
        }
        if (o.fp8) {
            uint8_t* p8 = o.fp8 + row * o.ld_fp8 + c;
            if (wide & 8)
                *(uint32_t*)p8 =
                    (uint32_t)f8[0] | ((uint32_t)f8[1] << 8) | ((uint32_t)f8[2] << 16) | ((uint32_t)f8[3] << 24);
            else
                for (int j = 0; j < 4; ++j) p8[j] = f8[j];
        }
    }
    eb = group_sum<LPR>(eb);
    e8 = group_sum<LPR>(e8);
    if (li == 0) {
        if (o.scale) o.scale[row] = sc;
        if (o.err) {
            float fb = (float)sqrt(eb), f8 = (float)sqrt(e8);
            o.err[row] = (double)fb < sqrt(eb) ? nextafterf(fb, INFINITY) : fb;
            o.err[o.ld_err + row] = (double)f8 < sqrt(e8) ? nextafterf(f8, INFINITY) : f8;
        }
    }
}

// lo_thr = tau - max(nominal, band(e_max, e_max)) with e_max the largest row error.
__device__ __forceinline__ float lowp_band(float ei, float ej, float nominal, float acc_unit) {
    const float b = ei + ej + ei * ej + acc_unit * (1.f + ei) * (1.f + ej) + 9.5367431640625e-07f;  // + 2^-20
    return fmaxf(nominal, b);
}

// lo_thr in two steps: the largest row error (blocks over the rows, one
// atomic max of the float bits per wavefront into a zeroed word), then the band.
__global__ __launch_bounds__(256) void k_lowp_errmax(const float* __restrict__ err, int64_t n,
                                                     unsigned int* __restrict__ emax) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmaxf(m, err[i]);
    m = mrc_dev::wave_max(m);
    if ((threadIdx.x & 63) == 0) atomicMax(emax, __float_as_uint(m));  // non-negative floats order like their bits
}

// Largest row error of each 32-row block (0 for rows past n).
__global__ __launch_bounds__(256) void k_block_errmax(const float* __restrict__ err, int64_t n, int64_t nblk,
                                                      float* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= nblk) return;
    float m = 0.f;
    for (int64_t r = 32 * b; r < 32 * b + 32 && r < n; ++r) m = fmaxf(m, err[r]);
    out[b] = m;
}

__global__ void k_lowp_threshold(const unsigned int* __restrict__ emax, float tau, float nominal, float acc_unit,
                                 float* __restrict__ out) {
    const float e = __uint_as_float(*emax);
    out[0] = tau - lowp_band(e, e, nominal, acc_unit);
}

// Rescoring: every candidate with |s_lp - tau| <= band(e_i, e_j) gets the plain
// FP32 chain score over the natural-order unit signatures; outside the band
// the low-precision decision is already certain. Decided pairs are staged per
// workgroup in LDS and reserved in the output with one atomic per workgroup.
// stats: [0] rescored, [1] rescored within nominal, [2] flips outside nominal,
// [3] max |s_lp - s32| (float bits), [4] sum |s_lp - s32| (double bits).
constexpr int kRescoreChunk = 256;  // one candidate per thread and pass

// The plain chain of two natural-order rows; `wide` (the caller's rows are
// 16-byte aligned: k a multiple of 4 and an aligned base) reads 16 components
// per round trip, in the same ascending order as the scalar loop.
__device__ __forceinline__ float chain_rows(const float* __restrict__ a, const float* __restrict__ b, int k, bool wide) {
    float acc = 0.f;
    if (wide) {
        for (int c0 = 0; c0 < k; c0 += 16) {
            float4 va[4], vb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c0 + 4 * j < k) {
                    va[j] = *(const float4*)(a + c0 + 4 * j);
                    vb[j] = *(const float4*)(b + c0 + 4 * j);
                }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c0 + 4 * j < k) {
                    acc = __builtin_fmaf(va[j].x, vb[j].x, acc);
                    acc = __builtin_fmaf(va[j].y, vb[j].y, acc);
                    acc = __builtin_fmaf(va[j].z, vb[j].z, acc);
                    acc = __builtin_fmaf(va[j].w, vb[j].w, acc);
                }
        }
        return acc;
    }
    for (int cc = 0; cc < k; ++cc) acc = __builtin_fmaf(a[cc], b[cc], acc);
    return acc;
}

__global__ __launch_bounds__(256) void k_rescore(const mrc_pair* __restrict__ cand,
                                                 const unsigned long long* __restrict__ n_cand_ptr,
                                                 int64_t cand_cap, const float* __restrict__ unit, int k,
                                                 const float* __restrict__ err, float tau, float nominal,
                                                 float acc_unit, PairSink out,
                                                 unsigned long long* __restrict__ stats) {
    __shared__ mrc_pair sbuf[kRescoreChunk];
    __shared__ int scount;
    __shared__ unsigned long long sbase;
    __shared__ unsigned long long s_nb, s_nn, s_flip, s_max;
    __shared__ double s_sum;
    const int64_t nc = min((int64_t)*n_cand_ptr, cand_cap);
    if (threadIdx.x == 0) {
        s_nb = s_nn = s_flip = s_max = 0;
        s_sum = 0.0;
    }
    for (int64_t c0 = (int64_t)blockIdx.x * kRescoreChunk; c0 < nc; c0 += (int64_t)gridDim.x * kRescoreChunk) {
        if (threadIdx.x == 0) scount = 0;
        __syncthreads();
        const int64_t c1 = min(nc, c0 + kRescoreChunk);
        for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
            const mrc_pair p = cand[c];
            const float ei = err[p.i], ej = err[p.j];
            const float band = lowp_band(ei, ej, nominal, acc_unit);
            float s = p.s;
            int flags = 0;
            bool keep;
            if (p.s >= tau + band) {
                keep = true;
            } else if (p.s < tau - band) {
                keep = false;
            } else {
                const float acc = chain_rows(unit + (int64_t)p.i * k, unit + (int64_t)p.j * k, k, (k & 3) == 0);
                keep = acc >= tau;
                const float d = fabsf(p.s - acc);
                atomicAdd(&s_nb, 1ull);
                if (fabsf(p.s - tau) <= nominal) atomicAdd(&s_nn, 1ull);
                else if ((p.s >= tau) != keep) atomicAdd(&s_flip, 1ull);
                atomicMax(&s_max, (unsigned long long)__float_as_uint(d));
                atomicAdd(&s_sum, (double)d);
                s = acc;
                flags = 1;
            }
            if (keep) sbuf[atomicAdd(&scount, 1)] = mrc_pair{p.i, p.j, s, flags};
        }
        __syncthreads();
        const int cnt = scount;
        if (threadIdx.x == 0 && cnt > 0) sbase = atomicAdd(out.counter, (unsigned long long)cnt);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += 256) {
            const int64_t dst = (int64_t)sbase + e;
            if (dst < out.capacity) out.pairs[dst] = sbuf[e];
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_nb) atomicAdd(&stats[0], s_nb);
        if (s_nn) atomicAdd(&stats[1], s_nn);
        if (s_flip) atomicAdd(&stats[2], s_flip);
        if (s_max) atomicMax(&stats[3], s_max);
        if (s_sum != 0.0) atomicAdd((double*)&stats[4], s_sum);
    }
}

// Plain score of listed pairs (one thread per pair, same chain).
__global__ void k_score_pairs(const float* __restrict__ u, int k, const int32_t* __restrict__ ii,
                              const int32_t* __restrict__ jj, int64_t np, float* __restrict__ out, bool wide) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    out[p] = chain_rows(u + (int64_t)ii[p] * k, u + (int64_t)jj[p] * k, k, wide);
}

}  // namespace

namespace mrc {

int mfma_chunks(int k);

mrc_status launch_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit,
                            uint16_t* bf16, uint8_t* fp8, float* scale, float* err, hipStream_t s,
                            float* umfma, int64_t* clear, int n_clear) {
    if (k > 64 * kMaxPerLane) return fail(MRC_E_INVAL, "k exceeds 1024");
    NormOut o{unit, k, bf16, k, fp8, k, scale, err, n, umfma, 16 * mfma_chunks(k), n, 1};
    o.clear = clear;
    o.n_clear = n_clear;
    if (umfma) o.n_pad = ceil_div(n, 128) * 128;  // the FP32 kernel's 128-row tiles
    return launch_normalise_rows(ctx, sig, n, k, o, s);
}

mrc_status launch_normalise_rows(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, const NormLayout& o,
                                 hipStream_t s) {
    if (k > 64 * kMaxPerLane) return fail(MRC_E_INVAL, "k exceeds 1024");
    if (o.n_clear > 256) return fail(MRC_E_INVAL, "normalise: at most 256 words to clear");
    if (o.n_pad == 0) return o.n_clear > 0 ? clear_words(ctx, o.clear, o.n_clear, s) : MRC_OK;
    ScopedTimer tm(ctx, "normalise", s);
    // k a multiple of 4: four components per lane, vector accesses where the
    // rows are aligned for them (the results do not depend on which)
    auto al = [](const void* p, unsigned a) { return ((uintptr_t)p & (a - 1)) == 0; };
    const int wide = (al(sig, 16) ? 1 : 0) | (o.unit && al(o.unit, 16) && o.ld_unit % 4 == 0 ? 2 : 0) |
                     (o.bf16 && al(o.bf16, 8) && o.ld_bf16 % 4 == 0 ? 4 : 0) |
                     (o.fp8 && al(o.fp8, 4) && o.ld_fp8 % 4 == 0 ? 8 : 0);
    if (k % 4 == 0) {
        int lpr = 4;
        while (lpr < 64 && 4 * lpr < k) lpr *= 2;
        const int vpl = (int)ceil_div(k, 4 * lpr);
        const int64_t rows_per_block = 4 * (64 / lpr);
        const dim3 grid((unsigned)ceil_div(o.n_pad, rows_per_block));
        switch (lpr * 8 + vpl) {
#define MRC_NV(L, V)                                                                              \
    case L * 8 + V:                                                                               \
        hipLaunchKernelGGL((k_normalise_vec<L, V>), grid, dim3(256), 0, s, sig, n, k, o, wide);   \
        break;
            MRC_NV(4, 1) MRC_NV(8, 1) MRC_NV(16, 1) MRC_NV(32, 1) MRC_NV(64, 1) MRC_NV(64, 2) MRC_NV(64, 3)
            MRC_NV(64, 4)
#undef MRC_NV
            default: return fail(MRC_E_INVAL, "normalise: no row shape for this k");
        }
    } else {
        hipLaunchKernelGGL(k_normalise, dim3((unsigned)ceil_div(o.n_pad, 4)), dim3(256), 0, s, sig, n, k, o);
    }
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

__global__ __launch_bounds__(256) void k_err_max(const float* __restrict__ e16, const float* __restrict__ e8,
                                                 int64_t n, float* __restrict__ errmax) {
    float m16 = 0.f, m8 = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        m16 = fmaxf(m16, e16[i]);
        m8 = fmaxf(m8, e8[i]);
    }
    m16 = mrc_dev::wave_max(m16);
    m8 = mrc_dev::wave_max(m8);
    // non-negative floats order like their bit patterns
    if ((threadIdx.x & 63) == 0) {
        atomicMax((unsigned int*)&errmax[0], __float_as_uint(m16));
        atomicMax((unsigned int*)&errmax[1], __float_as_uint(m8));
    }
}

mrc_status launch_err_max(mrc_ctx* ctx, const float* e16, const float* e8, int64_t n, float* errmax, hipStream_t s) {
    if (n <= 0) return MRC_OK;
    hipLaunchKernelGGL(k_err_max, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, s, e16, e8,
                       n, errmax);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

int mfma_chunks(int k) {
    const int nc = (int)ceil_div(k, 16);
    for (int c : {2, 4, 6, 8, 12, 16, 24, 32, 48, 64})
        if (nc <= c) return c;
    return -1;
}

int lowp_steps(int precision, int k) {
    const int step = precision == MRC_PREC_BF16 ? 32 : 128;
    int nk = (int)ceil_div(k, step);
    nk += nk & 1;  // even step count
    return nk;
}

mrc_status launch_compare_lowp(mrc_ctx* ctx, int32_t precision, const uint8_t* q, int ldq_bytes,
                               const float* scale, int64_t n, int32_t k, const float* d_lo_thr,
                               const float* err, float tau, float nominal, PairSink cand, hipStream_t s) {
    if (n < 2) return MRC_OK;
    if (precision == MRC_PREC_BF16) {
        ScopedTimer tm(ctx, "compare_lowp", s);
        return launch_compare_bf16(ctx, q, ldq_bytes, n, d_lo_thr, cand, s);
    }
    // 32-row blocks of the 256-row padded codes; the margin (2^-16) covers the
    // FP32 rounding of both threshold formulas (a few 1e-7 at most)
    const int64_t nblk = ceil_div(n, 256) * 8;
    void* be = nullptr;
    MRC_TRY(scratch(ctx, "lp_blk_err", (size_t)nblk * sizeof(float), &be));
    hipLaunchKernelGGL(k_block_errmax, dim3((unsigned)ceil_div(nblk, 256)), dim3(256), 0, s, err, n, nblk,
                       (float*)be);
    MRC_HIP_TRY(ctx, hipGetLastError());
    const double margin = 1.52587890625e-05;
    const BlockBand bb{(const float*)be, (float)((double)tau + 1.0 - 9.5367431640625e-07 - margin),
                       (float)((double)tau - (double)nominal - margin), 1.f + lowp_acc_unit(precision, k)};
    ScopedTimer tm(ctx, "compare_lowp", s);
    return launch_compare_fp8(ctx, q, ldq_bytes, scale, n, d_lo_thr, bb, cand, s);
}

// Accumulation slack of a low-precision score relative to |a_i||a_j|. BF16
// products are exact and the matrix cores accumulate them like FP32 adds
// (measured deviations of a few FP32 ulps): 3k * 2^-24. The FP8 matrix-core
// path accumulates with a shorter significand (measured up to ~2^-15
// relative on the signature workloads); the slack used is 2^-10.
float lowp_acc_unit(int precision, int k) {
    const double bf = 3.0 * k * 5.9604644775390625e-08;
    return (float)(precision == MRC_PREC_FP8 ? std::max(bf, 9.765625e-04) : bf);
}

mrc_status launch_lowp_threshold(mrc_ctx* ctx, int precision, const float* err, int64_t n, float tau,
                                 float nominal, int k, unsigned int* d_emax, float* d_out, hipStream_t s) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 1024));
    hipLaunchKernelGGL(k_lowp_errmax, dim3((unsigned)blocks), dim3(256), 0, s, err, n, d_emax);
    hipLaunchKernelGGL(k_lowp_threshold, dim3(1), dim3(1), 0, s, (const unsigned int*)d_emax, tau, nominal,
                       lowp_acc_unit(precision, k), d_out);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_rescore2(mrc_ctx* ctx, int precision, const mrc_pair* cand, const unsigned long long* n_cand,
                           int64_t cand_cap, const float* unit, int32_t k, const float* err, float tau, float nominal,
                           PairSink out, unsigned long long* stats, hipStream_t s) {
    ScopedTimer tm(ctx, "rescore", s);
    hipLaunchKernelGGL(k_rescore, dim3(1024), dim3(256), 0, s, cand, n_cand, cand_cap, unit, k, err, tau, nominal,
                       lowp_acc_unit(precision, k), out, stats);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_score_pairs(mrc_ctx* ctx, const float* unit, int32_t k, const int32_t* ii,
                              const int32_t* jj, int64_t n_pairs, float* out, hipStream_t s) {
    if (n_pairs == 0) return MRC_OK;
    const bool wide = (k & 3) == 0 && ((uintptr_t)unit & 15) == 0;
    hipLaunchKernelGGL(k_score_pairs, dim3((unsigned)ceil_div(n_pairs, 256)), dim3(256), 0, s, unit, k, ii, jj,
                       n_pairs, out, wide);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
