// Device code shared by the all-pairs kernels (FP32 plain path and the BF16 /
// FP8 candidate search): the 64x64 wavefront tiles over the band order, the
// compact flag epilogue with per-wavefront pair staging, and the
// low-precision candidate kernel (instantiated per precision in the files
// that launch it).
#pragma once

#include "common.h"

namespace {

using namespace mrc;

typedef float f32x4 __attribute__((ext_vector_type(4)));


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
};

// Epilogue of one 64x64 wavefront tile, half H (accumulator rows x = 2H, 2H+1).
// Lane (li, lg) holds acc[x][y][r] = score of row ib + 16x + r, column
// jb + 16y (ib = row0 + 4lg, jb = col0 + li). Each lane first builds a bitmask
// of its flagged slots (score >= thr, and i < j < n outside interior tiles);
// a wavefront scan of the counts gives every lane its output positions; lanes
// with flags park their 32 scores in LDS (scr) so that the flagged ones can be
// read back by slot index, and write their pairs to the stage (or, for more
// flags than the stage holds, straight to the output).
template <int H>
__device__ __forceinline__ void tile_half(const f32x4 (&acc)[4][4], float thr, bool interior, int ib, int jb,
                                          int n, float* __restrict__ scr, PairStage& st, const PairSink& sink) {
    const int lane = __lane_id();
    uint32_t m = 0;
#pragma unroll
    for (int xx = 0; xx < 2; ++xx)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                m |= (acc[2 * H + xx][y][r] >= thr ? 1u : 0u) << (xx * 16 + y * 4 + r);
    if (!interior) {
        uint32_t valid = 0;
#pragma nounroll
        for (int sl = 0; sl < 32; ++sl) {
            const int i = ib + 16 * (2 * H + (sl >> 4)) + (sl & 3), j = jb + 16 * ((sl >> 2) & 3);
            if (i < j && j < n) valid |= 1u << sl;
        }
        m &= valid;
    }
    const int cnt = __popc(m);
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    if (total == 0) return;
    if (m) {
#pragma unroll
        for (int xx = 0; xx < 2; ++xx)
#pragma unroll
            for (int y = 0; y < 4; ++y) *(f32x4*)(scr + ((xx * 4 + y) * 64 + lane) * 4) = acc[2 * H + xx][y];
    }
    if (st.n + total > kStage) st.flush(sink);
    const bool direct = total > kStage;
    int64_t pos;
    if (direct) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(sink.counter, (unsigned long long)total);
        pos = (int64_t)__shfl(base, 0, 64) + incl - cnt;
    } else {
        pos = st.n + incl - cnt;
        st.n += total;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    while (m) {
        const int sl = __ffs(m) - 1;
        m &= m - 1;
        const int xx = sl >> 4, y = (sl >> 2) & 3, r = sl & 3;
        const mrc_pair pr{ib + 16 * (2 * H + xx) + r, jb + 16 * y, scr[((xx * 4 + y) * 64 + lane) * 4 + r], 0};
        if (direct) {
            if (pos < sink.capacity) sink.pairs[pos] = pr;
        } else {
            st.buf[pos] = pr;
        }
        ++pos;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Whole epilogue of one 64x64 wavefront tile (lane layout as in tile_half). A
// tile whose largest score is below thr in every lane (the common case away
// from duplicates) ends after a max tree.
__device__ __forceinline__ void tile_epilogue(const f32x4 (&acc)[4][4], float thr, bool interior, int ib, int jb,
                                              int n, float* __restrict__ scr, PairStage& st, const PairSink& sink) {
    float mx[16];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            mx[x * 4 + y] = fmaxf(fmaxf(acc[x][y][0], acc[x][y][1]), fmaxf(acc[x][y][2], acc[x][y][3]));
#pragma unroll
    for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
        for (int i = 0; i < w; ++i) mx[i] = fmaxf(mx[i], mx[i + w]);
    if (__ballot(mx[0] >= thr) == 0) return;
    tile_half<0>(acc, thr, interior, ib, jb, n, scr, st, sink);
    tile_half<1>(acc, thr, interior, ib, jb, n, scr, st, sink);
}

// LDS of the all-pairs kernels (4 wavefronts): pair stages and score parking.
struct TileLds {
    mrc_pair stage[4][kStage];
    float scr[4][2048];
};

// ---------------------------------------------------------------- BF16 / FP8 forms

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Element width (bytes) and k per MFMA step of each low-precision form.
template <int PREC> struct LowpTraits;
template <> struct LowpTraits<MRC_PREC_BF16> { static constexpr int kStep = 32, kBytes = 2, kLaneBytes = 16; };
template <> struct LowpTraits<MRC_PREC_FP8> { static constexpr int kStep = 128, kBytes = 1, kLaneBytes = 32; };

// Operand fragment of one 16-row block for one MFMA step: lane (row li, group
// lg) holds kLaneBytes consecutive bytes of its row at k = c0 + lg * (kStep/4).
template <int PREC> struct Frag;
template <> struct Frag<MRC_PREC_BF16> {
    i32x4 v;
    __device__ __forceinline__ void load(const uint8_t* p) { v = *(const i32x4*)p; }
};
template <> struct Frag<MRC_PREC_FP8> {
    i32x4 lo, hi;
    __device__ __forceinline__ void load(const uint8_t* p) {
        lo = *(const i32x4*)p;
        hi = *(const i32x4*)(p + 16);
    }
};

__device__ __forceinline__ f32x4 mma(const Frag<MRC_PREC_BF16>& a, const Frag<MRC_PREC_BF16>& b, f32x4 c) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, &a.v, 16);
    __builtin_memcpy(&bv, &b.v, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mma(const Frag<MRC_PREC_FP8>& a, const Frag<MRC_PREC_FP8>& b, f32x4 c) {
    const i32x8 av = {a.lo[0], a.lo[1], a.lo[2], a.lo[3], a.hi[0], a.hi[1], a.hi[2], a.hi[3]};
    const i32x8 bv = {b.lo[0], b.lo[1], b.lo[2], b.lo[3], b.hi[0], b.hi[1], b.hi[2], b.hi[3]};
    // formats 0/0: both operands float8 e4m3; E8M0 block scales 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
}

// Candidate search of the low-precision forms: same persistent band-ordered
// 64x64 wavefront tiles as the FP32 path. A pair becomes a candidate when its
// low-precision score is >= lo_thr = tau - (the largest rescoring band over all
// rows); the rescoring kernel then decides each candidate exactly.
// q: [n_pad][ldq] bytes of codes (zero padded), scale: [n_pad] (FP8 only).
template <int PREC, int NK>
__global__ __launch_bounds__(256) void k_compare_lowp(const uint8_t* __restrict__ q, int ldq_bytes,
                                                      const float* __restrict__ scale, int n,
                                                      const float* __restrict__ lo_thr_ptr, TileOrder ord,
                                                      PairSink cand) {
    using T = LowpTraits<PREC>;
    static_assert(NK % 2 == 0, "even step count");
    __shared__ TileLds lds;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    PairStage st{lds.stage[wave], 0};
    float* scr = lds.scr[wave];
    const float lo_thr = *lo_thr_ptr;
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    const int64_t stride = per_xcd_blocks * 4;
    int64_t t = t_lo + bx * 4 + wave;
    if (t >= t_hi) return;
    TileOrder::Cursor cur = ord.seek(t);
    int bi, bj;
    ord.tile(cur, t, &bi, &bj);
    constexpr int kStepBytes = T::kStep * T::kBytes;
    const uint8_t* pa = q + (int64_t)(bi * kWT + li) * ldq_bytes + lg * T::kLaneBytes;
    const uint8_t* pb = q + (int64_t)(bj * kWT + li) * ldq_bytes + lg * T::kLaneBytes;
    Frag<PREC> a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        a[0][x].load(pa + (int64_t)16 * x * ldq_bytes);
        b[0][x].load(pb + (int64_t)16 * x * ldq_bytes);
    }
    while (true) {
        const int64_t tn = t + stride;
        const bool more = tn < t_hi;
        int ni = 0, nj = 0;
        if (more) ord.tile(cur, tn, &ni, &nj);
        f32x4 acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int row0 = bi * kWT, col0 = bj * kWT;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int cur_b = c & 1, nxt = cur_b ^ 1;
            if (c + 1 < NK) {
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x].load(pa + (int64_t)16 * x * ldq_bytes + kStepBytes * (c + 1));
                    b[nxt][x].load(pb + (int64_t)16 * x * ldq_bytes + kStepBytes * (c + 1));
                }
            } else if (more) {
                pa = q + (int64_t)(ni * kWT + li) * ldq_bytes + lg * T::kLaneBytes;
                pb = q + (int64_t)(nj * kWT + li) * ldq_bytes + lg * T::kLaneBytes;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x].load(pa + (int64_t)16 * x * ldq_bytes);
                    b[nxt][x].load(pb + (int64_t)16 * x * ldq_bytes);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = mma(a[cur_b][x], b[cur_b][y], acc[x][y]);
            __builtin_amdgcn_sched_barrier(0);
        }
        const bool interior = row0 + kWT <= col0 && col0 + kWT <= n;
        const int ib = row0 + 4 * lg, jb = col0 + li;
        if constexpr (PREC == MRC_PREC_FP8) {
            float cs[4];
#pragma unroll
            for (int y = 0; y < 4; ++y) cs[y] = scale[jb + 16 * y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float rs = scale[ib + 16 * x + r];
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y][r] = acc[x][y][r] * rs * cs[y];
                }
        }
        tile_epilogue(acc, lo_thr, interior, ib, jb, n, scr, st, cand);
        if (!more) break;
        t = tn;
        bi = ni;
        bj = nj;
    }
    st.flush(cand);
}


// Launch of the candidate kernel of one precision over the band-ordered tiles.
template <int PREC>
mrc_status launch_lowp_kernel(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, const float* scale, int64_t n, int nk,
                              const float* d_lo_thr, const TileOrder& ord, int64_t grid, PairSink cand,
                              hipStream_t s) {
#define MRC_LP(c)                                                                                        \
    case c: {                                                                                            \
        const int64_t pgrid = persistent_grid(ctx, (const void*)k_compare_lowp<PREC, c>, 256, grid);     \
        hipLaunchKernelGGL((k_compare_lowp<PREC, c>), dim3((unsigned)pgrid), dim3(256), 0, s, q, ldq_bytes, \
                           scale, (int)n, d_lo_thr, ord, cand);                                          \
    } break;
    if constexpr (PREC == MRC_PREC_BF16) {
        switch (nk) {
            MRC_LP(2) MRC_LP(4) MRC_LP(6) MRC_LP(8) MRC_LP(10) MRC_LP(12) MRC_LP(16) MRC_LP(20) MRC_LP(24) MRC_LP(32)
            default: return fail(MRC_E_INVAL, "unsupported k for the BF16 form");
        }
    } else {
        switch (nk) {
            MRC_LP(2) MRC_LP(4) MRC_LP(6) MRC_LP(8)
            default: return fail(MRC_E_INVAL, "unsupported k for the FP8 form");
        }
    }
#undef MRC_LP
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace
