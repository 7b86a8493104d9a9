// Device code shared by the all-pairs kernels (FP32 plain path and the BF16 /
// FP8 candidate search): the 64x64 wavefront tiles of the FP32 path over the
// band order, its compact flag epilogue, the per-wavefront pair staging, and
// the operand vector types of the low-precision matrix-core steps.
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

// (the buffer is typed as LDS: through a generic pointer its stores would be
// FLAT operations, after which the compiler can only wait for all memory
// operations in flight)
// (16-byte pairs held as a builtin 4-int vector, which stores to LDS directly)
typedef int pair_bits __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) pair_bits lds_pair;
static_assert(sizeof(mrc_pair) == sizeof(pair_bits), "a pair is 16 bytes");
__device__ __forceinline__ void stage_put(lds_pair* buf, int pos, const mrc_pair& p) {
    pair_bits v;
    __builtin_memcpy(&v, &p, sizeof v);
    buf[pos] = v;
}
__device__ __forceinline__ mrc_pair stage_get(const lds_pair* buf, int pos) {
    const pair_bits v = buf[pos];
    mrc_pair p;
    __builtin_memcpy(&p, &v, sizeof p);
    return p;
}
struct PairStage {
    lds_pair* buf;  // LDS, kStage entries of this wavefront
    int n;          // staged entries (wavefront-uniform)
    __device__ PairStage(mrc_pair* lds_buf, int n0) : buf((lds_pair*)lds_buf), n(n0) {}

    __device__ __forceinline__ void flush(const PairSink& sink) {
        if (n == 0) return;
        const int lane = __lane_id();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(sink.counter, (unsigned long long)n);
        base = __shfl(base, 0, 64);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int e = lane; e < n; e += 64) {
            const int64_t dst = (int64_t)base + e;
            if (dst < sink.capacity) sink.pairs[dst] = stage_get(buf, e);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        n = 0;
    }
};

// Sum over the wavefront of a per-lane count below 64 (one ballot per bit).
__device__ __forceinline__ int wave_total6(int cnt) {
    int t = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) t += __popcll(__ballot((cnt >> b) & 1)) << b;
    return t;
}

// Output position of this lane in a round of writes: the lanes of `act` take
// consecutive positions from `base` in lane order.
__device__ __forceinline__ int64_t round_pos(int64_t base, uint64_t act) {
    return base + (int64_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
}

// Flag marks of one half of a 64x64 wavefront tile (accumulator rows x = 2H,
// 2H+1): bit xx*16 + y*4 + r is set when acc[2H+xx][y][r] >= thr. The sign of
// score - thr decides, which for finite values is the comparison itself (a
// difference is zero only for equal operands, and a flush to zero keeps its
// sign); a funnel shift moves each sign into the word, one instruction per
// score.
template <int H>
__device__ __forceinline__ uint32_t half_marks(const f32x4 (&acc)[4][4], float thr) {
    uint32_t below = 0;
#pragma unroll
    for (int b = 31; b >= 0; --b)
        below = __builtin_amdgcn_alignbit(below, __float_as_uint(acc[2 * H + (b >> 4)][(b >> 2) & 3][b & 3] - thr), 31);
    return ~below;
}

// Epilogue of one 64x64 wavefront tile, half H (accumulator rows x = 2H, 2H+1),
// from its marks m (half_marks). Lane (li, lg) holds acc[x][y][r] = score of
// row ib + 16x + r, column jb + 16y (ib = row0 + 4lg, jb = col0 + li). Outside
// interior tiles the marks keep only i < j < n. Lanes with flags park their
// 32 scores in LDS (scr) so that the flagged ones can be read back by slot
// index; the pairs go to the stage (or, for more flags than the stage holds,
// straight to the output) in rounds: each lane with marks left writes its
// lowest one, and a round's lanes take consecutive positions, so the stores
// of a round are contiguous.
template <int H>
__device__ __forceinline__ void tile_half(const f32x4 (&acc)[4][4], uint32_t m, bool interior, int ib, int jb,
                                          int n, float* __restrict__ scr, PairStage& st, const PairSink& sink) {
    const int lane = __lane_id();
    if (!interior) {
        uint32_t valid = 0;
#pragma nounroll
        for (int sl = 0; sl < 32; ++sl) {
            const int i = ib + 16 * (2 * H + (sl >> 4)) + (sl & 3), j = jb + 16 * ((sl >> 2) & 3);
            if (i < j && j < n) valid |= 1u << sl;
        }
        m &= valid;
    }
    const int total = wave_total6(__popc(m));
    if (total == 0) return;
    if (m) {
#pragma unroll
        for (int xx = 0; xx < 2; ++xx)
#pragma unroll
            for (int y = 0; y < 4; ++y) *(f32x4*)(scr + ((xx * 4 + y) * 64 + lane) * 4) = acc[2 * H + xx][y];
    }
    if (st.n + total > kStage) st.flush(sink);
    const bool direct = total > kStage;
    int64_t base;
    if (direct) {
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(sink.counter, (unsigned long long)total);
        base = (int64_t)__shfl(b, 0, 64);
    } else {
        base = st.n;
        st.n += total;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    while (true) {
        const uint64_t act = __ballot(m != 0);
        if (act == 0) break;
        if (m) {
            const int sl = __ffs(m) - 1;
            m &= m - 1;
            const int xx = sl >> 4, y = (sl >> 2) & 3, r = sl & 3;
            const mrc_pair pr{ib + 16 * (2 * H + xx) + r, jb + 16 * y, scr[((xx * 4 + y) * 64 + lane) * 4 + r], 0};
            const int64_t pos = round_pos(base, act);
            if (direct) {
                if (pos < sink.capacity) sink.pairs[pos] = pr;
            } else {
                stage_put(st.buf, (int)pos, pr);
            }
        }
        base += __popcll(act);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Whole epilogue of one 64x64 wavefront tile (lane layout as in tile_half):
// both halves' marks first, so that a tile with no score >= thr in any lane
// (the common case away from duplicates) ends after one ballot.
__device__ __forceinline__ void tile_epilogue(const f32x4 (&acc)[4][4], float thr, bool interior, int ib, int jb,
                                              int n, float* __restrict__ scr, PairStage& st, const PairSink& sink) {
    const uint32_t m0 = half_marks<0>(acc, thr), m1 = half_marks<1>(acc, thr);
    if (__ballot((m0 | m1) != 0) == 0) return;
    tile_half<0>(acc, m0, interior, ib, jb, n, scr, st, sink);
    tile_half<1>(acc, m1, interior, ib, jb, n, scr, st, sink);
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

}  // namespace
