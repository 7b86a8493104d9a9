// BF16 candidate search of the all-pairs comparison, LDS-tiled.
//
// Each workgroup (4 wavefronts, one per SIMD: matrix-core streams of several
// wavefronts on one SIMD run slower than one) computes 256x256 blocks of the
// upper triangle of Q Q^T (Q: bfloat16 codes of the unit signatures, rows
// padded to a multiple of 256 with zeros); wavefront (wr, wc) owns the 128x128
// quarter at rows 128wr, columns 128wc, as 4x4 blocks of 32x32x16 matrix-core
// products accumulating in FP32. Operands pass through LDS in chunks of 32
// components (64-byte rows whose four 16-byte parts are XOR-swizzled by
// (row / 4) % 4, so that both the coalesced chunk stores and the 16-byte
// fragment reads of 16 consecutive rows hit distinct banks), double-buffered,
// with the next chunk loaded into registers while the current one is
// multiplied. Every score is
// compared with the candidate threshold; blocks without any score at or above
// it end after a max tree.
//
// 32x32x16 operand / result layouts (lane l): A fragment = row l % 32,
// components 8 (l / 32) .. +8 of the 16-component step (B the same with
// columns); result value i of the block = row 8 (i / 4) + 4 (l / 32) + i % 4,
// column l % 32.
#include "allpairs.h"
#include "common.h"

using namespace mrc;

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 256;          // workgroup tile (rows = columns)
constexpr int kKC = 32;           // components per LDS chunk
constexpr int kLdsRow = 32;       // LDS row stride in bfloat16 (64 bytes, parts swizzled)
constexpr int kBufElems = kBM * kLdsRow;

struct Bf16Lds {
    uint16_t a[2][kBufElems];
    uint16_t b[2][kBufElems];
    mrc_pair stage[4][kStage];
    float scr[4][16 * 64];
};

// Chunk kc (32 components) of the 256-row panels at rows ra / rb: this
// thread's 4 + 4 segments of 16 bytes (segment s = t + 256 e: row s / 4,
// part s % 4).
struct ChunkRegs {
    u32x4 a[4], b[4];
};

__device__ __forceinline__ void load_chunk(ChunkRegs& g, const uint8_t* __restrict__ q, int ldq_bytes, int64_t ra,
                                           int64_t rb, int kc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = threadIdx.x + 256 * e, row = s >> 2, part = s & 3;
        const int64_t off = (int64_t)kc * kKC * 2 + part * 16;
        g.a[e] = *(const u32x4*)(q + (ra + row) * ldq_bytes + off);
        g.b[e] = *(const u32x4*)(q + (rb + row) * ldq_bytes + off);
    }
}

__device__ __forceinline__ void store_chunk(const ChunkRegs& g, uint16_t* __restrict__ la, uint16_t* __restrict__ lb) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = threadIdx.x + 256 * e, row = s >> 2, part = s & 3;
        const int pos = row * kLdsRow + ((part ^ ((row >> 2) & 3)) * 8);
        *(u32x4*)(la + pos) = g.a[e];
        *(u32x4*)(lb + pos) = g.b[e];
    }
}

// Stage the flagged entries of one result slot across the wavefront.
__device__ __forceinline__ void stage_add(PairStage& st, const PairSink& sink, bool flag, int i, int j, float s) {
    const unsigned long long m = __ballot(flag);
    if (m == 0) return;
    const int cnt = __popcll(m);
    if (st.n + cnt > kStage) st.flush(sink);
    if (flag) {
        const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        st.buf[st.n + r] = mrc_pair{i, j, s, 0};
    }
    st.n += cnt;
}

template <int NKC>
__global__ __launch_bounds__(256, 1) void k_compare_bf16(const uint8_t* __restrict__ q, int ldq_bytes, int n,
                                                         const float* __restrict__ lo_thr_ptr, TileOrder ord,
                                                         PairSink cand) {
    static_assert(NKC % 2 == 0, "even chunk count");
    __shared__ Bf16Lds lds;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    PairStage st{lds.stage[wave], 0};
    float* scr = lds.scr[wave];
    const float thr = *lo_thr_ptr;
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    int64_t t = t_lo + bx;
    if (t >= t_hi) return;
    TileOrder::Cursor cur = ord.seek(t);
    int bi, bj;
    ord.tile(cur, t, &bi, &bj);
    ChunkRegs g;
    load_chunk(g, q, ldq_bytes, (int64_t)bi * kBM, (int64_t)bj * kBM, 0);
    store_chunk(g, lds.a[0], lds.b[0]);
    __syncthreads();
    // fragment reads: row (l % 32) of each 32-row block, part 2s + l / 32 of
    // step s, at its swizzled position (blocks start at multiples of 32 rows,
    // so the swizzle depends on l % 32 only)
    const int frow = lane & 31, swz = (frow >> 2) & 3;
    const int fpart0 = ((0 + (lane >> 5)) ^ swz) * 8, fpart1 = ((2 + (lane >> 5)) ^ swz) * 8;
    while (true) {
        const int64_t tn = t + per_xcd_blocks;
        const bool more = tn < t_hi;
        int ni = bi, nj = bj;
        if (more) ord.tile(cur, tn, &ni, &nj);
        f32x16 acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = f32x16{};
        for (int kc = 0; kc < NKC; ++kc) {
            const int cb = kc & 1;
            // next chunk of this block pair, or the first chunk of the next one
            if (kc + 1 < NKC) load_chunk(g, q, ldq_bytes, (int64_t)bi * kBM, (int64_t)bj * kBM, kc + 1);
            else if (more) load_chunk(g, q, ldq_bytes, (int64_t)ni * kBM, (int64_t)nj * kBM, 0);
            const uint16_t* la = lds.a[cb] + (wr * 128 + frow) * kLdsRow;
            const uint16_t* lb = lds.b[cb] + (wc * 128 + frow) * kLdsRow;
#pragma unroll
            for (int s = 0; s < kKC / 16; ++s) {
                const int fp = s == 0 ? fpart0 : fpart1;
                bf16x8 fa[4], fb[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const u32x4 va = *(const u32x4*)(la + x * 32 * kLdsRow + fp);
                    const u32x4 vb = *(const u32x4*)(lb + x * 32 * kLdsRow + fp);
                    __builtin_memcpy(&fa[x], &va, 16);
                    __builtin_memcpy(&fb[x], &vb, 16);
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fb[y], acc[x][y], 0, 0, 0);
            }
            if (kc + 1 < NKC || more) store_chunk(g, lds.a[cb ^ 1], lds.b[cb ^ 1]);
            __syncthreads();
        }
        // ---- candidates of this wavefront's 128x128 quarter
        const int row0 = bi * kBM + wr * 128, col0 = bj * kBM + wc * 128;
        float mx[16];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                float m[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) m[i] = fmaxf(acc[x][y][i], acc[x][y][i + 8]);
#pragma unroll
                for (int w = 4; w >= 1; w >>= 1)
#pragma unroll
                    for (int i = 0; i < w; ++i) m[i] = fmaxf(m[i], m[i + w]);
                mx[x * 4 + y] = m[0];
                __builtin_amdgcn_sched_barrier(0);
            }
        float mall = mx[0];
#pragma unroll
        for (int i = 1; i < 16; ++i) mall = fmaxf(mall, mx[i]);
        if (__ballot(mall >= thr) != 0) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    if (__ballot(mx[x * 4 + y] >= thr) == 0) continue;
                    // park the block's 16 scores, then walk them
#pragma unroll
                    for (int i = 0; i < 16; ++i) scr[i * 64 + lane] = acc[x][y][i];
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    __builtin_amdgcn_wave_barrier();
#pragma nounroll
                    for (int i = 0; i < 16; ++i) {
                        const float v = scr[i * 64 + lane];
                        const int r = row0 + x * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                        const int c = col0 + y * 32 + (lane & 31);
                        stage_add(st, cand, v >= thr && r < c && c < n, r, c, v);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                }
        }
        if (!more) break;
        t = tn;
        bi = ni;
        bj = nj;
    }
    st.flush(cand);
}

}  // namespace

namespace mrc {

mrc_status launch_compare_bf16(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, int64_t n, int nk,
                               const float* d_lo_thr, PairSink cand, hipStream_t s) {
    TileOrder ord;
    int64_t grid = 0;
    MRC_TRY(make_tile_order(ctx, (int)ceil_div(n, kBM), 1, &ord, &grid, s));
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 8)
        cus = 256;
    (void)hipGetLastError();
    const int64_t pgrid = std::min<int64_t>((grid + 7) / 8 * 8, cus / 8 * 8);
#define MRC_BF(c)                                                                                        \
    case c:                                                                                              \
        hipLaunchKernelGGL(k_compare_bf16<c>, dim3((unsigned)pgrid), dim3(256), 0, s, q, ldq_bytes, (int)n, \
                           d_lo_thr, ord, cand);                                                         \
        break;
    switch (nk) {
        MRC_BF(2) MRC_BF(4) MRC_BF(6) MRC_BF(8) MRC_BF(10) MRC_BF(12) MRC_BF(16) MRC_BF(20) MRC_BF(24) MRC_BF(32)
        default: return fail(MRC_E_INVAL, "unsupported k for the BF16 form");
    }
#undef MRC_BF
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
