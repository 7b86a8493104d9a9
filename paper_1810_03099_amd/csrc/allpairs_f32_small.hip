// FP32 plain path of the all-pairs comparison for short signatures (k <= 64)
// and very long ones (k > 512, where the 128x128 tiles of allpairs_f32.hip run
// out of registers): the same chain (every score bit-identical to
// acc = fmaf(u_ic, u_jc, acc), c = 0..k-1, on the FP32 matrix cores), over
// 64x64 wavefront tiles with two wavefronts per SIMD. With few components per
// pair a tile's products are short, and the second wavefront's products hide
// one wavefront's flag walk, which dense candidate sets make long. Built with
// the accumulators in VGPRs (its epilogue reads every accumulator).
#include "allpairs.h"
#include "common.h"

using namespace mrc;

namespace {

// Persistent wavefronts: workgroup p runs on XCD p % 8 and its wavefronts walk
// that XCD's contiguous share of the band-ordered tiles. Each tile is 64x64;
// the 16-column chunks are fully unrolled (NC even) and the first chunk of
// the next tile is loaded during the last chunk of the current one; the next
// tile's coordinates are found before the current tile's products.
template <int NC>
__global__ __launch_bounds__(256) void k_compare_f32(const float* __restrict__ u, int n, float tau, TileOrder ord,
                                                     PairSink sink) {
    static_assert(NC % 2 == 0, "even chunk count");
    __shared__ TileLds lds;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    PairStage st{lds.stage[wave], 0};
    float* scr = lds.scr[wave];
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    const int64_t stride = per_xcd_blocks * 4;
    int64_t t = t_lo + bx * 4 + wave;
    if (t >= t_hi) return;
    TileOrder::Cursor cur = ord.seek(t);
    int bi, bj;
    ord.tile(cur, t, &bi, &bj);
    // fragment (16-row block x of the tile, chunk c) of a 64-row panel p
    auto frag = [&](const float* p, int x, int c) { return *(const f32x4*)(p + ((int64_t)x * NC + c) * 256); };
    auto panel = [&](int blk) { return u + ((int64_t)blk * 4 * NC * 64 + lane) * 4; };
    const float* pa = panel(bi);
    const float* pb = panel(bj);
    f32x4 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        a[0][x] = frag(pa, x, 0);
        b[0][x] = frag(pb, x, 0);
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
        for (int c = 0; c < NC; ++c) {
            const int cur_b = c & 1, nxt = cur_b ^ 1;
            if (c + 1 < NC) {
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x] = frag(pa, x, c + 1);
                    b[nxt][x] = frag(pb, x, c + 1);
                }
            } else if (more) {
                // first chunk of the next tile (NC even: it goes to buffer 0)
                pa = panel(ni);
                pb = panel(nj);
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    a[nxt][x] = frag(pa, x, 0);
                    b[nxt][x] = frag(pb, x, 0);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cur_b][x][m], b[cur_b][y][m], acc[x][y], 0,
                                                                         0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        const bool interior = row0 + kWT <= col0 && col0 + kWT <= n;
        const int ib = row0 + 4 * lg, jb = col0 + li;
        tile_epilogue(acc, tau, interior, ib, jb, n, scr, st, sink);
        if (!more) break;
        t = tn;
        bi = ni;
        bj = nj;
    }
    st.flush(sink);
}

// k in (32, 64] (four 16-column chunks): a ring of four chunk buffers in
// registers feeds the matrix-core products (240 registers: two wavefronts per
// SIMD, so that one's flag walk overlaps the other's products, as the 64 KB
// of LDS per workgroup also allows): the loads of chunk c + 3 are issued before
// the products of chunk c (during a tile's chunks 1-3, the next tile's chunks
// 0-2), so three chunks are in flight while one is multiplied. Chunk c of
// every tile lives in buffer c, so the ring needs no register copies, and the
// loads are unconditional (without a next tile: this one again), so the
// compiler's waits stay exact. Same products in the same order as
// k_compare_f32: every score is the plain chain.
__global__ __launch_bounds__(256, 1) void k_compare_f32r(const float* __restrict__ u, int n, float tau,
                                                         TileOrder ord, PairSink sink) {
    constexpr int NC = 4;
    __shared__ TileLds lds;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    PairStage st{lds.stage[wave], 0};
    float* scr = lds.scr[wave];
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    const int64_t stride = per_xcd_blocks * 4;
    int64_t t = t_lo + bx * 4 + wave;
    if (t >= t_hi) return;
    TileOrder::Cursor cur = ord.seek(t);
    int bi, bj;
    ord.tile(cur, t, &bi, &bj);
    // a 64-row panel (16 KB) as a buffer: wavefront-uniform descriptor, the
    // lane's fixed 16-byte offset, the fragment's offset in a scalar register
    constexpr int kPanelB = 64 * NC * 64;
    auto panel = [&](int blk) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(u + (int64_t)blk * (kPanelB / 4)), (short)0, kPanelB,
                                                 0x00020000);
    };
    const int lane16 = 16 * lane;
    auto frag = [&](__amdgpu_buffer_rsrc_t p, int x, int c) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(p, lane16, (x * NC + c) * 1024, 0);
        f32x4 f;
        __builtin_memcpy(&f, &v, 16);
        return f;
    };
    __amdgpu_buffer_rsrc_t pa = panel(bi), pb = panel(bj);
    f32x4 ra[NC][4], rb[NC][4];  // [chunk = buffer][16-row block]
    auto load = [&](__amdgpu_buffer_rsrc_t p, __amdgpu_buffer_rsrc_t q, int c) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            ra[c][x] = frag(p, x, c);
            rb[c][x] = frag(q, x, c);
        }
    };
    load(pa, pb, 0);
    load(pa, pb, 1);
    load(pa, pb, 2);
    while (true) {
        const int64_t tn = t + stride;
        const bool more = tn < t_hi;
        int ni = bi, nj = bj;
        if (more) ord.tile(cur, tn, &ni, &nj);
        const __amdgpu_buffer_rsrc_t na = panel(ni), nb = panel(nj);
        f32x4 acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int row0 = bi * kWT, col0 = bj * kWT;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // chunk c + 3: this tile's last chunk, then the next tile's first three
            if (c == 0) load(pa, pb, 3);
            else load(na, nb, c - 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[c][x][m], rb[c][y][m], acc[x][y], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        const bool interior = row0 + kWT <= col0 && col0 + kWT <= n;
        const int ib = row0 + 4 * lg, jb = col0 + li;
        tile_epilogue(acc, tau, interior, ib, jb, n, scr, st, sink);
        if (!more) break;
        t = tn;
        bi = ni;
        bj = nj;
        pa = na;
        pb = nb;
    }
    st.flush(sink);
}

}  // namespace

namespace mrc {

mrc_status launch_compare_f32_small(mrc_ctx* ctx, const float* umfma, int64_t n, int32_t k, float tau,
                                    PairSink sink, hipStream_t s, int64_t* table) {
    if (n < 2) return MRC_OK;
    TileOrder ord;
    int64_t grid = 0;
    MRC_TRY(make_tile_order(ctx, (int)ceil_div(n, kWT), 4, &ord, &grid, s, table));
    const int nc = mfma_chunks(k);
    ScopedTimer tm(ctx, "compare_f32", s);
    if (nc == 4) {
        const int64_t pgrid = persistent_grid(ctx, (const void*)k_compare_f32r, 256, grid);
        hipLaunchKernelGGL(k_compare_f32r, dim3((unsigned)pgrid), dim3(256), 0, s, umfma, (int)n, tau, ord, sink);
        MRC_HIP_TRY(ctx, hipGetLastError());
        return MRC_OK;
    }
    switch (nc) {
#define MRC_NC(c)                                                                                        \
    case c: {                                                                                            \
        const int64_t pgrid = persistent_grid(ctx, (const void*)k_compare_f32<c>, 256, grid);            \
        hipLaunchKernelGGL(k_compare_f32<c>, dim3((unsigned)pgrid), dim3(256), 0, s, umfma, (int)n, tau, ord,   \
                           sink);                                                                        \
    } break;
        MRC_NC(2) MRC_NC(4) MRC_NC(48) MRC_NC(64)
#undef MRC_NC
        default: return fail(MRC_E_INVAL, "chunk count not instantiated for the 64x64 kernel");
    }
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
