// FP32 plain path of the all-pairs comparison (Eq. 1 applied to two
// signatures): every pair i < j gets the score
//   acc = 0; acc = fmaf(u_ic, u_jc, acc), c = 0..k-1,
// computed on the FP32 matrix cores, whose 16x16x4 step is that chain over its
// four k-values in lane-group order, so consuming the components in ascending
// order keeps every score bit-identical to the chain. Pairs with acc >= tau
// are appended to the output.
//
// Persistent wavefronts, one per SIMD (matrix-core streams of several
// wavefronts on one SIMD run slower than one): workgroup p runs on XCD p % 8
// and its wavefronts walk that XCD's contiguous share of the band-ordered
// 128x128 tiles of the upper triangle. A wavefront computes its tile as 8x8
// blocks of 16x16 products accumulating in the 256 accumulation registers;
// the operands (fragment-major unit signatures: each 16-row x 16-column
// fragment is one contiguous 1 KB load) come straight from global memory, one
// 16-column chunk ahead in a second register set, the next tile's first chunk
// during the current tile's last. The epilogue runs the 64x64 flag walk on
// each quadrant. Used for 64 < k <= 512 (allpairs_f32_small.hip covers the
// rest).
#include <type_traits>

#include "allpairs.h"
#include "common.h"

using namespace mrc;

namespace {

constexpr int kTW = 128;  // wavefront tile (rows = columns)

template <int NC>
__global__ __launch_bounds__(256, 1) void k_compare_f32w(const float* __restrict__ u, int n, float tau,
                                                         TileOrder ord, PairSink sink) {
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
    // fragment (16-row block rb, 16-column chunk c), this lane's 4 floats
    auto frag = [&](int rb, int c) { return *(const f32x4*)(u + (((int64_t)rb * NC + c) * 64 + lane) * 4); };
    f32x4 a[2][8], b[2][8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        a[0][x] = frag(bi * 8 + x, 0);
        b[0][x] = frag(bj * 8 + x, 0);
    }
    while (true) {
        const int64_t tn = t + stride;
        const bool more = tn < t_hi;
        int ni = bi, nj = bj;  // without a next tile: this one again (valid, unused)
        if (more) ord.tile(cur, tn, &ni, &nj);
        f32x4 acc[8][8];
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        // chunk c in buffer B (= c % 2): the next chunk, or the next tile's first
        // (NC even: into buffer 0), is loaded first; no branch, so the waits
        // for the current chunk stay exact
        auto chunk = [&](int c, auto bc) __attribute__((always_inline)) {
            constexpr int B = decltype(bc)::value;
            const bool last = c + 1 == NC;
            const int ra = last ? ni : bi, rbb = last ? nj : bj, cn = last ? 0 : c + 1;
#pragma unroll
            for (int x = 0; x < 8; ++x) {
                a[B ^ 1][x] = frag(ra * 8 + x, cn);
                b[B ^ 1][x] = frag(rbb * 8 + x, cn);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int x = 0; x < 8; ++x)
#pragma unroll
                    for (int y = 0; y < 8; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[B][x][m], b[B][y][m], acc[x][y], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        };
#pragma unroll
        for (int c = 0; c < NC; c += 2) {
            chunk(c, std::integral_constant<int, 0>{});
            chunk(c + 1, std::integral_constant<int, 1>{});
        }
        // flag walk per 64x64 quadrant (lane (li, lg) holds acc[x][y][r] = score
        // of row 16x + 4lg + r, column 16y + li of the tile)
#pragma unroll
        for (int qx = 0; qx < 2; ++qx)
#pragma unroll
            for (int qy = 0; qy < 2; ++qy) {
                const int row0 = bi * kTW + 64 * qx, col0 = bj * kTW + 64 * qy;
                if (col0 + 64 <= row0) continue;  // below the diagonal (diagonal tiles only)
                f32x4 q[4][4];
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) q[x][y] = acc[4 * qx + x][4 * qy + y];
                const bool interior = row0 + 64 <= col0 && col0 + 64 <= n;
                tile_epilogue(q, tau, interior, row0 + 4 * lg, col0 + li, n, scr, st, sink);
            }
        if (!more) break;
        t = tn;
        bi = ni;
        bj = nj;
    }
    st.flush(sink);
}

}  // namespace

namespace mrc {

mrc_status launch_compare_f32(mrc_ctx* ctx, const float* umfma, int64_t n, int32_t k, float tau, PairSink sink,
                              hipStream_t s, int64_t* table) {
    if (n < 2) return MRC_OK;
    const int nc = mfma_chunks(k);
    // short signatures: the flag walk outweighs the short products (64x64 tiles,
    // two wavefronts per SIMD); very long ones: too many registers for 128x128
    if (nc <= 4 || nc > 32) return launch_compare_f32_small(ctx, umfma, n, k, tau, sink, s, table);
    TileOrder ord;
    int64_t grid = 0;
    MRC_TRY(make_tile_order(ctx, (int)ceil_div(n, kTW), 4, &ord, &grid, s, table));
    ScopedTimer tm(ctx, "compare_f32", s);
    switch (nc) {
#define MRC_NC(c)                                                                                          \
    case c: {                                                                                              \
        const int64_t pgrid = persistent_grid(ctx, (const void*)k_compare_f32w<c>, 256, grid);             \
        hipLaunchKernelGGL(k_compare_f32w<c>, dim3((unsigned)pgrid), dim3(256), 0, s, umfma, (int)n, tau, ord, \
                           sink);                                                                          \
    } break;
        MRC_NC(6) MRC_NC(8) MRC_NC(12) MRC_NC(16) MRC_NC(24) MRC_NC(32)
#undef MRC_NC
        default: return fail(MRC_E_INVAL, "k exceeds 1024");
    }
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
