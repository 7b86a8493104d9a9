// Low-precision candidate search of the all-pairs comparison (BF16 and FP8
// e4m3 codes of the unit signatures), LDS-tiled.
//
// Each workgroup (4 wavefronts, one per SIMD: matrix-core streams of several
// wavefronts on one SIMD run slower than one) computes 256x256 blocks of the
// upper triangle of Q Q^T (Q: the codes, rows padded to a multiple of 256 with
// zeros); wavefront (wr, wc) owns the 128x128 quarter at rows 128wr, columns
// 128wc, as 4x4 blocks of 32x32 matrix-core products accumulating in FP32
// (BF16: 32x32x16 steps; FP8: 32x32x64 steps whose E8M0 operand scales apply
// the rows' power-of-two code scales, so the accumulators hold the scaled
// scores). Operands pass through LDS in chunks of 128 bytes per row (64 BF16
// or 128 FP8 components), loaded by buffer loads straight into LDS (no
// register staging) one chunk ahead into the other of two buffers, the loads
// interleaved with the first step's products; each 128-byte row holds its
// eight 16-byte parts XOR-swizzled by (row / 2) % 8, so the 16-byte fragment
// reads of 16 consecutive rows hit distinct banks. The fragment reads of step
// s + 1 are issued before the products of step s (scheduling fences keep the
// compiler from sinking them), so LDS latency hides behind 16 products. Every
// score is compared with the candidate threshold (FP8: a 32x32 block whose
// maximum passes the global one is then held to its own, from its rows'
// largest errors); blocks without any score at or above it end after a max
// tree.
//
// 32x32 operand / result layouts (lane l): A fragment = row l % 32, the
// (l / 32)-th half of the step's components (8 BF16 = 16 bytes, or 32 FP8 =
// 32 bytes; B the same with columns); result value i of the block = row
// 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
#include <type_traits>

#include "allpairs.h"
#include "common.h"

using namespace mrc;

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kBM = 256;          // workgroup tile (rows = columns)
constexpr int kRowB = 128;        // LDS bytes per row of a chunk (8 parts of 16 bytes, swizzled)
constexpr int kBufB = kBM * kRowB;
constexpr int kStageB = 256;      // staged pairs per wavefront
// Band height of the tile order (tile rows per band). Measured at 200k rows x
// k = 256: FP8 4.78 ms with bands of 8, 4.49 ms with 10, 4.56 ms with 12 or 20;
// BF16 the same for all of them.
constexpr int kLdsBand = 10;

struct LdsTiles {
    uint8_t a[2][kBufB];          // [buffer][256 rows x 128 bytes] of the row panel
    uint8_t b[2][kBufB];          // the same for the column panel
    mrc_pair stage[4][kStageB];
    float scr[4][16 * 64];        // parked scores of one 32x32 block per wavefront
};

// Matrix-core step of each form: steps per 128-byte chunk and 16-byte parts
// per lane and step (kSteps * kParts = 4 in both).
template <int PREC> struct Form;
template <> struct Form<MRC_PREC_BF16> {
    static constexpr int kSteps = 4, kParts = 1;
    typedef bf16x8 frag;
};
template <> struct Form<MRC_PREC_FP8> {
    static constexpr int kSteps = 2, kParts = 2;
    typedef i32x8 frag;
};

__device__ __forceinline__ f32x16 mma(const bf16x8& a, const bf16x8& b, const f32x16& c, int, int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// formats 0 / 0: both operands float8 e4m3; sa / sb: E8M0 scales of the
// lane's row of A and of B (byte 0)
__device__ __forceinline__ f32x16 mma(const i32x8& a, const i32x8& b, const f32x16& c, int sa, int sb) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}

// E8M0 code of a power-of-two float scale (its biased exponent; 0 for 0).
__device__ __forceinline__ int e8m0(float s) { return (int)((__float_as_uint(s) >> 23) & 0xFFu); }

template <int V>
using ic = std::integral_constant<int, V>;

// NKC: 128-byte chunks per row (ldq_bytes = 128 NKC). scale: FP8 row scales
// (powers of two), [rows of q]; unused for BF16. lo_thr_ptr: the candidate
// threshold for every pair (device, one float). bb: FP8 per-block thresholds
// (BlockBand); unused for BF16.
template <int PREC, int NKC>
__global__ __launch_bounds__(256, 1) void k_compare_lds(const uint8_t* __restrict__ q, int ldq_bytes,
                                                        const float* __restrict__ scale, int n,
                                                        const float* __restrict__ lo_thr_ptr, TileOrder ord,
                                                        BlockBand bb, PairSink cand) {
    using F = Form<PREC>;
    using frag = typename F::frag;
    constexpr bool kFp8 = PREC == MRC_PREC_FP8;
    __shared__ LdsTiles lds;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    PairStage st{lds.stage[wave], 0};
    const float thr = *lo_thr_ptr;
    const int64_t xcd = blockIdx.x % 8, per_xcd_blocks = gridDim.x / 8, bx = blockIdx.x / 8;
    const int64_t t_lo = ord.n_tiles * xcd / 8, t_hi = ord.n_tiles * (xcd + 1) / 8;
    int64_t t = t_lo + bx;
    if (t >= t_hi) return;
    TileOrder::Cursor cur = ord.seek(t);
    int bi, bj;
    ord.tile(cur, t, &bi, &bj);

    // Operand loads: load i (0..7) of a chunk fills rows 64 wave + 8 i .. +8 of
    // both panels; lane l writes stored part l % 8 of row l / 8 there, i.e.
    // chunk part (l % 8) ^ ((row / 2) % 8), where (row / 2) % 8 = l / 16 + 4 (i % 2).
    // Per lane only two byte offsets occur (even / odd i); the rest of the
    // address is wavefront-uniform (buffer descriptor of the panel + offset).
    uint32_t voff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
        voff[h] = (uint32_t)((wave * 64 + (lane >> 3)) * ldq_bytes + (((lane & 7) ^ ((lane >> 4) + 4 * h)) * 16));
    const int panel_bytes = kBM * ldq_bytes;
    auto rsrc = [&](int blk) {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(q + (int64_t)blk * panel_bytes), (short)0, panel_bytes,
                                                 0x00020000);
    };
    // load i of chunk kc (rows 64 wave + 8 i .. +8 of both panels) into buffer b
    auto issue_load = [&](auto bc, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb, int kc, int i)
        __attribute__((always_inline)) {
        constexpr int b = decltype(bc)::value;
        const int so = kc * kRowB + i * 8 * ldq_bytes;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void*)(lds.a[b] + (wave * 64 + i * 8) * kRowB), 16,
                                                 voff[i & 1], so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void*)(lds.b[b] + (wave * 64 + i * 8) * kRowB), 16,
                                                 voff[i & 1], so, 0, 0);
    };
    auto issue_chunk = [&](auto bc, __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rb, int kc)
        __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 8; ++i) issue_load(bc, ra, rb, kc, i);
    };
    // Fragment reads: row l % 32 of each 32-row block; part h of step s is
    // chunk part kParts (2s + l / 32) + h, read at its stored position (blocks
    // start at multiples of 32 rows, so the swizzle depends on l % 32 only).
    const int frow = lane & 31, swz = (frow >> 1) & 7, fhi = lane >> 5;
    const uint8_t* pa[4];
    const uint8_t* pb[4];
#pragma unroll
    for (int s = 0; s < F::kSteps; ++s)
#pragma unroll
        for (int h = 0; h < F::kParts; ++h) {
            const int po = ((F::kParts * (2 * s + fhi) + h) ^ swz) * 16;
            pa[s * F::kParts + h] = &lds.a[0][0] + (wr * 128 + frow) * kRowB + po;
            pb[s * F::kParts + h] = &lds.b[0][0] + (wc * 128 + frow) * kRowB + po;
        }
    frag fa[2][4], fb[2][4];
    auto read_a = [&](auto bc, int s, int x, frag& r) __attribute__((always_inline)) {
        constexpr int b = decltype(bc)::value;
#pragma unroll
        for (int h = 0; h < F::kParts; ++h) {
            const u32x4 v = *(const u32x4*)(pa[s * F::kParts + h] + b * kBufB + x * 32 * kRowB);
            __builtin_memcpy((uint8_t*)&r + 16 * h, &v, 16);
        }
    };
    auto read_b = [&](auto bc, int s, int y, frag& r) __attribute__((always_inline)) {
        constexpr int b = decltype(bc)::value;
#pragma unroll
        for (int h = 0; h < F::kParts; ++h) {
            const u32x4 v = *(const u32x4*)(pb[s * F::kParts + h] + b * kBufB + y * 32 * kRowB);
            __builtin_memcpy((uint8_t*)&r + 16 * h, &v, 16);
        }
    };
    auto read_step = [&](auto bc, int s, frag (&ra)[4], frag (&rb)[4]) __attribute__((always_inline)) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            read_a(bc, s, x, ra[x]);
            read_b(bc, s, x, rb[x]);
        }
    };
    // FP8: E8M0 scales of the lane's rows (row l % 32 of block x of the row
    // quarter, of block y of the column quarter), loaded one block pair ahead
    int sa[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0}, nsa[4] = {0, 0, 0, 0}, nsb[4] = {0, 0, 0, 0};
    // and the largest row errors of the 32-row blocks (per-block candidate thresholds)
    float ea[4] = {0.f, 0.f, 0.f, 0.f}, eb[4] = {0.f, 0.f, 0.f, 0.f}, nea[4] = {0.f, 0.f, 0.f, 0.f},
          neb[4] = {0.f, 0.f, 0.f, 0.f};
    auto load_scales = [&](int ti, int tj, int (&ra)[4], int (&rb)[4], float (&xa)[4], float (&xb)[4])
        __attribute__((always_inline)) {
        if constexpr (kFp8) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                ra[x] = e8m0(scale[ti * kBM + wr * 128 + x * 32 + frow]);
                rb[x] = e8m0(scale[tj * kBM + wc * 128 + x * 32 + frow]);
                xa[x] = bb.blk_err[ti * 8 + wr * 4 + x];
                xb[x] = bb.blk_err[tj * 8 + wc * 4 + x];
            }
        }
    };

    __amdgpu_buffer_rsrc_t qa = rsrc(bi), qb = rsrc(bj);
    load_scales(bi, bj, sa, sb, ea, eb);
    issue_chunk(ic<0>{}, qa, qb, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    read_step(ic<0>{}, 0, fa[0], fb[0]);

    f32x16 acc[4][4];
    float mx[16];  // largest score of each 32x32 block of the finished tile
    // three-input maxima: 16 values in 8 instructions
    auto tree = [&](int x, int y) __attribute__((always_inline)) {
        float m0 = fmaxf(fmaxf(acc[x][y][0], acc[x][y][1]), acc[x][y][2]);
        float m1 = fmaxf(fmaxf(acc[x][y][3], acc[x][y][4]), acc[x][y][5]);
        float m2 = fmaxf(fmaxf(acc[x][y][6], acc[x][y][7]), acc[x][y][8]);
        float m3 = fmaxf(fmaxf(acc[x][y][9], acc[x][y][10]), acc[x][y][11]);
        float m4 = fmaxf(fmaxf(acc[x][y][12], acc[x][y][13]), acc[x][y][14]);
        m0 = fmaxf(fmaxf(m0, m1), acc[x][y][15]);
        m2 = fmaxf(fmaxf(m2, m3), m4);
        return fmaxf(m0, m2);
    };
    // One chunk in buffer b. The loads of the following chunk (of this block
    // pair, or the first of the next pair) go to the other buffer, one after
    // each product of the first step; the reads of step s + 1 are issued
    // before the products of step s, and the reads of the following chunk's
    // first step (of this block pair) before the last products, after the
    // barrier that makes that chunk visible. FP8 fragments are twice as wide:
    // there the A fragments have one buffer, fragment x of the next step read
    // right after the four products that use fragment x of this one.
    auto chunk = [&](auto bc, int kc, bool more, __amdgpu_buffer_rsrc_t nqa, __amdgpu_buffer_rsrc_t nqb, auto lc)
        __attribute__((always_inline)) {
        constexpr bool lastc = decltype(lc)::value;  // the block pair's last chunk
        constexpr int b = decltype(bc)::value;
        const bool next_here = kc + 1 < NKC;
        // what the loads fetch: the next chunk of this pair, else the first of
        // the next pair (without a next pair: the first chunk of this one
        // again, into a buffer nobody reads any more), chosen without branches
        const __amdgpu_buffer_rsrc_t la = next_here ? qa : nqa, lb = next_here ? qb : nqb;
        const int lkc = next_here ? kc + 1 : 0;
        (void)more;
#pragma unroll
        for (int s = 0; s < F::kSteps; ++s) {
            const bool last = s + 1 == F::kSteps;
            if (!last) {
                if constexpr (kFp8) {
#pragma unroll
                    for (int y = 0; y < 4; ++y) read_b(bc, s + 1, y, fb[(s + 1) & 1][y]);
                } else {
                    read_step(bc, s + 1, fa[(s + 1) & 1], fb[(s + 1) & 1]);
                }
            } else {
                // the following chunk is in LDS for every wavefront, and no
                // wavefront reads buffer b any more
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (next_here) {
                    if constexpr (kFp8) {
#pragma unroll
                        for (int y = 0; y < 4; ++y) read_b(ic<b ^ 1>{}, 0, y, fb[0][y]);
                    } else {
                        read_step(ic<b ^ 1>{}, 0, fa[0], fb[0]);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            if (lastc && s + 1 == F::kSteps) {
                // last products of the block pair: the max tree of block j - 4
                // goes in after the product of block j (its last product, four
                // products back, has finished), the last four after the loop
                const auto& fa_s = kFp8 ? fa[0] : fa[s & 1];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    acc[j >> 2][j & 3] = mma(fa_s[j >> 2], fb[s & 1][j & 3], acc[j >> 2][j & 3], sa[j >> 2], sb[j & 3]);
                    if (j >= 4) mx[j - 4] = tree((j - 4) >> 2, (j - 4) & 3);
                }
#pragma unroll
                for (int j = 12; j < 16; ++j) mx[j] = tree(j >> 2, j & 3);
                __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
#pragma unroll
                for (int g = 0; g < 12; ++g) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 24, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            } else if constexpr (kFp8) {
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    if (s == 0) {
                        issue_load(ic<b ^ 1>{}, la, lb, lkc, 2 * x);
                        issue_load(ic<b ^ 1>{}, la, lb, lkc, 2 * x + 1);
                    }
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = mma(fa[0][x], fb[s & 1][y], acc[x][y], sa[x], sb[y]);
                    if (s == 0) {
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (!last) read_a(bc, s + 1, x, fa[0][x]);
                    else if (next_here) read_a(ic<b ^ 1>{}, 0, x, fa[0][x]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                if (s == 0) issue_chunk(ic<b ^ 1>{}, la, lb, lkc);
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = mma(fa[s & 1][x], fb[s & 1][y], acc[x][y], sa[x], sb[y]);
                if (s == 0) {  // product, load, product, load, ...
#pragma unroll
                    for (int g = 0; g < 16; ++g) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto tile = [&](auto pc) __attribute__((always_inline)) -> bool {
        constexpr int P = decltype(pc)::value;   // buffer of the first chunk
        const int64_t tn = t + per_xcd_blocks;
        const bool more = tn < t_hi;
        int ni = bi, nj = bj;
        if (more) ord.tile(cur, tn, &ni, &nj);
        const __amdgpu_buffer_rsrc_t nqa = rsrc(ni), nqb = rsrc(nj);
        load_scales(ni, nj, nsa, nsb, nea, neb);  // (ni, nj) = (bi, bj) without a next pair
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = f32x16{};
        int kc = 0;
#pragma unroll
        for (; kc + 2 < NKC; kc += 2) {
            chunk(ic<P>{}, kc, more, nqa, nqb, std::false_type{});
            chunk(ic<P ^ 1>{}, kc + 1, more, nqa, nqb, std::false_type{});
        }
        if constexpr ((NKC & 1) != 0) {
            chunk(ic<P>{}, kc, more, nqa, nqb, std::true_type{});
        } else {
            chunk(ic<P>{}, kc, more, nqa, nqb, std::false_type{});
            chunk(ic<P ^ 1>{}, kc + 1, more, nqa, nqb, std::true_type{});
        }
        // ---- candidates of this wavefront's 128x128 quarter (mx: from the last chunk)
        const int row0 = bi * kBM + wr * 128, col0 = bj * kBM + wc * 128;
        float mall = mx[0];
#pragma unroll
        for (int i = 1; i < 16; ++i) mall = fmaxf(mall, mx[i]);
        if (__ballot(mall >= thr) != 0) {
            float* scr = lds.scr[wave];
            const int c = (lane & 31);
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    if (__ballot(mx[x * 4 + y] >= thr) == 0) continue;
                    float tb = thr;
                    if constexpr (kFp8) {  // the block's own threshold (never below the global one)
                        tb = fmaxf(thr, fminf(bb.t_nom, fmaf(-(bb.g * (1.f + ea[x])), 1.f + eb[y], bb.c)));
                        if (__ballot(mx[x * 4 + y] >= tb) == 0) continue;
                    }
                    // park the block, then each lane finds its flagged values
                    // (row 8 (i / 4) + 4 (l / 32) + i % 4) and reads them back by index
#pragma unroll
                    for (int i = 0; i < 16; ++i) scr[i * 64 + lane] = acc[x][y][i];
                    __builtin_amdgcn_sched_barrier(0);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const int rb = row0 + x * 32 + 4 * (lane >> 5), cc = col0 + y * 32 + c;
                    uint32_t m = 0;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int r = rb + 8 * (i >> 2) + (i & 3);
                        m |= (scr[i * 64 + lane] >= tb && r < cc && cc < n ? 1u : 0u) << i;
                    }
                    const int total = wave_total6(__popc(m));
                    if (total == 0) continue;
                    __builtin_amdgcn_sched_barrier(0);
                    if (st.n + total > kStageB) st.flush(cand);
                    const bool direct = total > kStageB;  // more than a stage: straight to the output
                    int64_t base;
                    if (direct) {
                        unsigned long long b0 = 0;
                        if (lane == 0) b0 = atomicAdd(cand.counter, (unsigned long long)total);
                        base = (int64_t)__shfl(b0, 0, 64);
                    } else {
                        base = st.n;
                        st.n += total;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // rounds: each lane with marks left writes its lowest one,
                    // the round's lanes at consecutive positions
                    while (true) {
                        const uint64_t act = __ballot(m != 0);
                        if (act == 0) break;
                        if (m) {
                            const int i = __ffs(m) - 1;
                            m &= m - 1;
                            const mrc_pair pr{rb + 8 * (i >> 2) + (i & 3), cc, scr[i * 64 + lane], 0};
                            const int64_t pos = round_pos(base, act);
                            if (direct) {
                                if (pos < cand.capacity) cand.pairs[pos] = pr;
                            } else {
                                stage_put(st.buf, (int)pos, pr);
                            }
                        }
                        base += __popcll(act);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
        }
        if (!more) return false;
        // first step of the next block pair (its first chunk is in LDS)
        read_step(ic<(P + NKC) & 1>{}, 0, fa[0], fb[0]);
        t = tn;
        bi = ni;
        bj = nj;
        qa = nqa;
        qb = nqb;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            sa[x] = nsa[x];
            sb[x] = nsb[x];
            ea[x] = nea[x];
            eb[x] = neb[x];
        }
        return true;
    };
    while (true) {
        if (!tile(ic<0>{})) break;
        if constexpr ((NKC & 1) != 0)
            if (!tile(ic<1>{})) break;
    }
    st.flush(cand);
}

template <int PREC>
mrc_status launch_lds(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, const float* scale, int64_t n,
                      const float* d_lo_thr, BlockBand bb, PairSink cand, hipStream_t s) {
    if (ldq_bytes % kRowB != 0) return fail(MRC_E_INVAL, "low-precision rows must be whole 128-byte chunks");
    const int nkc = ldq_bytes / kRowB;
    TileOrder ord;
    int64_t grid = 0;
    MRC_TRY(make_tile_order(ctx, (int)ceil_div(n, kBM), 1, &ord, &grid, s, nullptr, kLdsBand));
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 8)
        cus = 256;
    (void)hipGetLastError();
    const int64_t pgrid = std::min<int64_t>((grid + 7) / 8 * 8, cus / 8 * 8);
#define MRC_LDS(c)                                                                                          \
    case c:                                                                                                 \
        hipLaunchKernelGGL((k_compare_lds<PREC, c>), dim3((unsigned)pgrid), dim3(256), 0, s, q, ldq_bytes, \
                           scale, (int)n, d_lo_thr, ord, bb, cand);                                         \
        break;
    if constexpr (PREC == MRC_PREC_BF16) {
        switch (nkc) {
            MRC_LDS(1) MRC_LDS(2) MRC_LDS(3) MRC_LDS(4) MRC_LDS(5) MRC_LDS(6) MRC_LDS(8) MRC_LDS(10) MRC_LDS(12)
            MRC_LDS(16)
            default: return fail(MRC_E_INVAL, "unsupported k for the BF16 form");
        }
    } else {
        switch (nkc) {
            MRC_LDS(1) MRC_LDS(2) MRC_LDS(3) MRC_LDS(4) MRC_LDS(5) MRC_LDS(6) MRC_LDS(8)
            default: return fail(MRC_E_INVAL, "unsupported k for the FP8 form");
        }
    }
#undef MRC_LDS
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace

namespace mrc {

int lowp_lds_chunks(int precision, int k) {
    const int need = (int)ceil_div((int64_t)k * (precision == MRC_PREC_BF16 ? 2 : 1), kRowB);
    static const int kInst[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int c : kInst)
        if (c >= need && (precision == MRC_PREC_BF16 || c <= 8)) return c;
    return -1;
}

mrc_status launch_compare_bf16(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, int64_t n, const float* d_lo_thr,
                               PairSink cand, hipStream_t s) {
    return launch_lds<MRC_PREC_BF16>(ctx, q, ldq_bytes, nullptr, n, d_lo_thr, BlockBand{nullptr, 0.f, 0.f, 0.f}, cand,
                                     s);
}

mrc_status launch_compare_fp8(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, const float* scale, int64_t n,
                              const float* d_lo_thr, BlockBand bb, PairSink cand, hipStream_t s) {
    return launch_lds<MRC_PREC_FP8>(ctx, q, ldq_bytes, scale, n, d_lo_thr, bb, cand, s);
}

}  // namespace mrc
