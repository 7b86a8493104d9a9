// Query against a resident signature database (Section 1: each new page is
// compared with all stored pages through the signatures).
//
// For every query: the topk database rows of highest MRC (score descending,
// id ascending) and the number of rows with MRC >= tau.
//
// Queries go in groups of 16 as the B operand of 16x16 matrix-core tiles
// whose A operand is 64 database rows, so lane (li, lg) of a wavefront holds
// the scores of query li against 16 of the 64 rows.
//
// Two passes. The first finds, for each query, 16 high-scoring rows of a
// prefix of the database: every lane keeps the best row of its own stream
// (its lane group's rows of its wavefront's tiles), and the 16 best of these
// stream maxima per query (distinct rows, nearly always the prefix's own 16
// best) give E16, the smallest exact (chain) score among them: the exact
// 16th best over all rows is at least E16. The second pass collects every row
// whose score is >= min(E16 - b, tau - b) (b: the query's rescoring band
// against the database's BF16/FP8 codes, 0 for FP32 scores, which are the
// plain chain itself), with up to 4 query groups per wavefront sharing each
// database fragment; the candidates, a superset of the exact top-16 and of
// all rows >= tau, are then scored with the FP32 chain.
#include <algorithm>

#include "common.h"

using namespace mrc;

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kTop = 16;
constexpr int kTileRows = 64;
constexpr int64_t kPrefixMin = 16384;  // rows of the first pass: this many, or 1/16 of the database

template <int PREC> struct QT;
template <> struct QT<MRC_PREC_FP32> {
    static constexpr int kChunkBytes = 64, kLaneBytes = 16;
    struct F { f32x4 v; };
    __device__ static F load(const uint8_t* p) { return F{*(const f32x4*)p}; }
    __device__ static f32x4 mma(const F& a, const F& b, f32x4 c) {
#pragma unroll
        for (int m = 0; m < 4; ++m) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[m], b.v[m], c, 0, 0, 0);
        return c;
    }
};
template <> struct QT<MRC_PREC_BF16> {
    static constexpr int kChunkBytes = 64, kLaneBytes = 16;
    struct F { i32x4 v; };
    __device__ static F load(const uint8_t* p) { return F{*(const i32x4*)p}; }
    __device__ static f32x4 mma(const F& a, const F& b, f32x4 c) {
        bf16x8 av, bv;
        __builtin_memcpy(&av, &a.v, 16);
        __builtin_memcpy(&bv, &b.v, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    }
};
template <> struct QT<MRC_PREC_FP8> {
    static constexpr int kChunkBytes = 128, kLaneBytes = 32;
    struct F { i32x4 lo, hi; };
    __device__ static F load(const uint8_t* p) { return F{*(const i32x4*)p, *(const i32x4*)(p + 16)}; }
    __device__ static f32x4 mma(const F& a, const F& b, f32x4 c) {
        const i32x8 av = {a.lo[0], a.lo[1], a.lo[2], a.lo[3], a.hi[0], a.hi[1], a.hi[2], a.hi[3]};
        const i32x8 bv = {b.lo[0], b.lo[1], b.lo[2], b.lo[3], b.hi[0], b.hi[1], b.hi[2], b.hi[3]};
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
};

// (s, id) ordering of the results: score descending, id ascending.
__device__ __forceinline__ bool better(float s1, int64_t i1, float s2, int64_t i2) {
    return s1 > s2 || (s1 == s2 && i1 < i2);
}

// Insert (v, j) into a list sorted best first; precondition: it beats the last.
__device__ __forceinline__ void top_insert(float (&s)[kTop], int (&id)[kTop], float v, int j) {
    bool placed = false;
#pragma unroll
    for (int p = kTop - 1; p > 0; --p) {
        if (!placed) {
            if (better(v, j, s[p - 1], id[p - 1])) {
                s[p] = s[p - 1];
                id[p] = id[p - 1];
            } else {
                s[p] = v;
                id[p] = j;
                placed = true;
            }
        }
    }
    if (!placed) {
        s[0] = v;
        id[0] = j;
    }
}

// Candidate marks of one query group on one 64-row tile: bit 4x + r of lane
// (li, lg) is set when row row0 + 16x + 4lg + r scores at least the query's
// threshold. The sign of score - threshold decides, which for finite values
// is the comparison itself (a difference is zero only for equal operands, and
// a flush to zero keeps its sign); a funnel shift moves each sign into the
// word, one instruction per score. Invalid queries carry threshold +inf;
// rowmask clears rows past the end of the database.
__device__ __forceinline__ uint32_t tile_marks(const f32x4 (&acc)[4], float thr, uint32_t rowmask) {
#pragma clang fp contract(off)  // (the score as rounded, not fused into the difference)
    uint32_t below = 0;
#pragma unroll
    for (int e = 15; e >= 0; --e)
        below = __builtin_amdgcn_alignbit(below, __float_as_uint(acc[e >> 2][e & 3] - thr), 31);
    return ~below & rowmask;
}

// The marks with a per-row threshold thr - b e_r (FP8: e = the errors of the
// lane's 16 rows, e[x][r] for row row0 + 16x + 4lg + r): the threshold is
// one fused multiply-add per score, then the same sign test.
__device__ __forceinline__ uint32_t tile_marks_rows(const f32x4 (&acc)[4], float thr, float b, const f32x4 (&e)[4],
                                                   uint32_t rowmask) {
#pragma clang fp contract(off)  // (the score as rounded, not fused into the difference)
    uint32_t below = 0;
#pragma unroll
    for (int i = 15; i >= 0; --i) {
        const float t = __builtin_fmaf(-b, e[i >> 2][i & 3], thr);
        below = __builtin_amdgcn_alignbit(below, __float_as_uint(acc[i >> 2][i & 3] - t), 31);
    }
    return ~below & rowmask;
}

// The marks a tile's rows allow: all 16, except on the last tile, where the
// rows at or past rows_left (counted from the tile's first row) drop out.
__device__ __forceinline__ uint32_t tile_rowmask(int64_t rows_left, int lg) {
    if (rows_left >= kTileRows) return 0xffffu;
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e)
        if (16 * (e >> 2) + 4 * lg + (e & 3) < rows_left) m |= 1u << e;
    return m;
}

// One step of an all-lanes (score, id) reduction: each lane compares with
// the lane a DPP pattern names (within its row of 16) and keeps the better.
template <int CTRL>
__device__ __forceinline__ void best_step(float& v, int& id) {
    const float ov = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
    const int oi = __builtin_amdgcn_mov_dpp(id, CTRL, 0xf, 0xf, true);
    if (better(ov, oi, v, id)) {
        v = ov;
        id = oi;
    }
}

// The best (score, id) of the wavefront, returned in every lane: within each
// row of 16 lanes by DPP (quad lanes xor 1, xor 2, then rotations of the row
// by 4 and by 8: every lane then holds its row's best), then the four rows'
// bests read from lanes 0, 16, 32, 48 (no LDS round trips).
__device__ __forceinline__ void wave_best(float& v, int& id) {
    best_step<0xb1>(v, id);   // quad_perm [1, 0, 3, 2]
    best_step<0x4e>(v, id);   // quad_perm [2, 3, 0, 1]
    best_step<0x124>(v, id);  // row_ror:4
    best_step<0x128>(v, id);  // row_ror:8
    float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    int bi = __builtin_amdgcn_readlane(id, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16 * r));
        const int ci = __builtin_amdgcn_readlane(id, 16 * r);
        if (better(c, ci, b, bi)) {
            b = c;
            bi = ci;
        }
    }
    v = b;
    id = bi;
}

// The best topk (score, id) pairs of a workgroup's 256 lists (one sorted
// list per thread; id 0x7fffffff marks an empty entry): each wavefront takes
// the best topk of its 64 lists (repeatedly the best head across lanes) into
// LDS (ss, si: 4 kTop entries each), then wavefront 0 takes the best topk of
// those four and hands entry p to emit(p, score, id) on its lane 0. Every
// thread of the workgroup calls it (it holds a workgroup barrier).
template <typename Emit>
__device__ __forceinline__ void block_top(const float (&ts)[kTop], const int (&ti)[kTop], int topk, float* ss,
                                          int* si, Emit emit) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int h = 0;
    for (int p = 0; p < topk; ++p) {
        float hs = -INFINITY;
        int hi = 0x7fffffff;
#pragma unroll
        for (int x = 0; x < kTop; ++x)
            if (x == h) {
                hs = ts[x];
                hi = ti[x];
            }
        float bs = hs;
        int bi = hi;
        wave_best(bs, bi);
        if (bi != 0x7fffffff && hi == bi && hs == bs) ++h;  // ids are unique: one lane pops
        if (lane == 0) {
            ss[w * kTop + p] = bs;
            si[w * kTop + p] = bi;
        }
    }
    __syncthreads();
    if (w != 0) return;
    const int src = (lane >> 4) * kTop + (lane & 15);  // lane: entry (lane & 15) of wavefront lane >> 4
    float v = (lane & 15) < topk ? ss[src] : -INFINITY;
    int id = (lane & 15) < topk ? si[src] : 0x7fffffff;
    for (int p = 0; p < topk; ++p) {
        float bs = v;
        int bi = id;
        wave_best(bs, bi);
        if (bi != 0x7fffffff && id == bi && v == bs) {  // (ids are unique: one lane)
            v = -INFINITY;
            id = 0x7fffffff;
        }
        if (lane == 0) emit(p, bs, bi);
    }
}

struct ScanArgs {
    const uint8_t* db;        // [rows_pad][ld_db] codes (FP32: matrix-core layout floats)
    int ld_db;                // bytes per row
    const float* db_scale;    // FP8 row scales
    int64_t rows;             // rows scanned (a prefix of the database snapshot, or all of it)
    const uint8_t* q;         // [nq_pad][ld_q] query codes, same layout
    int ld_q;
    const float* q_scale;
    int nq;
    float tau;
    // MODE_TOP: each query's stream maxima, [nq][streams] (16 per workgroup
    // of k_query_scan, 4 per workgroup of the LDS-shared kernel)
    float* part_s;
    int32_t* part_id;
    // MODE_COLLECT: candidates with score >= thr[q]
    const float* thr;         // per query: the threshold (FP8: its part C_q without the row term)
    const float* thr_b;       // FP8: per query B_q, the row term's coefficient (threshold C_q - B_q e_r)
    const float* row_err;     // FP8: per database row e_r, its code's error bound
    int32_t* cand;            // [nq][cap] row ids
    int32_t* ccount;          // [nq]
    int cap;
    // persistent collection: items (query block, kPersistTiles tiles) taken in
    // order from a zeroed device counter
    unsigned long long* work;
    int64_t n_items;          // query blocks x tile ranges
    int64_t tile_ranges;      // tile ranges per query block
};

// Tiles per work item of the persistent collection.
constexpr int kPersistTiles = 16;

// Slots for a tile's marks: every lane with marks adds its count to its
// query's candidate counter (a query's lanes take their ranges in any order:
// the final pass orders the candidates itself).
template <int G>
__device__ __forceinline__ void reserve_marks(const ScanArgs& a, const uint32_t (&m)[G], const int (&q)[G],
                                              int (&base)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        base[g] = 0;
        if (m[g]) base[g] = atomicAdd(&a.ccount[q[g]], __popc(m[g]));
    }
}

// Write the row ids of a tile's marks into their slots; those past the
// capacity are dropped (the counter still counts them: the host grows the
// capacity and collects again).
template <int G>
__device__ __forceinline__ void write_marks(const ScanArgs& a, const uint32_t (&m)[G], const int (&q)[G],
                                            const int (&base)[G], int64_t row0, int lg) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        uint32_t mm = m[g];
        int b = base[g];
        int32_t* dst = a.cand + (int64_t)q[g] * a.cap;
        const int r0 = (int)row0 + 4 * lg;
        while (mm) {
            const int e = __builtin_ctz(mm);
            mm &= mm - 1;
            if (b < a.cap) dst[b] = r0 + 16 * (e >> 2) + (e & 3);
            ++b;
        }
    }
}

enum { MODE_TOP = 0, MODE_COLLECT = 1 };

// One workgroup per (share of the database, block of 16 G queries): its 4
// wavefronts take turns over the share's 64-row tiles, and each wavefront
// holds the G query groups' fragments, so every database fragment it loads
// feeds G products (G > 1: collection only, where a lane keeps no lists).
template <int PREC, int NK, int MODE, int G, bool PERS = false>
__global__ __launch_bounds__(256) void k_query_scan(ScanArgs a) {
    using T = QT<PREC>;
    static_assert(MODE == MODE_COLLECT || G == 1, "top lists for one query group per wavefront");
    static_assert(!PERS || MODE == MODE_COLLECT, "the persistent form collects");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    // query fragments of every group and chunk stay in registers (rows of the
    // padded query arrays: every group of the block is readable)
    typename T::F qb[G][NK];
    int q[G];
    bool qvalid[G];
    float qsc[G], thr[G], thrb[G];
    // collection: the previous tile's marks, their reserved slots and first
    // row (written once the next tile's loads have returned, by when the
    // slot atomics issued before them have too)
    uint32_t pm[G];
    int pb[G];
    int64_t prow0 = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        pm[g] = 0;
        pb[g] = 0;
    }
    // the query fragments of block y (PERS: the block of the current item)
    auto load_queries = [&](int64_t y) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            q[g] = (int)((y * G + g) * 16 + li);
            qvalid[g] = q[g] < a.nq;
            const uint8_t* pq = a.q + (int64_t)q[g] * a.ld_q + lg * T::kLaneBytes;
#pragma unroll
            for (int c = 0; c < NK; ++c) qb[g][c] = T::load(pq + c * T::kChunkBytes);
            qsc[g] = (PREC == MRC_PREC_FP8) ? a.q_scale[q[g]] : 1.f;
            if (MODE == MODE_COLLECT) {
                const float t = qvalid[g] ? a.thr[q[g]] : INFINITY;
                thr[g] = t == t ? t : INFINITY;  // (no marks for a NaN threshold)
                thrb[g] = (PREC == MRC_PREC_FP8 && qvalid[g]) ? a.thr_b[q[g]] : 0.f;
            }
        }
    };
    int64_t cur_y = PERS ? -1 : (int64_t)blockIdx.y;
    if (!PERS) load_queries(cur_y);
    // MODE_TOP: the best (score, row) of the lane's stream of rows (lane
    // group lg of this wavefront's tiles, ascending)
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    const int64_t n_tiles = (a.rows + kTileRows - 1) / kTileRows;
    // grid form: this wavefront's tiles t0, t0 + stride, ...; persistent form:
    // each wavefront takes items (query block, kPersistTiles tiles) from the
    // work counter until it passes the item count (every wavefront ends
    // there), starting from an empty range so that the first pass takes an
    // item and loads its query block before any tile is scanned
    int64_t t = PERS ? 0 : (int64_t)blockIdx.x * 4 + wave, t_end = PERS ? 0 : n_tiles;
    const int64_t stride = PERS ? 1 : (int64_t)gridDim.x * 4;
    while (true) {
        if (PERS && t >= t_end) {
            if (MODE == MODE_COLLECT) {  // the pending marks belong to the current query block
                write_marks(a, pm, q, pb, prow0, lg);
#pragma unroll
                for (int g = 0; g < G; ++g) pm[g] = 0;
            }
            unsigned long long it = 0;
            if (lane == 0) it = atomicAdd(a.work, 1ull);
            const int64_t item = (int64_t)__shfl(it, 0, 64);
            if (item >= a.n_items) break;
            const int64_t y = item / a.tile_ranges, rg = item % a.tile_ranges;
            if (y != cur_y) {
                cur_y = y;
                load_queries(y);
            }
            t = rg * kPersistTiles;
            t_end = min(n_tiles, t + kPersistTiles);
        }
        if (!PERS && t >= n_tiles) break;
        const int64_t row0 = t * kTileRows;
        const uint8_t* pa = a.db + (row0 + li) * a.ld_db + lg * T::kLaneBytes;
        f32x4 acc[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[g][x] = f32x4{0.f, 0.f, 0.f, 0.f};
        typename T::F fa[2][4];
#pragma unroll
        for (int x = 0; x < 4; ++x) fa[0][x] = T::load(pa + (int64_t)16 * x * a.ld_db);
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int cur = c & 1, nxt = cur ^ 1;
            if (c + 1 < NK) {
#pragma unroll
                for (int x = 0; x < 4; ++x)
                    fa[nxt][x] = T::load(pa + (int64_t)16 * x * a.ld_db + (c + 1) * T::kChunkBytes);
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int x = 0; x < 4; ++x) acc[g][x] = T::mma(fa[cur][x], qb[g][c], acc[g][x]);
        }
        // lane holds query li of each group against rows row0 + 16x + 4lg + r
        // (ascending ids in this order)
        f32x4 rerr[4];  // FP8 collection: the errors of the lane's rows (the per-row band)
        if (PREC == MRC_PREC_FP8) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                if (MODE == MODE_COLLECT) rerr[x] = *(const f32x4*)(a.row_err + row0 + 16 * x + 4 * lg);
                const f32x4 sc = *(const f32x4*)(a.db_scale + row0 + 16 * x + 4 * lg);  // rows padded to 64
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[g][x][r] = acc[g][x][r] * sc[r] * qsc[g];
            }
        }
        if constexpr (MODE == MODE_TOP) {
            const int64_t rows_left = a.rows - row0;
            if (rows_left < kTileRows) {  // the last tile: rows past the end take no part
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (16 * (e >> 2) + 4 * lg + (e & 3) >= rows_left) acc[0][e >> 2][e & 3] = -INFINITY;
            }
            float tv = -INFINITY;  // the tile's best of the lane's 16 (the first of equals)
            int te = 0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float v = acc[0][e >> 2][e & 3];
                if (v > tv) {
                    tv = v;
                    te = e;
                }
            }
            if (tv > bv) {
                bv = tv;
                bi = (int)row0 + 16 * (te >> 2) + 4 * lg + (te & 3);
            }
        } else {
            uint32_t m[G];
            const uint32_t rm = tile_rowmask(a.rows - row0, lg);
#pragma unroll
            for (int g = 0; g < G; ++g)
                m[g] = PREC == MRC_PREC_FP8 ? tile_marks_rows(acc[g], thr[g], thrb[g], rerr, rm)
                                            : tile_marks(acc[g], thr[g], rm);
            write_marks(a, pm, q, pb, prow0, lg);
            reserve_marks(a, m, q, pb);
#pragma unroll
            for (int g = 0; g < G; ++g) pm[g] = m[g];
            prow0 = row0;
        }
        t += stride;
    }
    if (MODE == MODE_COLLECT) {
        write_marks(a, pm, q, pb, prow0, lg);
        return;
    }
    // stream (blockIdx.x * 4 + wave) * 4 + lg of each query: distinct rows in
    // every stream, so any 16 stream maxima are 16 distinct rows
    if (qvalid[0]) {
        const int64_t o = (int64_t)q[0] * ((int64_t)gridDim.x * 16) + (blockIdx.x * 4 + wave) * 4 + lg;
        a.part_s[o] = bv;
        a.part_id[o] = bi;
    }
}

// Per query: topk high-scoring rows of its `total` stream maxima, one
// workgroup per query: each thread takes the best of its share (the maximum
// of a coarser stream), then block_top picks the best topk of those 256
// (distinct rows, as any set of stream maxima).
__global__ __launch_bounds__(256) void k_query_merge(const float* __restrict__ part_s, const int32_t* __restrict__ part_id,
                                                     int64_t total, int topk, mrc_hit* __restrict__ out) {
    __shared__ float ss[4 * kTop];
    __shared__ int si[4 * kTop];
    const int q = blockIdx.x;
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int64_t e0 = threadIdx.x; e0 < total; e0 += 256 * 8) {  // 8 entries per round trip
        float v[8];
        int id[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = e0 + 256 * u;
            v[u] = e < total ? part_s[(int64_t)q * total + e] : -INFINITY;
            id[u] = e < total ? part_id[(int64_t)q * total + e] : 0x7fffffff;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (id[u] != 0x7fffffff && better(v[u], id[u], bv, bi)) {
                bv = v[u];
                bi = id[u];
            }
    }
    float ts[kTop];
    int ti[kTop];
#pragma unroll
    for (int p = 0; p < kTop; ++p) {
        ts[p] = p == 0 ? bv : -INFINITY;
        ti[p] = p == 0 ? bi : 0x7fffffff;
    }
    block_top(ts, ti, topk, ss, si, [&](int p, float bs, int b) {
        out[(int64_t)q * topk + p].id = b == 0x7fffffff ? -1 : b;
        out[(int64_t)q * topk + p].s = b == 0x7fffffff ? 0.f : bs;
        out[(int64_t)q * topk + p].flags = 0;
    });
}


// The plain FP32 chain acc = fmaf(q_c, r_c, acc), c = 0..kp-1, of a query
// held in LDS in natural order (zero past k) and a database row in the
// matrix-core layout (each 16-component block stored with its 4x4 sub-blocks
// transposed; zero past k): fmaf(0, 0, acc) is acc, so this is the chain
// over k. nb = kp / 16 blocks (even); a lane reads four row blocks per round
// trip (16-byte loads) and the matching query blocks from LDS (the same
// address in every lane), then consumes them in component order.
__device__ __forceinline__ float chain_blocks(const f32x4* qs, const f32x4* __restrict__ dr, int nb) {
    float acc = 0.f;
    int b = 0;
    for (; b + 4 <= nb; b += 4) {
        f32x4 blk[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) blk[j] = dr[4 * b + j];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            f32x4 qv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) qv[j] = qs[4 * (b + h) + j];
#pragma unroll
            for (int c = 0; c < 16; ++c) acc = __builtin_fmaf(qv[c >> 2][c & 3], blk[4 * h + (c & 3)][c >> 2], acc);
        }
    }
    if (b < nb) {  // the last two blocks
        f32x4 blk[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) blk[j] = dr[4 * b + j];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 qv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) qv[j] = qs[4 * (b + h) + j];
#pragma unroll
            for (int c = 0; c < 16; ++c) acc = __builtin_fmaf(qv[c >> 2][c & 3], blk[4 * h + (c & 3)][c >> 2], acc);
        }
    }
    return acc;
}

// Per query (one wavefront each): E16 = the smallest exact score of the 16
// first-pass rows (a row id of -1: fewer than 16 rows, E16 = -inf), the band
// b = e_q + e_r + e_q e_r + a (1 + e_q)(1 + e_r) + 2^-20 of the query's
// low-precision error e_q against a row's e_r (none for FP32 scores, which
// are the chain itself: db_err is NULL), and the collection threshold
// min(E16 - b, tau - b). With thr_b (FP8) the band is the row's own:
// b = A + B e_r, thr = min(E16, tau) - A and thr_b = B, and the collection
// tests score >= thr - B e_r; otherwise e_r is the database's largest error
// (db_err) and thr is the whole threshold. It also zeroes the
// query's candidate count, and block 0 the capacity signal and the
// persistent collection's work counter (when given), so the collection
// needs no clearing launches of its own.
__global__ __launch_bounds__(256) void k_query_e16(const mrc_hit* __restrict__ lp_top, int nq,
                                                   const float* __restrict__ qunit, int k,
                                                   const float* __restrict__ db_umfma, int kp, float tau,
                                                   const float* __restrict__ db_err, const float* __restrict__ q_err,
                                                   float acc_unit, float* __restrict__ thr, float* __restrict__ thr_b,
                                                   int32_t* __restrict__ ccount, unsigned long long* __restrict__ cap_word,
                                                   unsigned long long* __restrict__ work) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *cap_word = 0ull;
        if (work) *work = 0ull;
    }
    __shared__ f32x4 qs[4][256];  // each wavefront's query, kp <= 1024 components
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + w;
    if (q >= nq) return;  // (no workgroup barrier below: each wavefront on its own)
    float* qf = (float*)qs[w];
    for (int c = lane; c < kp; c += 64) qf[c] = c < k ? qunit[(int64_t)q * k + c] : 0.f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float v = INFINITY;
    if (lane < kTop) {
        const int64_t row = lp_top[(int64_t)q * kTop + lane].id;
        v = row < 0 ? -INFINITY : chain_blocks(qs[w], (const f32x4*)(db_umfma + row * kp), kp / 16);
    }
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    if (lane == 0) {
        // b = A + B e_db with A = e_q + a (1 + e_q) + 2^-20, B = 1 + e_q + a (1 + e_q)
        float A = 0.f, B = 0.f;
        if (db_err) {
            const float ei = q_err[q];
            A = ei + acc_unit * (1.f + ei) + 9.5367431640625e-07f;
            B = 1.f + ei + acc_unit * (1.f + ei);
        }
        if (thr_b) {  // per-row band: the collection subtracts B e_r itself
            thr[q] = fminf(v, tau) - A;
            thr_b[q] = B;
        } else {
            const float b = db_err ? A + B * *db_err : 0.f;
            thr[q] = fminf(v - b, tau - b);
        }
        ccount[q] = 0;
    }
}

// Exact decisions for the collected candidates of each query (one workgroup
// per query): the FP32 chain (chain_blocks) of the query and each candidate
// row, then the top list (block_top) and the hit count.
__global__ __launch_bounds__(256) void k_query_final(const int32_t* __restrict__ cand, const int32_t* __restrict__ ccount,
                                                     int cap, const float* __restrict__ qunit, int k,
                                                     const float* __restrict__ db_umfma, int kp, float tau, int topk,
                                                     mrc_hit* __restrict__ out, int32_t* __restrict__ n_hits,
                                                     int flags, unsigned long long* __restrict__ err) {
    __shared__ f32x4 qs[256];  // the query, kp <= 1024 components
    __shared__ float ss[4 * kTop];
    __shared__ int si[4 * kTop];
    __shared__ int sh[4];
    const int q = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nc = ccount[q];
    if (nc > cap) {  // (the same for the whole workgroup)
        if (threadIdx.x == 0) atomicOr(err, kErrQueryCap);
        return;
    }
    float* qf = (float*)qs;
    for (int c = threadIdx.x; c < kp; c += 256) qf[c] = c < k ? qunit[(int64_t)q * k + c] : 0.f;
    __syncthreads();
    float ts[kTop];
    int ti[kTop];
#pragma unroll
    for (int p = 0; p < kTop; ++p) {
        ts[p] = -INFINITY;
        ti[p] = 0x7fffffff;
    }
    int hits = 0;
    for (int e = threadIdx.x; e < nc; e += 256) {
        const int row = cand[(int64_t)q * cap + e];
        const float acc = chain_blocks(qs, (const f32x4*)(db_umfma + (int64_t)row * kp), kp / 16);
        hits += acc >= tau ? 1 : 0;
        if (better(acc, row, ts[kTop - 1], ti[kTop - 1])) top_insert(ts, ti, acc, row);
    }
    hits = mrc_dev::wave_sum(hits);
    if (lane == 0) sh[w] = hits;
    block_top(ts, ti, topk, ss, si, [&](int p, float bs, int bi) {
        out[(int64_t)q * topk + p].id = bi == 0x7fffffff ? -1 : bi;
        out[(int64_t)q * topk + p].s = bi == 0x7fffffff ? 0.f : bs;
        out[(int64_t)q * topk + p].flags = flags;
    });
    if (threadIdx.x == 0) n_hits[q] = sh[0] + sh[1] + sh[2] + sh[3];  // (written before block_top's barrier)
}


// Collection for large batches: the 4 wavefronts of a workgroup each hold G
// query groups and read the same 64-row database tile from LDS, so a tile
// comes from memory once per 64 G queries. Tiles are staged through
// registers into a second LDS buffer while the current one is used; one
// workgroup barrier per tile (every wavefront walks the same tiles).
constexpr int kLdsRowMax = 1024;  // bytes per database row this kernel stages

// Two wavefronts per SIMD (256 registers each) where the query fragments
// and accumulators leave room in that budget: one's products then overlap
// the other's marks, writes and barrier waits.
template <int PREC, int NK, int G>
constexpr int collect_waves() {
    return PREC != MRC_PREC_FP8 && G * NK * QT<PREC>::kLaneBytes / 4 + 16 * G <= 128 ? 2 : 1;
}

template <int PREC, int NK, int G, int MODE, bool PERS = false>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256), amdgpu_waves_per_eu(collect_waves<PREC, NK, G>())))
void k_query_collect_lds(ScanArgs a) {
    static_assert(!PERS || MODE == MODE_COLLECT, "the persistent form collects");
    using T = QT<PREC>;
    constexpr int ROW = NK * T::kChunkBytes;  // bytes per database row (= a.ld_db)
    constexpr int LD = ROW + 16;              // padded LDS row
    constexpr int PIECES = ROW / 16;          // 16-byte pieces per row
    constexpr int PER = kTileRows * PIECES / 256;
    static_assert(ROW <= kLdsRowMax && (kTileRows * PIECES) % 256 == 0, "tile staging shape");
    __shared__ __align__(16) uint8_t buf[2][kTileRows * LD];
    __shared__ int64_t s_item;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    typename T::F qb[G][NK];
    int q[G];
    bool qvalid[G];
    float qsc[G], thr[G], thrb[G];
    // the fragments of query block y (rows of the padded query arrays)
    auto load_queries = [&](int64_t y) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            q[g] = (int)(((y * 4 + wave) * G + g) * 16 + li);
            qvalid[g] = q[g] < a.nq;
            const uint8_t* pq = a.q + (int64_t)q[g] * a.ld_q + lg * T::kLaneBytes;
#pragma unroll
            for (int c = 0; c < NK; ++c) qb[g][c] = T::load(pq + c * T::kChunkBytes);
            qsc[g] = (PREC == MRC_PREC_FP8) ? a.q_scale[q[g]] : 1.f;
            const float th = qvalid[g] ? a.thr[q[g]] : INFINITY;
            thr[g] = th == th ? th : INFINITY;  // (no marks for a NaN threshold)
            thrb[g] = (PREC == MRC_PREC_FP8 && MODE == MODE_COLLECT && qvalid[g]) ? a.thr_b[q[g]] : 0.f;
        }
    };
    const int64_t n_tiles = (a.rows + kTileRows - 1) / kTileRows;
    // staging: a tile is 64 consecutive rows of ROW bytes; thread piece j is
    // the 16 bytes at tile offset 16 (threadIdx.x + 256 j), read through a
    // per-tile buffer descriptor (uniform base, one lane offset, the piece's
    // offset a constant)
    i32x4 st[PER];
    const int voff = 16 * threadIdx.x;
    auto stage_load = [&](int64_t tile) {
        const auto rs = __builtin_amdgcn_make_buffer_rsrc((void*)(a.db + tile * (kTileRows * ROW)), (short)0,
                                                          kTileRows * ROW, 0x00020000);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, 4096 * j, 0);
            __builtin_memcpy(&st[j], &v, 16);
        }
    };
    int cur = 0;
    int64_t cur_y = -1;
    // the previous tile's marks, their reserved slots and first row: written
    // after the next tile's staging loads have returned (the slot atomics,
    // issued before them, have too), so the atomics' latency hides behind a
    // tile of products
    uint32_t pm[G];
    int pb[G];
    int64_t prow0 = 0;
    // MODE_TOP: the best (score, row) of each lane's stream of rows (lane
    // group lg of this workgroup's tiles, ascending)
    float bv[G];
    int bi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        pm[g] = 0;
        pb[g] = 0;
        bv[g] = -INFINITY;
        bi[g] = 0x7fffffff;
    }
    // grid form: one pass over tiles blockIdx.x, + gridDim.x, ... of query
    // block blockIdx.y; persistent form: items (query block, kPersistTiles
    // tiles) taken by the workgroup from the work counter until it passes the
    // item count (the same value for every wavefront: all leave together)
    while (true) {
        int64_t t, t_end, step;
        if (PERS) {
            if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.work, 1ull);
            __syncthreads();
            const int64_t item = s_item;
            __syncthreads();
            if (item >= a.n_items) break;
            const int64_t y = item / a.tile_ranges, rg = item % a.tile_ranges;
            if (y != cur_y) {
                cur_y = y;
                load_queries(y);
            }
            t = rg * kPersistTiles;
            t_end = min(n_tiles, t + kPersistTiles);
            step = 1;
        } else {
            load_queries(blockIdx.y);
            t = blockIdx.x;
            t_end = n_tiles;
            step = gridDim.x;
        }
    if (t < t_end) {
        stage_load(t);  // (the database's rows are padded to whole tiles)
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int pc = threadIdx.x + 256 * j, r = pc / PIECES, c = pc % PIECES;
            *(i32x4*)(&buf[cur][r * LD + c * 16]) = st[j];
        }
    }
    __syncthreads();
    for (; t < t_end; t += step) {
        const int64_t tn = t + step;
        const bool more = tn < t_end;
        // the next tile's loads overlap this tile's products (without a next
        // tile: this one again, valid and unused, so that nothing branches
        // around the staged values)
        stage_load(more ? tn : t);
        // (the scheduler keeps the loads here, a tile of products ahead of
        // their use, and the marks below ahead of the pending writes)
        __builtin_amdgcn_sched_barrier(0);
        const int64_t row0 = t * kTileRows;
        const uint8_t* pa = &buf[cur][li * LD + lg * T::kLaneBytes];
        f32x4 acc[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[g][x] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            typename T::F fa[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) fa[x] = T::load(pa + 16 * x * LD + c * T::kChunkBytes);
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int x = 0; x < 4; ++x) acc[g][x] = T::mma(fa[x], qb[g][c], acc[g][x]);
        }
        f32x4 rerr[4];  // FP8 collection: the errors of the lane's rows (the per-row band)
        if (PREC == MRC_PREC_FP8) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                if (MODE == MODE_COLLECT) rerr[x] = *(const f32x4*)(a.row_err + row0 + 16 * x + 4 * lg);
                const f32x4 sc = *(const f32x4*)(a.db_scale + row0 + 16 * x + 4 * lg);
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[g][x][r] = acc[g][x][r] * sc[r] * qsc[g];
            }
        }
        auto stage_store = [&]() {  // (after the last tile: written, never read)
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int pc = threadIdx.x + 256 * j, r = pc / PIECES, c = pc % PIECES;
                *(i32x4*)(&buf[cur ^ 1][r * LD + c * 16]) = st[j];
            }
        };
        if constexpr (MODE == MODE_COLLECT) {
            uint32_t m[G];
            const uint32_t rm = tile_rowmask(a.rows - row0, lg);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                m[g] = PREC == MRC_PREC_FP8 ? tile_marks_rows(acc[g], thr[g], thrb[g], rerr, rm)
                                            : tile_marks(acc[g], thr[g], rm);
                asm volatile("" : "+v"(m[g]));  // (computed here, not sunk to its use)
            }
            __builtin_amdgcn_sched_barrier(0);
            stage_store();
            write_marks(a, pm, q, pb, prow0, lg);
            reserve_marks(a, m, q, pb);
#pragma unroll
            for (int g = 0; g < G; ++g) pm[g] = m[g];
            prow0 = row0;
        } else {
            const int64_t rows_left = a.rows - row0;
            if (rows_left < kTileRows) {  // the last tile: rows past the end take no part
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        if (16 * (e >> 2) + 4 * lg + (e & 3) >= rows_left) acc[g][e >> 2][e & 3] = -INFINITY;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // the tile's best of the lane's 16 (the first of equals: rows
                // ascend with e), then against the stream's best so far
                float tv = -INFINITY;
                int te = 0;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const float v = acc[g][e >> 2][e & 3];
                    if (v > tv) {
                        tv = v;
                        te = e;
                    }
                }
                if (tv > bv[g]) {
                    bv[g] = tv;
                    bi[g] = (int)row0 + 16 * (te >> 2) + 4 * lg + (te & 3);
                }
            }
            stage_store();
        }
        __syncthreads();
        cur ^= 1;
    }
        if constexpr (MODE == MODE_COLLECT) {  // the pending marks belong to this query block
            write_marks(a, pm, q, pb, prow0, lg);
#pragma unroll
            for (int g = 0; g < G; ++g) pm[g] = 0;
        }
        if (!PERS) break;
    }
    if constexpr (MODE == MODE_TOP) {
        // stream blockIdx.x * 4 + lg of each query: distinct rows in every
        // stream, so any 16 stream maxima are 16 distinct rows
        const int64_t streams = (int64_t)gridDim.x * 4;
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (q[g] < a.nq) {
                const int64_t o = (int64_t)q[g] * streams + blockIdx.x * 4 + lg;
                a.part_s[o] = bv[g];
                a.part_id[o] = bi[g];
            }
    }
}

// pers: the persistent form (grid = the workgroups resident at once, at most
// a.n_items), else `grid`
template <int PREC, int G, int NK, int MODE>
bool launch_collect_lds_nk(mrc_ctx* ctx, bool pers, const ScanArgs& a, dim3 grid, hipStream_t s) {
    if constexpr (NK * QT<PREC>::kChunkBytes <= kLdsRowMax && G * NK * QT<PREC>::kLaneBytes / 4 <= 128) {
        if constexpr (MODE == MODE_COLLECT) {
            if (pers) {
                const void* kf = (const void*)k_query_collect_lds<PREC, NK, G, MODE, true>;
                const int64_t pg = persistent_grid(ctx, kf, 256, a.n_items);
                hipLaunchKernelGGL((k_query_collect_lds<PREC, NK, G, MODE, true>), dim3((unsigned)pg), dim3(256), 0,
                                   s, a);
                return true;
            }
        }
        hipLaunchKernelGGL((k_query_collect_lds<PREC, NK, G, MODE>), grid, dim3(256), 0, s, a);
        return true;
    } else {
        return false;
    }
}

// false: no instantiation for this shape (the caller uses k_query_scan)
template <int PREC, int G, int MODE = MODE_COLLECT>
bool launch_collect_lds(mrc_ctx* ctx, bool pers, int nk, const ScanArgs& a, dim3 grid, hipStream_t s) {
#define MRC_Q(c) case c: return launch_collect_lds_nk<PREC, G, c, MODE>(ctx, pers, a, grid, s);
    if constexpr (PREC == MRC_PREC_FP32) {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) MRC_Q(12) MRC_Q(16) default: return false; }
    } else if constexpr (PREC == MRC_PREC_BF16) {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) MRC_Q(10) MRC_Q(12) MRC_Q(16) default: return false; }
    } else {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) default: return false; }
    }
#undef MRC_Q
}

// G query groups per wavefront when their fragments fit in 128 registers.
// pers (collection only): the persistent form, items per wavefront.
template <int PREC, int MODE, int G, int NK>
bool launch_scan_nk(mrc_ctx* ctx, bool pers, const ScanArgs& a, dim3 grid, hipStream_t s) {
    if constexpr (G == 1 || G * NK * QT<PREC>::kLaneBytes / 4 <= 128) {
        if constexpr (MODE == MODE_COLLECT) {
            if (pers) {
                const void* kf = (const void*)k_query_scan<PREC, NK, MODE, G, true>;
                const int64_t pg = persistent_grid(ctx, kf, 256, ceil_div(a.n_items, 4));
                hipLaunchKernelGGL((k_query_scan<PREC, NK, MODE, G, true>), dim3((unsigned)pg), dim3(256), 0, s, a);
                return true;
            }
        }
        hipLaunchKernelGGL((k_query_scan<PREC, NK, MODE, G>), grid, dim3(256), 0, s, a);
        return true;
    } else {
        return false;
    }
}

template <int PREC, int MODE, int G>
mrc_status launch_scan(mrc_ctx* ctx, int nk, const ScanArgs& a, dim3 grid, hipStream_t s, bool pers = false) {
    bool ok = false;
#define MRC_Q(c) case c: ok = launch_scan_nk<PREC, MODE, G, c>(ctx, pers, a, grid, s); break;
    if constexpr (PREC == MRC_PREC_FP32) {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) MRC_Q(12) MRC_Q(16) MRC_Q(24) MRC_Q(32) default: break; }
    } else if constexpr (PREC == MRC_PREC_BF16) {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) MRC_Q(10) MRC_Q(12) MRC_Q(16) default: break; }
    } else {
        switch (nk) { MRC_Q(2) MRC_Q(4) MRC_Q(6) MRC_Q(8) default: break; }
    }
#undef MRC_Q
    if (!ok) return fail(MRC_E_INVAL, "query: unsupported k");
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

template <int PREC>
mrc_status launch_scan_any(mrc_ctx* ctx, int mode, int g, int nk, const ScanArgs& a, dim3 grid, hipStream_t s,
                           bool pers = false) {
    if (mode == MODE_TOP) return launch_scan<PREC, MODE_TOP, 1>(ctx, nk, a, grid, s);
    if (g == 4) return launch_scan<PREC, MODE_COLLECT, 4>(ctx, nk, a, grid, s, pers);
    if (g == 2) return launch_scan<PREC, MODE_COLLECT, 2>(ctx, nk, a, grid, s, pers);
    return launch_scan<PREC, MODE_COLLECT, 1>(ctx, nk, a, grid, s, pers);
}

}  // namespace

namespace mrc {

// Database layouts (shared with the insert path).
DbLayout db_layout(int32_t k) {
    DbLayout L;
    L.kp = 16 * mfma_chunks(k);
    L.ldb = lowp_steps(MRC_PREC_BF16, k) * 32;
    L.ld8 = lowp_steps(MRC_PREC_FP8, k) * 128;
    return L;
}

mrc_status run_query(mrc_ctx* ctx, const mrc_db* db, int64_t rows, const mrc_model* m, const mrc_docs* qd,
                     int32_t topk, float tau, int32_t precision, mrc_hit* topk_out, int32_t* n_hits, hipStream_t s) {
    const int64_t nq = qd->n_docs;
    const int k = db->k;
    const DbLayout L = db_layout(k);
    const int64_t nq_pad = ceil_div(nq > 0 ? nq : 1, 256) * 256;  // whole query blocks of every scan
    // sign and normalise the queries into every layout the scan needs
    void *sig, *unit, *umf, *qb, *q8, *qsc, *qerr;
    MRC_TRY(scratch(ctx, "q_sig", (size_t)nq_pad * k * 4, &sig));
    MRC_TRY(scratch(ctx, "q_unit", (size_t)nq_pad * k * 4, &unit));
    MRC_TRY(scratch(ctx, "q_umfma", (size_t)nq_pad * L.kp * 4, &umf));
    MRC_TRY(scratch(ctx, "q_bf16", (size_t)nq_pad * L.ldb * 2, &qb));
    MRC_TRY(scratch(ctx, "q_fp8", (size_t)nq_pad * L.ld8, &q8));
    MRC_TRY(scratch(ctx, "q_scale", (size_t)nq_pad * 4, &qsc));
    MRC_TRY(scratch(ctx, "q_err", (size_t)2 * nq_pad * 4, &qerr));
    MRC_TRY(launch_sign(ctx, m, qd, (float*)sig, nullptr, s));
    NormLayout o{(float*)unit, k, (uint16_t*)qb, L.ldb, (uint8_t*)q8, L.ld8, (float*)qsc, (float*)qerr, nq_pad,
                 (float*)umf, L.kp, nq_pad};
    MRC_TRY(launch_normalise_rows(ctx, (const float*)sig, nq, k, o, s));
    if (nq == 0) return MRC_OK;
    const bool fp32 = precision == MRC_PREC_FP32, bf = precision == MRC_PREC_BF16;
    if ((bf && !db->d_bf16) || (precision == MRC_PREC_FP8 && !db->d_fp8))
        return fail(MRC_E_STATE, "mrc_query: the database holds no copy in this precision");
    ScanArgs a{};
    a.nq = (int)nq;
    a.tau = tau;
    int nk, lane_regs;
    if (fp32) {
        a.db = (const uint8_t*)db->d_unit;
        a.ld_db = L.kp * 4;
        a.q = (const uint8_t*)umf;
        nk = L.kp / 16;
        lane_regs = 4;
    } else {
        a.db = bf ? (const uint8_t*)db->d_bf16 : db->d_fp8;
        a.ld_db = bf ? L.ldb * 2 : L.ld8;
        a.db_scale = db->d_scale;
        a.q = bf ? (const uint8_t*)qb : (const uint8_t*)q8;
        a.q_scale = (const float*)qsc;
        nk = bf ? L.ldb / 32 : L.ld8 / 128;
        lane_regs = bf ? 4 : 8;
    }
    a.ld_q = a.ld_db;
    auto scan = [&](int mode, int g, dim3 grid, bool pers = false) {
        if (fp32) return launch_scan_any<MRC_PREC_FP32>(ctx, mode, g, nk, a, grid, s, pers);
        if (bf) return launch_scan_any<MRC_PREC_BF16>(ctx, mode, g, nk, a, grid, s, pers);
        return launch_scan_any<MRC_PREC_FP8>(ctx, mode, g, nk, a, grid, s, pers);
    };
    auto grid_for_rows = [&](int64_t r, int64_t groups) {
        const int64_t tiles = std::max<int64_t>(1, ceil_div(r, kTileRows));
        const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, groups), ceil_div(tiles, 4)));
        return dim3(gx, (unsigned)groups);
    };
    ScopedTimer tm(ctx, "query", s);
    // pass 1: 16 high-scoring rows of a prefix of the database for each
    // query (the 16 best of the per-stream maxima: distinct rows, nearly
    // always the prefix's own 16 best), their exact scores (a lower bound for
    // the whole: any 16 rows' smallest exact score is at most the exact 16th
    // best), and the collection threshold thr = min(E16 - b, tau - b) (b = 0
    // for FP32 scores, which are the chain itself). FP8's band is wide: its
    // first pass takes the whole database, so that E16 is as high as it can be
    const int64_t sample = precision == MRC_PREC_FP8
                               ? rows
                               : std::min<int64_t>(rows, std::max<int64_t>(kPrefixMin, ceil_div(rows, 16)));
    // G query groups per wavefront in the collection (and the LDS-shared
    // first pass): as many as the batch fills and 128 registers hold
    int g = nq <= 16 ? 1 : nq <= 48 ? 2 : 4;
    while (g > 1 && g * nk * lane_regs > 128) g /= 2;
    // batches above 64 queries: the LDS-shared forms (64 g queries per
    // workgroup, all four wavefronts on the same tiles) where they are built
    const bool lds_form = nq > 64;
    auto lds_launch = [&](int mode, bool pers, dim3 grid) {
        if (fp32)
            return mode == MODE_TOP
                       ? (g == 4 ? launch_collect_lds<MRC_PREC_FP32, 4, MODE_TOP>(ctx, pers, nk, a, grid, s)
                          : g == 2 ? launch_collect_lds<MRC_PREC_FP32, 2, MODE_TOP>(ctx, pers, nk, a, grid, s)
                                   : launch_collect_lds<MRC_PREC_FP32, 1, MODE_TOP>(ctx, pers, nk, a, grid, s))
                       : (g == 4 ? launch_collect_lds<MRC_PREC_FP32, 4>(ctx, pers, nk, a, grid, s)
                          : g == 2 ? launch_collect_lds<MRC_PREC_FP32, 2>(ctx, pers, nk, a, grid, s)
                                   : launch_collect_lds<MRC_PREC_FP32, 1>(ctx, pers, nk, a, grid, s));
        if (bf)
            return mode == MODE_TOP
                       ? (g == 4 ? launch_collect_lds<MRC_PREC_BF16, 4, MODE_TOP>(ctx, pers, nk, a, grid, s)
                          : g == 2 ? launch_collect_lds<MRC_PREC_BF16, 2, MODE_TOP>(ctx, pers, nk, a, grid, s)
                                   : launch_collect_lds<MRC_PREC_BF16, 1, MODE_TOP>(ctx, pers, nk, a, grid, s))
                       : (g == 4 ? launch_collect_lds<MRC_PREC_BF16, 4>(ctx, pers, nk, a, grid, s)
                          : g == 2 ? launch_collect_lds<MRC_PREC_BF16, 2>(ctx, pers, nk, a, grid, s)
                                   : launch_collect_lds<MRC_PREC_BF16, 1>(ctx, pers, nk, a, grid, s));
        return mode == MODE_TOP
                   ? (g == 4 ? launch_collect_lds<MRC_PREC_FP8, 4, MODE_TOP>(ctx, pers, nk, a, grid, s)
                      : g == 2 ? launch_collect_lds<MRC_PREC_FP8, 2, MODE_TOP>(ctx, pers, nk, a, grid, s)
                               : launch_collect_lds<MRC_PREC_FP8, 1, MODE_TOP>(ctx, pers, nk, a, grid, s))
                   : (g == 4 ? launch_collect_lds<MRC_PREC_FP8, 4>(ctx, pers, nk, a, grid, s)
                      : g == 2 ? launch_collect_lds<MRC_PREC_FP8, 2>(ctx, pers, nk, a, grid, s)
                               : launch_collect_lds<MRC_PREC_FP8, 1>(ctx, pers, nk, a, grid, s));
    };
    auto lds_grid = [&](int64_t r) {
        const int64_t tiles = std::max<int64_t>(1, ceil_div(r, kTileRows));
        const int64_t groups = ceil_div(nq, 64 * g);
        return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, groups), tiles)), (unsigned)groups);
    };
    // the first pass's partial entries per query: top lists of kTop per
    // workgroup (k_query_scan), or one stream maximum per lane group and
    // workgroup (the LDS-shared form: 4 gx streams, each over distinct rows)
    const dim3 g1 = grid_for_rows(sample, ceil_div(nq, 16));
    const dim3 g1l = lds_grid(sample);
    const int64_t per_q = std::max<int64_t>((int64_t)g1.x * kTop, (int64_t)g1l.x * 4);
    void *ps, *pi, *thr, *cand, *cc, *mtop;
    MRC_TRY(scratch(ctx, "q_part_s", (size_t)nq * per_q * 4, &ps));
    MRC_TRY(scratch(ctx, "q_part_id", (size_t)nq * per_q * 4, &pi));
    MRC_TRY(scratch(ctx, "q_thr", (size_t)nq * 4, &thr));
    MRC_TRY(scratch(ctx, "q_top_lp", (size_t)nq * kTop * sizeof(mrc_hit), &mtop));
    a.rows = sample;
    a.part_s = (float*)ps;
    a.part_id = (int32_t*)pi;
    int64_t entries = (int64_t)g1.x * kTop;
    if (lds_form && lds_launch(MODE_TOP, false, g1l)) {
        MRC_HIP_TRY(ctx, hipGetLastError());
        entries = (int64_t)g1l.x * 4;
    } else {
        MRC_TRY(scan(MODE_TOP, 1, g1));
    }
    hipLaunchKernelGGL(k_query_merge, dim3((unsigned)nq), dim3(256), 0, s, (const float*)ps, (const int32_t*)pi,
                       entries, kTop, (mrc_hit*)mtop);
    // (no nominal floor under the band: every candidate is rescored exactly,
    // so the band only has to keep each row whose exact score reaches the
    // threshold)
    const bool pers = ctx->scan_form == MRC_SCAN_PERSISTENT;
    void* work = nullptr;
    if (pers) MRC_TRY(scratch(ctx, "q_work", 256, &work));
    MRC_TRY(scratch(ctx, "q_ccount", (size_t)ceil_div(nq, 2) * 8, &cc));  // (whole words: cleared as such)
    unsigned long long* cap_word = (unsigned long long*)(ctx->d_flags + kQueryCapWord);
    // FP8: the band of each (query, row) pair from the row's own error (the
    // database keeps every row's), so well-quantised rows get a narrower
    // window; BF16 errors barely vary between rows: the largest serves
    const bool per_row = precision == MRC_PREC_FP8;
    void* thrb = nullptr;
    if (per_row) MRC_TRY(scratch(ctx, "q_thr_b", (size_t)nq * 4, &thrb));
    hipLaunchKernelGGL(k_query_e16, dim3((unsigned)ceil_div(nq, 4)), dim3(256), 0, s, (const mrc_hit*)mtop, (int)nq,
                       (const float*)unit, k, db->d_unit, L.kp, tau,
                       fp32 ? (const float*)nullptr : db->d_errmax + (bf ? 0 : 1),
                       (const float*)qerr + (bf ? 0 : nq_pad), fp32 ? 0.f : lowp_acc_unit(precision, k), (float*)thr,
                       (float*)thrb, (int32_t*)cc, cap_word, (unsigned long long*)work);
    a.thr_b = (const float*)thrb;
    a.row_err = per_row ? db->d_err + db->cap_pad : nullptr;
    MRC_HIP_TRY(ctx, hipGetLastError());
    // pass 2: every row at or above the threshold, G query groups per
    // wavefront, then exact decisions; grow the per-query capacity on overflow
    a.rows = rows;
    const dim3 g2 = lds_form ? lds_grid(rows) : grid_for_rows(rows, ceil_div(nq, 16 * g));
    // persistent form: items of kPersistTiles tiles per query block, taken
    // from a counter in context scratch (zeroed before each collection)
    a.work = (unsigned long long*)work;
    a.tile_ranges = ceil_div(std::max<int64_t>(1, ceil_div(rows, kTileRows)), kPersistTiles);
    auto collect = [&]() -> mrc_status {
        if (lds_form) {
            a.n_items = ceil_div(nq, 64 * g) * a.tile_ranges;
            if (lds_launch(MODE_COLLECT, pers, g2)) {
                MRC_HIP_TRY(ctx, hipGetLastError());
                return MRC_OK;
            }
        }
        a.n_items = ceil_div(nq, 16 * g) * a.tile_ranges;
        return scan(MODE_COLLECT, g, grid_for_rows(rows, ceil_div(nq, 16 * g)), pers);
    };
    int cap = 2048;
    auto it = ctx->scratch.find("q_cand");
    if (it != ctx->scratch.end()) cap = std::max<int64_t>(cap, (int64_t)(it->second.second / 4 / nq));
    for (int attempt = 0; attempt < 3; ++attempt) {
        MRC_TRY(scratch(ctx, "q_cand", (size_t)nq * cap * 4, &cand));
        if (attempt > 0) {  // (the first collection's counters were zeroed by k_query_e16)
            MRC_TRY(clear_words(ctx, (int64_t*)cc, ceil_div(nq, 2), s));
            MRC_TRY(clear_words(ctx, (int64_t*)cap_word, 1, s));
            if (pers) MRC_TRY(clear_words(ctx, (int64_t*)work, 1, s));
        }
        a.thr = (const float*)thr;
        a.cand = (int32_t*)cand;
        a.ccount = (int32_t*)cc;
        a.cap = cap;
        MRC_TRY(collect());
        hipLaunchKernelGGL(k_query_final, dim3((unsigned)nq), dim3(256), 0, s, (const int32_t*)cand,
                           (const int32_t*)cc, cap, (const float*)unit, k, db->d_unit, L.kp, tau, topk, topk_out,
                           n_hits, fp32 ? 0 : 1, cap_word);
        MRC_HIP_TRY(ctx, hipGetLastError());
        // word 0 holds the signing pass's input errors (the scans ran on
        // whatever the early-returning document kernels left, in bounds);
        // the capacity signal has a word of its own
        MRC_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, (kQueryCapWord + 1) * sizeof(int64_t),
                                        hipMemcpyDeviceToHost, s));
        MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
        if (ctx->h_flags[0] & (kErrOffsets | kErrToken | kErrDocLen))
            return fail(MRC_E_INVAL, "mrc_query: malformed offsets, token ids or document lengths");
        ctx->query_attempts = attempt + 1;
        if (!(ctx->h_flags[kQueryCapWord] & kErrQueryCap)) return MRC_OK;
        std::vector<int32_t> counts(nq);
        MRC_HIP_TRY(ctx, hipMemcpy(counts.data(), cc, (size_t)nq * 4, hipMemcpyDeviceToHost));
        cap = std::max(cap, *std::max_element(counts.begin(), counts.end()));
    }
    return fail(MRC_E_NOMEM, "mrc_query: candidate capacity");
}

}  // namespace mrc
