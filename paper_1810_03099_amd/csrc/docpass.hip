// Per-document passes over the token CSR (Section 4: the TF-IDF vector of a
// document and its cosine against each of the k reference parts).
//
// A document's tokens become term counts in a hash table: in LDS for
// documents up to kMediumMax tokens (one wavefront per short document, one
// 256-thread workgroup per medium document), and in a per-workgroup [V] count
// array in global memory for longer documents. The passes are
//  * COUNT (model build): the distinct terms of each document and their
//    counts, written at the document's token offset; document frequencies are
//    then a histogram of those lists (k_df_hist / k_df_sum, LDS counters per
//    vocabulary slice, no global atomics);
//  * SIGN: the signature straight from the table;
//  * CSR: unit TF-IDF weights for the exact-cosine comparator.
// k_sign_counts signs from the COUNT lists, so a corpus that built the model
// is signed without hashing it again.
//
// Signing needs, per document d and part j,
//   num_j = sum over terms t of part j of tf_t * c_t,   c_t = idf_t * rho_t,
//   |w_d|^2 = sum over terms t of (tf_t * idf_t)^2,
// and sig_dj = num_j / (|w_d| |r_j|). Both sums are formed exactly in integer
// fixed point: c * 2^32 is an integer for the weights that occur (c >= 1), and
// for idf in [1, 32), idf = m * 2^(E-23) with integer m < 2^24, so
// (tf * idf)^2 * 2^46 = (tf * m)^2 * 2^(2E) is an integer; a 128-bit sum of
// these is exact for documents up to kMaxDocLen tokens. The results are thus
// independent of the order of summation: every pass, and any batch a document
// is part of, gives the same bits. |w_d| is the square root of that exact sum,
// rounded once to float64.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "exact_sums.h"

using namespace mrc;
using namespace mrc_exact;

namespace {

constexpr int kBlock = 256;
constexpr int kEmpty = -1;
constexpr int kHistSlice = 65536;  // vocabulary ids per LDS histogram slice (16-bit counters)
constexpr int kHistMaxSlices = 8;  // above this, df is counted with global atomics instead

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int hash_slot(int t, int log2_slots) {
    return (int)(((unsigned)t * 0x9E3779B1u) >> (32 - log2_slots));
}

template <int TEAM>
__device__ __forceinline__ void team_sync() {
    if constexpr (TEAM == 64) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    } else {
        __syncthreads();
    }
}

// Sum over a team (one wavefront, or the 4 wavefronts of a block); exact.
template <int TEAM>
__device__ __forceinline__ u128 team_sum(u128 v, u128* red) {
    v = wave_sum_u128(v);
    if constexpr (TEAM == 64) {
        return v;
    } else {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        u128 r = red[0];
#pragma unroll
        for (int i = 1; i < TEAM / 64; ++i) r += red[i];
        __syncthreads();
        return r;
    }
}

struct PassArgs {
    // SIGN / CSR
    const TermInfo* tinfo;
    const double* rinv;
    int k;
    int vocab;         // entries of tinfo
    int ref_idf;       // 1: rho_t = idf_t, so c_t = idf^2
    float* sig;
    float* norm;
    // COUNT: distinct terms and counts of document d at [off[d], off[d] + nnz[d])
    // (the document's remaining slots up to off[d + 1] are not written)
    int32_t* cnt_term;
    int32_t* cnt_tf;
    int32_t* cnt_nnz;
    // CSR: unit TF-IDF weights w = tf * idf / |w_d| of each distinct term.
    // Ranks below H go to the dense head matrix (matrix-core layout, ld ldh);
    // the others are listed at the document's token offset (ent_*), counted
    // per rank in pcount, and their number stored in nnz_tail.
    const int32_t* rank_of;
    const int32_t* term_at;  // SIGN from count lists: rank -> term (the hot-term cache)
    int H;
    int ldh;
    float* wh;
    int32_t* ent_rank;
    float* ent_w;
    int32_t* nnz_tail;
    uint32_t* pcount;
};

enum { MODE_COUNT = 0, MODE_SIGN = 1, MODE_CSR = 2 };

__device__ __forceinline__ float ref_coef(const PassArgs& a, float idf) { return a.ref_idf ? idf * idf : idf; }

// Emit one distinct term of document d (MODE_COUNT / MODE_CSR). `pos` is the
// entry's index in the document's list (MODE_COUNT).
template <int MODE>
__device__ __forceinline__ void emit_term(const PassArgs& a, int64_t d, int64_t o, int t, unsigned tf, double nrm,
                                          int pos, int* tcount) {
    if constexpr (MODE == MODE_COUNT) {
        a.cnt_term[o + pos] = t;
        a.cnt_tf[o + pos] = (int32_t)tf;
    } else {
        const float w = (float)((double)tf * (double)a.tinfo[t].idf / nrm);
        const int r = a.rank_of[t];
        if (r < a.H) {
            a.wh[d * a.ldh + mrc_dev::mfma_col(r)] = w;
        } else {
            const int e = atomicAdd(tcount, 1);
            a.ent_rank[o + e] = r;
            a.ent_w[o + e] = w;
            atomicAdd(&a.pcount[r - a.H], 1u);
        }
    }
}

__device__ __forceinline__ void write_signature(const PassArgs& a, int64_t d, const unsigned long long* bins,
                                                double nrm, int tid, int team) {
    float* out = a.sig + d * a.k;
    for (int j = tid; j < a.k; j += team) {
        const double v = nrm > 0.0 ? mrc_dev::unfixed32(bins[j]) * a.rinv[j] / nrm : 0.0;
        out[j] = (float)v;
    }
    if (tid == 0 && a.norm) a.norm[d] = (float)nrm;
}

// Offsets check before any token is read: offsets[0] = 0, non-decreasing,
// offsets[n] <= n_tokens, no document longer than kMaxDocLen. Sets error bits;
// the document kernels then return at once. With `lists` set, it also lists
// the documents above kShortMax tokens by length class (lists[c n ..), counts
// in err[kClassCount + c], one atomic per wavefront and class), so that each
// listed pass visits only its own documents.
__global__ __launch_bounds__(256) void k_validate_offsets(const int64_t* __restrict__ off, int64_t n,
                                                          int64_t n_tokens, unsigned long long* __restrict__ err,
                                                          int32_t* __restrict__ lists) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false, too_long = false;
    int cls = -1;
    if (d <= n) {
        const int64_t o = off[d];
        if (d == 0) bad = o != 0;
        else bad = o < off[d - 1];
        if (d == n) {
            bad = bad || o > n_tokens || o < 0;
        } else {
            const int64_t L = off[d + 1] - o;
            cls = L <= kShortMax ? -1 : L <= kMidMax ? 0 : L <= kMedMax ? 1 : L <= kMediumMax ? 2 : 3;
            too_long = L > kMaxDocLen;
        }
    }
    if (bad) atomicOr(err, kErrOffsets);
    if (too_long) atomicOr(err, kErrDocLen);
    if (lists == nullptr) return;  // (kernel argument: the whole grid returns)
    // a wavefront's members of each class take consecutive slots of the
    // workgroup's share (LDS), which one global atomic per class reserves
    __shared__ unsigned int wg_cnt[kClasses];
    __shared__ unsigned long long wg_base[kClasses];
    if (threadIdx.x < kClasses) wg_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int lane = __lane_id();
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    unsigned int off_c[kClasses];
#pragma unroll
    for (int c = 0; c < kClasses; ++c) {
        const unsigned long long m = __ballot(cls == c);
        unsigned int o = 0u;
        if (m != 0 && lane == __ffsll((long long)m) - 1) o = atomicAdd(&wg_cnt[c], (unsigned int)__popcll(m));
        off_c[c] = m != 0 ? __shfl(o, __ffsll((long long)m) - 1, 64) + (unsigned int)__popcll(m & below) : 0u;
    }
    __syncthreads();
    if (threadIdx.x < kClasses)
        wg_base[threadIdx.x] =
            wg_cnt[threadIdx.x] ? atomicAdd(err + kClassCount + threadIdx.x, (unsigned long long)wg_cnt[threadIdx.x]) : 0ull;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kClasses; ++c)
        if (cls == c) lists[(int64_t)c * n + (int64_t)(wg_base[c] + off_c[c])] = (int32_t)d;
}

__global__ void k_clear_words(int64_t* __restrict__ p, int n) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ bool pass_disabled(const unsigned long long* err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kErrOffsets | kErrDocLen);
}

// LDS layout of one team: bins u64[kpad] | keys i32[SLOTS] | cnt i32[SLOTS] |
// used u16[SLOTS/2] (a document has at most SLOTS/2 tokens) | nused i32
// (+pad) | red (u128[4])
__host__ __device__ constexpr size_t team_lds_bytes(int kpad, int slots) {
    return (size_t)kpad * 8 + (size_t)slots * 9 + 16 + 64;
}

// Short (list == nullptr: every document with L <= hi_len) or listed (one
// length class of k_validate_offsets, *count of them) documents.
template <int MODE, int TEAM, int LOG2_SLOTS, int MAXPER>
__global__ __launch_bounds__(kBlock) void k_doc_lds(const int64_t* __restrict__ off, int64_t n_docs,
                                                    int lo_len, int hi_len,
                                                    const int32_t* __restrict__ tok,
                                                    int32_t V, PassArgs a, unsigned long long* __restrict__ err,
                                                    const int32_t* __restrict__ list,
                                                    const unsigned long long* __restrict__ count) {
    constexpr int SLOTS = 1 << LOG2_SLOTS;
    constexpr int TEAMS = kBlock / TEAM;
    extern __shared__ __align__(16) unsigned char smem[];
    const int kpad = MODE == MODE_SIGN ? ((a.k + 1) & ~1) : 0;
    const size_t tbytes = team_lds_bytes(kpad, SLOTS);
    const int team = threadIdx.x / TEAM;
    const int tid = threadIdx.x % TEAM;
    unsigned char* base = smem + (size_t)team * tbytes;
    unsigned long long* bins = (unsigned long long*)base;
    int* keys = (int*)(base + (size_t)kpad * 8);
    int* cnt = keys + SLOTS;
    unsigned short* used = (unsigned short*)(cnt + SLOTS);
    int* nused = (int*)(used + SLOTS / 2);
    u128* red = (u128*)(base + tbytes - 64);

    if (pass_disabled(err)) return;
    for (int s = tid; s < SLOTS; s += TEAM) {
        keys[s] = kEmpty;
        cnt[s] = 0;
    }
    for (int j = tid; j < kpad; j += TEAM) bins[j] = 0ull;
    if (tid == 0) *nused = 0;
    team_sync<TEAM>();

    const int64_t n_items = list ? (int64_t)__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : n_docs;
    for (int64_t item = (int64_t)blockIdx.x * TEAMS + team; item < n_items; item += (int64_t)gridDim.x * TEAMS) {
        const int64_t d = list ? (int64_t)list[item] : item;
        const int64_t o = off[d];
        const int64_t L64 = off[d + 1] - o;
        if (L64 <= lo_len || L64 > hi_len) {
            if (!(lo_len == 0 && L64 == 0)) continue;
        }
        const int L = (int)L64;
        // all of this thread's tokens (and their term data) are loaded before
        // the table is touched, so the loads overlap
        int t_r[MAXPER];
#pragma unroll
        for (int r = 0; r < MAXPER; ++r) {
            const int p = tid + r * TEAM;
            t_r[r] = p < L ? tok[o + p] : kEmpty;
        }
        TermInfo ti_r[MAXPER];
        if constexpr (MODE == MODE_CSR) {
#pragma unroll
            for (int r = 0; r < MAXPER; ++r)
                ti_r[r] = (unsigned)t_r[r] < (unsigned)V ? a.tinfo[t_r[r]] : TermInfo{1.f, -1};
        }
        // insert: the first probes of all of this thread's tokens go out
        // together, then each token probes on (linear) until its slot holds
        // it; the counts are added without waiting, and the slots this
        // thread claimed join the used list with one reservation
        int slot_r[MAXPER], prev_r[MAXPER];
        bool ok_r[MAXPER];
#pragma unroll
        for (int r = 0; r < MAXPER; ++r) {
            ok_r[r] = tid + r * TEAM < L;
            if (ok_r[r] && (unsigned)t_r[r] >= (unsigned)V) {
                atomicOr(err, kErrToken);
                ok_r[r] = false;
            }
            slot_r[r] = ok_r[r] ? hash_slot(t_r[r], LOG2_SLOTS) : 0;
        }
#pragma unroll
        for (int r = 0; r < MAXPER; ++r) prev_r[r] = ok_r[r] ? atomicCAS(&keys[slot_r[r]], kEmpty, t_r[r]) : kEmpty;
        uint32_t won = 0;
#pragma unroll
        for (int r = 0; r < MAXPER; ++r) {
            if (!ok_r[r]) {
                slot_r[r] = -1;
                continue;
            }
            int h = slot_r[r], prev = prev_r[r];
            while (prev != kEmpty && prev != t_r[r]) {
                h = (h + 1) & (SLOTS - 1);
                prev = atomicCAS(&keys[h], kEmpty, t_r[r]);
            }
            slot_r[r] = h;
            if (prev == kEmpty) won |= 1u << r;
        }
#pragma unroll
        for (int r = 0; r < MAXPER; ++r)
            if (slot_r[r] >= 0) atomicAdd(&cnt[slot_r[r]], 1);
        if (won) {
            int u = atomicAdd(nused, __popc(won));
#pragma unroll
            for (int r = 0; r < MAXPER; ++r)
                if (won & (1u << r)) used[u++] = (unsigned short)slot_r[r];
        }
        team_sync<TEAM>();
        double nrm = 0.0;
        if constexpr (MODE == MODE_SIGN) {
            // once per distinct term (not per occurrence): its term data, its
            // part sum tf x coefficient and its norm term (tf idf)^2, the
            // same integers as the per-occurrence sums
            const int nu0 = *nused;
            u128 nacc = 0;
            for (int u0 = tid; u0 < nu0; u0 += 4 * TEAM) {
                int tt[4];
                uint32_t tf[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int u = u0 + q * TEAM;
                    const int sl = u < nu0 ? (int)used[u] : -1;
                    tt[q] = sl >= 0 ? keys[sl] : -1;
                    tf[q] = sl >= 0 ? (uint32_t)cnt[sl] : 0u;
                }
                TermInfo ti[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) ti[q] = tt[q] >= 0 ? a.tinfo[tt[q]] : TermInfo{1.f, -1};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (tt[q] < 0) continue;
                    if (ti[q].part >= 0)
                        atomicAdd(&bins[ti[q].part], (unsigned long long)tf[q] * mrc_dev::fixed32(ref_coef(a, ti[q].idf)));
                    nacc += term_sq_fixed(tf[q], ti[q].idf);
                }
            }
            team_sync<TEAM>();  // (the part sums complete before they are read)
            nrm = norm_from_fixed(team_sum<TEAM>(nacc, red));
        } else if constexpr (MODE == MODE_CSR) {
            u128 nacc = 0;
#pragma unroll
            for (int r = 0; r < MAXPER; ++r)
                if (slot_r[r] >= 0) nacc += occ_sq_fixed((uint32_t)cnt[slot_r[r]], ti_r[r].idf);
            nrm = norm_from_fixed(team_sum<TEAM>(nacc, red));
        }
        if constexpr (MODE == MODE_SIGN) write_signature(a, d, bins, nrm, tid, TEAM);
        const int nu = *nused;
        if constexpr (MODE == MODE_COUNT) {
            for (int u = tid; u < nu; u += TEAM) {
                const int sl = used[u];
                emit_term<MODE_COUNT>(a, d, o, keys[sl], (unsigned)cnt[sl], 0.0, u, nullptr);
            }
            if (tid == 0) a.cnt_nnz[d] = nu;
        } else if constexpr (MODE == MODE_CSR) {
            int* tcount = (int*)red;
            team_sync<TEAM>();
            if (tid == 0) *tcount = 0;
            team_sync<TEAM>();
            for (int u = tid; u < nu; u += TEAM) {
                const int sl = used[u];
                emit_term<MODE_CSR>(a, d, o, keys[sl], (unsigned)cnt[sl], nrm, u, tcount);
            }
            team_sync<TEAM>();
            if (tid == 0) a.nnz_tail[d] = *tcount;
        }
        team_sync<TEAM>();
        for (int u = tid; u < nu; u += TEAM) {
            const int s = used[u];
            keys[s] = kEmpty;
            cnt[s] = 0;
        }
        for (int j = tid; j < kpad; j += TEAM) bins[j] = 0ull;
        team_sync<TEAM>();
        if (tid == 0) *nused = 0;
        team_sync<TEAM>();
    }
}

// Long documents (the last length class of k_validate_offsets): a [V]
// uint32 count table per workgroup in global memory (all zero between
// documents).
// Counts go first to a small LDS cache of terms (one slot per hashed id, the
// first term to claim a slot keeps it for the document), the rest to the
// global table; a long Zipf document repeats its hottest terms thousands of
// times, and same-address global atomics serialise in L2 where LDS ones are
// cheap. The cache is flushed into the global table (and, when signing, into
// the part sums: count x the term's fixed-point coefficient, the same integer
// as the sum of one coefficient per occurrence) before the norm pass.
constexpr int kLongUnroll = 8;
constexpr int kLongThreads = 1024;  // a workgroup per long document: 16 wavefronts
constexpr int kHotLog2 = 11;        // 2,048 cached terms (16 KB of LDS)
template <int MODE>
__global__ __launch_bounds__(kLongThreads) void k_doc_global(const int64_t* __restrict__ off, int32_t V,
                                                       const int32_t* __restrict__ tok, PassArgs a,
                                                       uint32_t* __restrict__ tables,
                                                       unsigned long long* __restrict__ err,
                                                       const int32_t* __restrict__ list,
                                                       const unsigned long long* __restrict__ count) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* bins = (unsigned long long*)smem;
    const int kpad = MODE == MODE_SIGN ? ((a.k + 1) & ~1) : 0;
    u128* red = (u128*)(smem + (size_t)kpad * 8);
    int* tcount = (int*)(red + kLongThreads / 64);
    __shared__ int hot_key[1 << kHotLog2];
    __shared__ uint32_t hot_cnt[1 << kHotLog2];
    uint32_t* cnt = tables + (size_t)blockIdx.x * (size_t)V;
    const int tid = threadIdx.x;
    if (pass_disabled(err)) return;
    for (int j = tid; j < kpad; j += kLongThreads) bins[j] = 0ull;
    for (int j = tid; j < (1 << kHotLog2); j += kLongThreads) {
        hot_key[j] = -1;
        hot_cnt[j] = 0u;
    }
    __syncthreads();
    const int64_t n_items = (int64_t)__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t d = list[item];
        const int64_t o = off[d];
        const int64_t L = off[d + 1] - o;
        // kLongUnroll tokens per thread and round: their loads, then their
        // term-table loads, then their atomics (one memory latency per round
        // rather than two per token)
        for (int64_t p0 = tid; p0 < L; p0 += (int64_t)kLongThreads * kLongUnroll) {
            int t[kLongUnroll];
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const int64_t p = p0 + (int64_t)u * kLongThreads;
                t[u] = p < L ? tok[o + p] : -1;
                if (p < L && (unsigned)t[u] >= (unsigned)V) {
                    atomicOr(err, kErrToken);
                    t[u] = -1;
                }
            }
            TermInfo ti[kLongUnroll];
            if constexpr (MODE == MODE_SIGN) {
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u) ti[u] = t[u] >= 0 ? a.tinfo[t[u]] : TermInfo{0.f, -1};
            }
            int held[kLongUnroll];
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u)
                held[u] = t[u] >= 0 ? atomicCAS(&hot_key[hash_slot(t[u], kHotLog2)], -1, t[u]) : -2;
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                if (t[u] < 0) continue;
                if (held[u] == -1 || held[u] == t[u]) {  // the slot is this term's
                    atomicAdd(&hot_cnt[hash_slot(t[u], kHotLog2)], 1u);
                    continue;
                }
                atomicAdd(&cnt[t[u]], 1u);
                if constexpr (MODE == MODE_SIGN) {
                    if (ti[u].part >= 0) atomicAdd(&bins[ti[u].part], mrc_dev::fixed32(ref_coef(a, ti[u].idf)));
                }
            }
        }
        __syncthreads();
        // flush the cached counts (and their part sums) into the global table
        for (int j = tid; j < (1 << kHotLog2); j += kLongThreads) {
            const int key = hot_key[j];
            if (key < 0) continue;
            const uint32_t c = hot_cnt[j];
            atomicAdd(&cnt[key], c);
            if constexpr (MODE == MODE_SIGN) {
                const TermInfo ti = a.tinfo[key];
                if (ti.part >= 0)
                    atomicAdd(&bins[ti.part], (unsigned long long)c * mrc_dev::fixed32(ref_coef(a, ti.idf)));
            }
            hot_key[j] = -1;
            hot_cnt[j] = 0u;
        }
        __threadfence();
        __syncthreads();
        double nrm = 0.0;
        if constexpr (MODE != MODE_COUNT) {
            u128 acc = 0;
            for (int64_t p0 = tid; p0 < L; p0 += (int64_t)kLongThreads * kLongUnroll) {
                int t[kLongUnroll];
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u) {
                    const int64_t p = p0 + (int64_t)u * kLongThreads;
                    t[u] = p < L ? tok[o + p] : -1;
                    if ((unsigned)t[u] >= (unsigned)V) t[u] = -1;
                }
                unsigned tf[kLongUnroll];
                float idf[kLongUnroll];
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u) {
                    tf[u] = t[u] >= 0 ? __hip_atomic_load(&cnt[t[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
                    idf[u] = t[u] >= 0 ? a.tinfo[t[u]].idf : 0.f;
                }
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u)
                    if (t[u] >= 0) acc += occ_sq_fixed(tf[u], idf[u]);
            }
            nrm = norm_from_fixed(team_sum<kLongThreads>(acc, red));
        }
        if constexpr (MODE == MODE_SIGN) {
            write_signature(a, d, bins, nrm, tid, kLongThreads);
        } else {
            // each distinct term once: the occurrence that swaps its count out emits it
            if (tid == 0) *tcount = 0;
            __syncthreads();
            for (int64_t p = tid; p < L; p += kLongThreads) {
                const int t = tok[o + p];
                if ((unsigned)t >= (unsigned)V) continue;
                const unsigned tf = atomicExch(&cnt[t], 0u);
                if (tf > 0) {
                    if constexpr (MODE == MODE_COUNT) {
                        emit_term<MODE_COUNT>(a, d, o, t, tf, 0.0, atomicAdd(tcount, 1), nullptr);
                    } else {
                        emit_term<MODE_CSR>(a, d, o, t, tf, nrm, 0, tcount);
                    }
                }
            }
            __syncthreads();
            if constexpr (MODE == MODE_COUNT) {
                if (tid == 0) a.cnt_nnz[d] = *tcount;
            } else {
                if (tid == 0) a.nnz_tail[d] = *tcount;
            }
        }
        __syncthreads();
        for (int64_t p0 = tid; p0 < L; p0 += (int64_t)kLongThreads * kLongUnroll) {
            int t[kLongUnroll];
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u) {
                const int64_t p = p0 + (int64_t)u * kLongThreads;
                t[u] = p < L ? tok[o + p] : -1;
            }
#pragma unroll
            for (int u = 0; u < kLongUnroll; ++u)
                if ((unsigned)t[u] < (unsigned)V) __hip_atomic_store(&cnt[t[u]], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int j = tid; j < kpad; j += kLongThreads) bins[j] = 0ull;
        __threadfence();
        __syncthreads();
    }
}

// Long documents over a small vocabulary (V <= kDirectMaxV, e.g. the 27^3
// character-3-gram space): one 1024-thread workgroup per document with a
// direct [V] count array in LDS (no hashing, no global atomics). The tokens
// are counted with LDS atomics (SIGN: the part sums per occurrence, as in
// every pass); then one scan of the array visits each distinct term once
// (its count, its norm term, its list entry), clearing it for the next
// document.
constexpr int kDirectThreads = 1024;
constexpr int kDirectMaxV = 32768;  // 128 KB of counts

template <int MODE>
__global__ __launch_bounds__(kDirectThreads) void k_doc_direct(const int64_t* __restrict__ off, int32_t V,
                                                               const int32_t* __restrict__ tok, PassArgs a,
                                                               unsigned long long* __restrict__ err,
                                                               const int32_t* __restrict__ list,
                                                               const unsigned long long* __restrict__ count) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* cnt = (uint32_t*)smem;                                          // [V]
    unsigned long long* bins = (unsigned long long*)(smem + (((size_t)V * 4 + 15) & ~(size_t)15));
    const int kpad = MODE == MODE_SIGN ? ((a.k + 1) & ~1) : 0;
    u128* red = (u128*)(bins + kpad);                                         // [16]
    int* tcount = (int*)(red + kDirectThreads / 64);
    const int tid = threadIdx.x;
    if (pass_disabled(err)) return;
    for (int t = tid; t < V; t += kDirectThreads) cnt[t] = 0u;
    for (int j = tid; j < kpad; j += kDirectThreads) bins[j] = 0ull;
    __syncthreads();
    const int64_t n_items = (int64_t)__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int64_t d = list[item];
        const int64_t o = off[d];
        const int64_t L = off[d + 1] - o;
        for (int64_t p = tid; p < L; p += kDirectThreads) {
            const int t = tok[o + p];
            if ((unsigned)t >= (unsigned)V) {
                atomicOr(err, kErrToken);
                continue;
            }
            atomicAdd(&cnt[t], 1u);
            if constexpr (MODE == MODE_SIGN) {
                const TermInfo ti = a.tinfo[t];
                if (ti.part >= 0) atomicAdd(&bins[ti.part], mrc_dev::fixed32(ref_coef(a, ti.idf)));
            }
        }
        if (tid == 0) *tcount = 0;
        __syncthreads();
        double nrm = 0.0;
        if constexpr (MODE != MODE_COUNT) {
            u128 acc = 0;
            for (int t = tid; t < V; t += kDirectThreads) {
                const uint32_t c = cnt[t];
                if (c) acc += term_sq_fixed(c, a.tinfo[t].idf);
            }
            nrm = norm_from_fixed(team_sum<kDirectThreads>(acc, red));
        }
        if constexpr (MODE == MODE_SIGN) write_signature(a, d, bins, nrm, tid, kDirectThreads);
        for (int t = tid; t < V; t += kDirectThreads) {
            const uint32_t c = cnt[t];
            if (c == 0u) continue;
            if constexpr (MODE == MODE_COUNT) emit_term<MODE_COUNT>(a, d, o, t, c, 0.0, atomicAdd(tcount, 1), nullptr);
            else if constexpr (MODE == MODE_CSR) emit_term<MODE_CSR>(a, d, o, t, c, nrm, 0, tcount);
            cnt[t] = 0u;
        }
        __syncthreads();
        if constexpr (MODE == MODE_COUNT) {
            if (tid == 0) a.cnt_nnz[d] = *tcount;
        } else if constexpr (MODE == MODE_CSR) {
            if (tid == 0) a.nnz_tail[d] = *tcount;
        }
        for (int j = tid; j < kpad; j += kDirectThreads) bins[j] = 0ull;
        __syncthreads();
    }
}

// ------------------------------------------------------------ df from counts

// One workgroup per (vocabulary slice, document range): the distinct terms of
// the range's documents (entries [off[d], off[d] + nnz[d]) of the count lists)
// that fall inside the slice are counted in LDS, two 16-bit counters per word
// (a term is listed at most once per document and a range holds at most 65535
// documents), and the slice's counts are written to partial[range][...].
// One wavefront per document: the entries of its next document and the list
// bounds of the one after are requested before the current one is counted, so
// the load latency overlaps the LDS atomics.
constexpr int kHistThreads = 1024;
constexpr int kHistPer = 8;  // entries per lane and pass (512 per wavefront pass: one pass for most documents)
__global__ __launch_bounds__(kHistThreads) void k_df_hist(const int64_t* __restrict__ off, int64_t n,
                                                          const int32_t* __restrict__ term,
                                                          const int32_t* __restrict__ nnz, int groups,
                                                          uint32_t* __restrict__ partial, int64_t words,
                                                          const unsigned long long* __restrict__ err) {
    constexpr int U = kHistPer, W = kHistThreads / 64;
    __shared__ uint32_t h[kHistSlice / 2];
    if (pass_disabled(err)) return;
    const int slice = blockIdx.x / groups, g = blockIdx.x % groups;
    const int t0 = slice * kHistSlice;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kHistSlice / 2; i += kHistThreads) h[i] = 0u;
    __syncthreads();
    const int64_t d_lo = n * g / groups, d_hi = n * (g + 1) / groups;
    // list bounds of document d (past the range: the range's last document, no entries)
    auto bounds = [&](int64_t d, int64_t& o, int& m) {
        const int64_t dl = min(d, d_hi - 1);
        o = off[dl];
        m = d < d_hi ? nnz[dl] : 0;
    };
    // entries e0 .. e0 + 64 U - 1 (-1 past the end)
    auto load = [&](int64_t o, int m, int e0, int32_t (&v)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * 64 + lane;
            v[u] = e < m ? term[o + e] : -1;
        }
    };
    auto count = [&](const int32_t (&v)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned t = (unsigned)(v[u] - t0);
            if (v[u] >= 0 && t < (unsigned)kHistSlice) atomicAdd(&h[t >> 1], 1u << ((t & 1u) * 16u));
        }
    };
    const int64_t d0 = d_lo + wave;
    if (d0 < d_hi) {
        int64_t o_c, o_n, o_nn;
        int m_c, m_n, m_nn;
        int32_t v_c[U], v_n[U];
        bounds(d0, o_c, m_c);
        bounds(d0 + W, o_n, m_n);
        load(o_c, m_c, 0, v_c);
        for (int64_t d = d0; d < d_hi; d += W) {
            bounds(d + 2 * W, o_nn, m_nn);
            load(o_n, m_n, 0, v_n);
            count(v_c);
            for (int e0 = 64 * U; e0 < m_c; e0 += 64 * U) {  // longer lists (rare)
                int32_t v_x[U];
                load(o_c, m_c, e0, v_x);
                count(v_x);
            }
            o_c = o_n, m_c = m_n, o_n = o_nn, m_n = m_nn;
#pragma unroll
            for (int u = 0; u < U; ++u) v_c[u] = v_n[u];
        }
    }
    __syncthreads();
    uint32_t* dst = partial + (size_t)g * (size_t)words + (size_t)(t0 / 2);
    for (int i = threadIdx.x; i < kHistSlice / 2; i += kHistThreads) dst[i] = h[i];
}

// df = the sum of the partial counts: 64 words per wavefront (coalesced), the
// 4 wavefronts of a block over interleaved quarters of the ranges.
__global__ __launch_bounds__(256) void k_df_sum(const uint32_t* __restrict__ partial, int groups, int64_t words,
                                                int32_t V, uint32_t* __restrict__ df) {
    __shared__ uint32_t red[2][4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * 64 + lane;
    uint32_t lo = 0, hi = 0;
    if (w < words) {
        for (int g = wv; g < groups; g += 4) {
            const uint32_t x = partial[(size_t)g * (size_t)words + (size_t)w];
            lo += x & 0xFFFFu;
            hi += x >> 16;
        }
    }
    red[0][wv][lane] = lo;
    red[1][wv][lane] = hi;
    __syncthreads();
    if (wv == 0 && w < words) {
        lo = red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
        hi = red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane];
        if (2 * w < V) df[2 * w] = lo;
        if (2 * w + 1 < V) df[2 * w + 1] = hi;
    }
}

// Large vocabularies: one atomic per distinct (document, term).
__global__ __launch_bounds__(256) void k_df_atomic(const int64_t* __restrict__ off, int64_t n,
                                                   const int32_t* __restrict__ term,
                                                   const int32_t* __restrict__ nnz, uint32_t* __restrict__ df,
                                                   const unsigned long long* __restrict__ err) {
    if (pass_disabled(err)) return;
    const int lane = threadIdx.x & 63;
    for (int64_t d = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64; d < n; d += (int64_t)gridDim.x * 4) {
        const int64_t o = off[d];
        const int m = nnz[d];
        for (int e = lane; e < m; e += 64) atomicAdd(&df[term[o + e]], 1u);
    }
}

// ------------------------------------------------------- sign from counts

// One wavefront per document over its distinct-term list (same exact sums as
// the hash passes, so the same signature bits).

// c * 2^32 for a float 1 <= c < 2^24 (the value mrc_dev::fixed32 gives, from
// the bits alone).
__device__ __forceinline__ unsigned long long fixed32_ge1(float c) {
    const uint32_t b = __float_as_uint(c);
    return (unsigned long long)((b & 0x7FFFFFu) | 0x800000u) << ((b >> 23) - 127u + 9u);
}

// Entries per lane and chunk of k_sign_counts (a list is signed 512 entries
// at a time).
constexpr int kSignPer = 8;
constexpr int kSignChunk = 64 * kSignPer;

// One chunk of a document's count list as this lane holds it (entry
// 64 r + lane of the chunk) and the term information gathered for it.
struct SignStage {
    int t[kSignPer];
    int f[kSignPer];
    TermInfo ti[kSignPer];
    int i;     // document index in the block (>= cnt: none)
    int m;     // entries in this chunk
    int last;  // the document's last chunk
};

// Each wavefront signs a contiguous block of documents (their offsets and
// list lengths held one per lane, 64 at a time), chunk by chunk (512 list
// entries), through a three-stage software pipeline: while chunk j is summed,
// the term information of chunk j + 1 is being gathered and the entries of
// chunk j + 2 are being loaded. The three stage buffers rotate by unrolling
// (no register copies, which would wait for every load in flight); the loads
// are buffer loads with a wavefront-uniform descriptor per chunk (lanes past
// its entries read 0: term 0 with count 0), so no address registers are
// formed per chunk and the waits the compiler places stay exact. Exact sums
// as in every signing pass: per chunk, |w_d|^2 as three 64-bit partial sums
// (at most 512 entries: each stays below 2^59) reduced over the wavefront
// and added to the document's 128-bit total; the part sums in 64-bit fixed
// point in LDS.
// HOT: 16 wavefronts per workgroup (one workgroup per CU) share an LDS copy of
// the term information of the most frequent terms (the first kHotSlots ranks,
// direct-mapped by a multiplicative hash of the term id; a slot keeps one of
// the terms that map to it): entries of those terms read LDS instead of
// gathering from the V-entry table, whose divergent requests bound the pass.
constexpr int kCacheLog2 = 13, kHotSlots = 1 << kCacheLog2;
constexpr int64_t kSignHotMinDocs = 65536;
__device__ __forceinline__ uint32_t hot_slot(int t) { return ((uint32_t)t * 2654435761u) >> (32 - kCacheLog2); }

template <bool HOT>
__global__ __launch_bounds__(HOT ? 1024 : 256) void k_sign_counts(const int64_t* __restrict__ off, int64_t n,
                                                     const int32_t* __restrict__ term,
                                                     const int32_t* __restrict__ tfv,
                                                     const int32_t* __restrict__ nnz, PassArgs a, int64_t per_wave,
                                                     const unsigned long long* __restrict__ err) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int R = kSignPer;
    constexpr int W = HOT ? 16 : 4;  // wavefronts per workgroup
    const int kpad = (a.k + 1) & ~1;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const uint32_t lane4 = 4u * (uint32_t)lane;
    unsigned long long* bins = (unsigned long long*)smem + (size_t)wave * kpad;
    double* rinv = (double*)smem + (size_t)W * kpad;  // 1 / |r_j|, staged once per workgroup
    int32_t* hot_tag = (int32_t*)(rinv + kpad);
    TermInfo* hot_info = (TermInfo*)(hot_tag + kHotSlots);
    if (pass_disabled(err)) return;
    for (int j = lane; j < kpad; j += 64) bins[j] = 0ull;
    for (int j = threadIdx.x; j < a.k; j += 64 * W) rinv[j] = a.rinv[j];
    if constexpr (HOT) {
        for (int j = threadIdx.x; j < kHotSlots; j += 64 * W) hot_tag[j] = -1;
        __syncthreads();
        const int top = min(kHotSlots, a.vocab);
        for (int r = threadIdx.x; r < top; r += 64 * W) {
            const int t = a.term_at[r];
            const uint32_t sl = hot_slot(t);
            if (atomicCAS(&hot_tag[sl], -1, t) == -1) hot_info[sl] = a.tinfo[t];
        }
    }
    __syncthreads();
    const int64_t first = ((int64_t)blockIdx.x * W + wave) * per_wave;
    const int64_t end = min(first + per_wave, n);
    // term table (ids < 2^24: byte offsets fit 32 bits)
    const __amdgpu_buffer_rsrc_t tbl =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.tinfo, (short)0, (int)(8 * a.vocab), 0x00020000);

    for (int64_t base = first; base < end; base += 64) {
        const int cnt = (int)min((int64_t)64, end - base);
        // this block's list offsets and lengths, one document per lane
        const int64_t dl = base + min(lane, cnt - 1);
        const int64_t o_l = off[dl];
        const int m_l = lane < cnt ? nnz[dl] : 0;
        auto o_at = [&](int i) {
            const int ii = min(i, cnt - 1);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)o_l, ii);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)o_l >> 32), ii);
            return (int64_t)(((uint64_t)hi << 32) | lo);
        };
        auto m_at = [&](int i) { return i < cnt ? __builtin_amdgcn_readlane(m_l, min(i, 63)) : 0; };
        // issue the loads of chunk c of document i (i >= cnt: nothing to load)
        auto load_chunk = [&](SignStage& b, int i, int c) {
            const int m = m_at(i);
            const int mc = i < cnt ? min(kSignChunk, m - kSignChunk * c) : 0;
            b.i = i;
            b.m = mc;
            b.last = kSignChunk * (c + 1) >= m;
            const int64_t o = (i < cnt ? o_at(i) : 0) + (int64_t)kSignChunk * c;
            const __amdgpu_buffer_rsrc_t rt =
                __builtin_amdgcn_make_buffer_rsrc((void*)(term + o), (short)0, 4 * mc, 0x00020000);
            const __amdgpu_buffer_rsrc_t rf =
                __builtin_amdgcn_make_buffer_rsrc((void*)(tfv + o), (short)0, 4 * mc, 0x00020000);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                b.t[r] = (int)__builtin_amdgcn_raw_buffer_load_b32(rt, (int)(lane4 + 256 * r), 0, 0);
                b.f[r] = (int)__builtin_amdgcn_raw_buffer_load_b32(rf, (int)(lane4 + 256 * r), 0, 0);
            }
        };
        auto gather = [&](SignStage& b) {
            if constexpr (HOT) {
                bool hit[R];
#pragma unroll
                for (int r = 0; r < R; ++r) hit[r] = hot_tag[hot_slot(b.t[r])] == b.t[r];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (hit[r]) {
                        b.ti[r] = hot_info[hot_slot(b.t[r])];
                    } else {
                        const auto v = __builtin_amdgcn_raw_buffer_load_b64(tbl, (int)(8u * (uint32_t)b.t[r]), 0, 0);
                        b.ti[r].idf = __uint_as_float(v[0]);
                        b.ti[r].part = (int)v[1];
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const auto v = __builtin_amdgcn_raw_buffer_load_b64(tbl, (int)(8u * (uint32_t)b.t[r]), 0, 0);
                    b.ti[r].idf = __uint_as_float(v[0]);
                    b.ti[r].part = (int)v[1];
                }
            }
        };
        // the chunk after (i, c)
        auto next = [&](int& i, int& c) {
            if (kSignChunk * (c + 1) < m_at(i)) {
                ++c;
            } else {
                ++i;
                c = 0;
            }
        };
        u128 total = 0;  // |w_d|^2 2^46 of the current document so far
        auto sum_chunk = [&](const SignStage& b) {
            // (tf idf)^2 = A^2 2^-46 with A = tf (mantissa(idf) << exponent(idf)) < 2^50, split at
            // bit 25 into three partial products below 2^50
            uint64_t s2 = 0, s1 = 0, s0 = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t f = (uint32_t)b.f[r];  // 0 past the chunk's entries
                const uint64_t A = (uint64_t)f * idf_scaled(b.ti[r].idf);
                const uint32_t hi = (uint32_t)(A >> 25), lo = (uint32_t)A & 0x1FFFFFFu;
                s2 += (uint64_t)hi * hi;
                s1 += (uint64_t)hi * lo;
                s0 += (uint64_t)lo * lo;
                if (r * 64 + lane < b.m && b.ti[r].part >= 0)
                    atomicAdd(&bins[b.ti[r].part], (unsigned long long)f * fixed32_ge1(ref_coef(a, b.ti[r].idf)));
            }
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) {
                s2 += __shfl_xor((unsigned long long)s2, sh, 64);
                s1 += __shfl_xor((unsigned long long)s1, sh, 64);
                s0 += __shfl_xor((unsigned long long)s0, sh, 64);
            }
            total += ((u128)s2 << 50) + ((u128)s1 << 26) + (u128)s0;
            if (!b.last) return;
            const int64_t d = base + b.i;
            const double nrm = norm_from_fixed(total);
            total = 0;
            // one wavefront owns `bins`, and LDS executes its operations in
            // order: compiler-only fences keep the next chunks' loads in flight
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            float* out = a.sig + d * a.k;
            for (int j = lane; j < a.k; j += 64)
                out[j] = (float)(nrm > 0.0 ? mrc_dev::unfixed32(bins[j]) * rinv[j] / nrm : 0.0);
            if (lane == 0 && a.norm) a.norm[d] = (float)nrm;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            for (int j = lane; j < kpad; j += 64) bins[j] = 0ull;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        };

        // the block's metadata is read here, before any list load is issued,
        // so no wait inside the loop is for it
        int i1 = 0, c1 = 0;
        next(i1, c1);
        int i2 = i1, c2 = c1;
        next(i2, c2);
        __builtin_amdgcn_sched_barrier(0);
        SignStage b0, b1, b2;
        load_chunk(b0, 0, 0);
        load_chunk(b1, i1, c1);
        gather(b0);
        // (i2, c2): the chunk whose loads are issued next
        while (true) {
            load_chunk(b2, i2, c2);
            next(i2, c2);
            gather(b1);
            __builtin_amdgcn_sched_barrier(0);  // the requests above go out before any wait
            sum_chunk(b0);
            if (b1.i >= cnt) break;
            load_chunk(b0, i2, c2);
            next(i2, c2);
            gather(b2);
            __builtin_amdgcn_sched_barrier(0);
            sum_chunk(b1);
            if (b2.i >= cnt) break;
            load_chunk(b1, i2, c2);
            next(i2, c2);
            gather(b0);
            __builtin_amdgcn_sched_barrier(0);
            sum_chunk(b2);
            if (b0.i >= cnt) break;
        }
    }
}

// ------------------------------------------------------------------- driver

constexpr int kShortTeam = 64, kShortLog2 = 10, kShortPer = kShortMax / 64;      // 1024 slots
constexpr int kMidTeam = 256, kMidLog2 = 12, kMidPer = kMidMax / 256;            // 4096 slots, 4 workgroups per CU
constexpr int kMedTeam = 256, kMedLog2 = 13, kMedPer = kMedMax / 256;            // 8192 slots
constexpr int kBigTeam = 256, kBigLog2 = 14, kBigPer = kMediumMax / 256;         // 16384 slots, 1 workgroup per CU
static_assert((1 << kShortLog2) >= 2 * kShortMax, "short table load factor");
static_assert((1 << kMidLog2) >= 2 * kMidMax, "mid table load factor");
static_assert((1 << kMedLog2) >= 2 * kMedMax, "medium table load factor");
static_assert((1 << kBigLog2) >= 2 * kMediumMax, "large table load factor");
static_assert((1 << kBigLog2) <= 65536, "slot indices are stored as uint16");

int grid_for(int64_t n_items_upper, int teams_per_block, int cap) {
    int64_t g = ceil_div(n_items_upper, teams_per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <int MODE>
mrc_status run_docpass(mrc_ctx* ctx, const mrc_docs* docs, int32_t V, const PassArgs& a, hipStream_t s,
                       const char* name) {
    const int64_t n = docs->n_docs;
    unsigned long long* err = (unsigned long long*)ctx->d_flags;
    void* lists = nullptr;
    if (n > 0) MRC_TRY(scratch(ctx, "doc_lists", (size_t)kClasses * (size_t)n * sizeof(int32_t), &lists));
    MRC_TRY(launch_validate_offsets(ctx, docs, s, (int32_t*)lists));
    if (n == 0) return MRC_OK;
    auto list = [&](int c) { return (const int32_t*)lists + (size_t)c * (size_t)n; };
    auto count = [&](int c) { return (const unsigned long long*)err + kClassCount + c; };
    const int kpad = MODE == MODE_SIGN ? ((a.k + 1) & ~1) : 0;
    ScopedTimer tm(ctx, name, s);
    {
        const size_t lds = team_lds_bytes(kpad, 1 << kShortLog2) * (kBlock / kShortTeam);
        const int grid = grid_for(n, kBlock / kShortTeam, 256 * 8);
        hipLaunchKernelGGL((k_doc_lds<MODE, kShortTeam, kShortLog2, kShortPer>), dim3(grid), dim3(kBlock),
                           lds, s, docs->offsets, n, 0, kShortMax, docs->tokens, V, a, err, nullptr, nullptr);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    {
        // the listed classes: up to kMidMax tokens with 4096-slot tables (four
        // workgroups per CU), up to kMedMax with 8192 slots, up to kMediumMax
        // with 16384 (147 KB: one workgroup per CU)
        const size_t lds_mid = team_lds_bytes(kpad, 1 << kMidLog2);
        hipLaunchKernelGGL((k_doc_lds<MODE, kMidTeam, kMidLog2, kMidPer>), dim3(grid_for(n, 1, 256 * 4)), dim3(kBlock),
                           lds_mid, s, docs->offsets, n, kShortMax, kMidMax, docs->tokens, V, a, err, list(0), count(0));
        MRC_HIP_TRY(ctx, hipGetLastError());
        const size_t lds = team_lds_bytes(kpad, 1 << kMedLog2);
        hipLaunchKernelGGL((k_doc_lds<MODE, kMedTeam, kMedLog2, kMedPer>), dim3(grid_for(n, 1, 256 * 2)), dim3(kBlock),
                           lds, s, docs->offsets, n, kMidMax, kMedMax, docs->tokens, V, a, err, list(1), count(1));
        MRC_HIP_TRY(ctx, hipGetLastError());
        const size_t lds_big = team_lds_bytes(kpad, 1 << kBigLog2);
        hipLaunchKernelGGL((k_doc_lds<MODE, kBigTeam, kBigLog2, kBigPer>), dim3(grid_for(n, 1, 256)), dim3(kBlock),
                           lds_big, s, docs->offsets, n, kMedMax, kMediumMax, docs->tokens, V, a, err, list(2),
                           count(2));
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    if (V <= kDirectMaxV) {
        // small vocabulary: counts directly in LDS, one workgroup per long document
        const size_t lds = (((size_t)V * 4 + 15) & ~(size_t)15) + (size_t)kpad * 8 +
                           (kDirectThreads / 64) * sizeof(u128) + 16;
        hipLaunchKernelGGL((k_doc_direct<MODE>), dim3(256), dim3(kDirectThreads), lds, s, docs->offsets, V,
                           docs->tokens, a, err, list(3), count(3));
        MRC_HIP_TRY(ctx, hipGetLastError());
    } else {
        const size_t table_bytes = (size_t)kLongBlocks * (size_t)V * sizeof(uint32_t);
        auto it = ctx->scratch.find("long_tables");
        const bool fresh = it == ctx->scratch.end() || it->second.second < table_bytes;
        void* tables = nullptr;
        MRC_TRY(scratch(ctx, "long_tables", table_bytes, &tables));
        if (fresh) MRC_HIP_TRY(ctx, hipMemsetAsync(tables, 0, ctx->scratch["long_tables"].second, s));
        const size_t lds = (size_t)kpad * 8 + (kLongThreads / 64) * sizeof(u128) + 16;
        hipLaunchKernelGGL((k_doc_global<MODE>), dim3(kLongBlocks), dim3(kLongThreads), lds, s, docs->offsets, V,
                           docs->tokens, a, (uint32_t*)tables, err, list(3), count(3));
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    return MRC_OK;
}

}  // namespace

namespace mrc {

mrc_status clear_words(mrc_ctx* ctx, int64_t* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_words, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, s, p, n);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_validate_offsets(mrc_ctx* ctx, const mrc_docs* docs, hipStream_t s, int32_t* lists) {
    // error word and, for the listed passes, the class counts (one launch:
    // the words between them are free at this point of every caller)
    MRC_TRY(clear_words(ctx, ctx->d_flags, lists ? kClassCount + kClasses : 1, s));
    const int64_t n = docs->n_docs;
    if (n == 0) return MRC_OK;
    hipLaunchKernelGGL(k_validate_offsets, dim3((unsigned)ceil_div(n + 1, 256)), dim3(256), 0, s, docs->offsets, n,
                       docs->n_tokens, (unsigned long long*)ctx->d_flags, lists);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status count_scratch(mrc_ctx* ctx, const mrc_docs* docs, CountLists* c) {
    const size_t T = (size_t)std::max<int64_t>(docs->n_tokens, 1);
    void *pt = nullptr, *pf = nullptr, *pn = nullptr;
    MRC_TRY(scratch(ctx, "count_term", T * sizeof(int32_t), &pt));
    MRC_TRY(scratch(ctx, "count_tf", T * sizeof(int32_t), &pf));
    MRC_TRY(scratch(ctx, "count_nnz", (size_t)std::max<int64_t>(docs->n_docs, 1) * sizeof(int32_t), &pn));
    c->term = (int32_t*)pt;
    c->tf = (int32_t*)pf;
    c->nnz = (int32_t*)pn;
    return MRC_OK;
}

mrc_status launch_counts(mrc_ctx* ctx, const mrc_docs* docs, int32_t V, const CountLists& c, hipStream_t s) {
    PassArgs a{};
    a.cnt_term = c.term;
    a.cnt_tf = c.tf;
    a.cnt_nnz = c.nnz;
    return run_docpass<MODE_COUNT>(ctx, docs, V, a, s, "counts");
}

mrc_status launch_df(mrc_ctx* ctx, const mrc_docs* docs, int32_t V, uint32_t* d_df, const CountLists& c,
                     hipStream_t s) {
    const int64_t n = docs->n_docs;
    PassArgs a{};
    a.cnt_term = c.term;
    a.cnt_tf = c.tf;
    a.cnt_nnz = c.nnz;
    MRC_TRY(run_docpass<MODE_COUNT>(ctx, docs, V, a, s, "df_count"));
    if (n == 0) {
        MRC_HIP_TRY(ctx, hipMemsetAsync(d_df, 0, (size_t)V * 4, s));
        return MRC_OK;
    }
    const unsigned long long* err = (const unsigned long long*)ctx->d_flags;
    ScopedTimer tm(ctx, "df_hist", s);
    const int slices = (int)ceil_div(V, kHistSlice);
    if (slices > kHistMaxSlices) {
        MRC_HIP_TRY(ctx, hipMemsetAsync(d_df, 0, (size_t)V * 4, s));
        hipLaunchKernelGGL(k_df_atomic, dim3(grid_for(n, 4, 256 * 8)), dim3(256), 0, s, docs->offsets, n, c.term,
                           c.nnz, d_df, err);
        MRC_HIP_TRY(ctx, hipGetLastError());
        return MRC_OK;
    }
    // document ranges of at most 65535 documents; about 256 workgroups in all
    const int64_t groups = std::max<int64_t>(ceil_div(n, 65535), std::min<int64_t>(ceil_div(256, slices), n));
    const int64_t words = (int64_t)slices * kHistSlice / 2;
    void* partial = nullptr;
    MRC_TRY(scratch(ctx, "df_partial", (size_t)groups * (size_t)words * sizeof(uint32_t), &partial));
    hipLaunchKernelGGL(k_df_hist, dim3((unsigned)(slices * groups)), dim3(kHistThreads), 0, s, docs->offsets, n,
                       c.term, c.nnz, (int)groups, (uint32_t*)partial, words, err);
    MRC_HIP_TRY(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_df_sum, dim3((unsigned)ceil_div(words, 64)), dim3(256), 0, s, (const uint32_t*)partial,
                       (int)groups, words, V, d_df);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_sign_counts(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const CountLists& c,
                              float* sig_out, float* norm_out, hipStream_t s) {
    const int64_t n = docs->n_docs;
    if (n == 0) return MRC_OK;
    PassArgs a{};
    a.tinfo = m->d_tinfo;
    a.rinv = m->d_rinv;
    a.k = m->k;
    a.vocab = m->vocab;
    a.ref_idf = m->spec.ref_weight == MRC_REF_IDF ? 1 : 0;
    a.sig = sig_out;
    a.norm = norm_out;
    a.term_at = m->d_term_at;
    const size_t kpad = (size_t)((m->k + 1) & ~1);
    ScopedTimer tm(ctx, "sign_counts", s);
    // persistent: every wavefront signs a contiguous block of documents with
    // the next two documents' loads in flight. With the hot-term cache (16
    // wavefronts' bins, rinv and the cache fit the LDS): one workgroup per CU.
    // Each workgroup fills its cache first, which pays from some 65k documents
    // on (200k docs, k = 256: 0.42 -> 0.37 ms; 1M, k = 128: 1.82 -> 1.55 ms;
    // 20k, k = 64: 36 -> 44 us, so small corpora keep the plain form)
    const size_t lds_hot = (16 + 1) * kpad * 8 + (size_t)kHotSlots * (4 + sizeof(TermInfo));
    if (n >= kSignHotMinDocs && lds_hot <= 160 * 1024) {
        int cus = 256;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
            cus = 256;
        (void)hipGetLastError();
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(cus, ceil_div(n, 16)));
        const int64_t per_wave = ceil_div(n, grid * 16);
        hipLaunchKernelGGL(k_sign_counts<true>, dim3((unsigned)grid), dim3(1024), lds_hot, s, docs->offsets, n, c.term,
                           c.tf, c.nnz, a, per_wave, (const unsigned long long*)ctx->d_flags);
    } else {
        const size_t lds = (size_t)5 * kpad * 8;  // 4 wavefronts' bins + rinv
        const int64_t grid = persistent_grid(ctx, (const void*)k_sign_counts<false>, 256, ceil_div(n, 4));
        const int64_t per_wave = ceil_div(n, grid * 4);
        hipLaunchKernelGGL(k_sign_counts<false>, dim3((unsigned)grid), dim3(256), lds, s, docs->offsets, n, c.term,
                           c.tf, c.nnz, a, per_wave, (const unsigned long long*)ctx->d_flags);
    }
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_csr(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const CsrOut& c, hipStream_t s) {
    PassArgs a{};
    a.tinfo = m->d_tinfo;
    a.rank_of = m->d_rank_of;
    a.H = c.H;
    a.ldh = c.ldh;
    a.wh = c.wh;
    a.ent_rank = c.ent_rank;
    a.ent_w = c.ent_w;
    a.nnz_tail = c.nnz_tail;
    a.pcount = c.pcount;
    return run_docpass<MODE_CSR>(ctx, docs, m->vocab, a, s, "csr");
}

mrc_status launch_sign(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, float* sig_out,
                       float* norm_out, hipStream_t s) {
    PassArgs a{};
    a.tinfo = m->d_tinfo;
    a.rinv = m->d_rinv;
    a.k = m->k;
    a.ref_idf = m->spec.ref_weight == MRC_REF_IDF ? 1 : 0;
    a.sig = sig_out;
    a.norm = norm_out;
    return run_docpass<MODE_SIGN>(ctx, docs, m->vocab, a, s, "sign");
}

}  // namespace mrc
