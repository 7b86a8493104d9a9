// Per-document passes over the token CSR: length classification, document
// frequency (model build) and MRC signing (Section 4: cosine of the TF-IDF
// vector of a document against each of the k reference parts).
//
// Every pass turns a document's token stream into term counts with a hash
// table: in LDS for documents up to kMediumMax tokens (one wavefront per
// short document, one 256-thread workgroup per medium document), and in a
// per-workgroup [V] count array in global memory for longer documents.
//
// Signing needs, per document d and part j,
//   num_j = sum over occurrences p with part(t_p) = j of c_p,  c_p = idf_t * rho_t,
//   |w_d|^2 = sum over occurrences p of tf(t_p) * idf(t_p)^2,
// and sig_dj = num_j / (|w_d| |r_j|). num_j is accumulated in exact 64-bit
// fixed point (c_p * 2^32 is an integer for the weights that occur), so it is
// exact and independent of order; the norm sums in a fixed per-document order
// (float32, float64 for documents longer than 10^4 tokens). A document's result
// therefore depends only on its own tokens, never on the batch around it.
#include "common.h"

using namespace mrc;

namespace {

constexpr int kBlock = 256;
constexpr int kEmpty = -1;
constexpr int kDfReplicas = 32;

enum : unsigned long long {
    kErrOffsets = 1ull,
    kErrToken = 2ull,
};

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

// Fixed-order sum over a team (one wavefront, or the 4 wavefronts of a block).
template <int TEAM, typename T>
__device__ __forceinline__ T team_sum(T v, T* red) {
    v = mrc_dev::wave_sum(v);
    if constexpr (TEAM == 64) {
        return v;
    } else {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        T r = red[0];
#pragma unroll
        for (int i = 1; i < TEAM / 64; ++i) r += red[i];
        __syncthreads();
        return r;
    }
}

struct SignArgs {
    const TermInfo* tinfo;
    const double* rinv;
    int k;
    int ref_idf;       // 1: rho_t = idf_t, so c_p = idf^2
    float* sig;
    float* norm;
    // MODE_CSR: unit TF-IDF weights w = tf * idf / |w_d| of each distinct term.
    // Ranks below H go to the dense head matrix (matrix-core layout, ld ldh);
    // the others are listed at the document's token offset (ent_*), counted
    // per rank in pcount, and their number stored in nnz_tail.
    const int32_t* rank_of;
    int H;
    int ldh;
    float* wh;
    int32_t* ent_rank;
    float* ent_w;
    int32_t* nnz_tail;
    uint32_t* pcount;
};

enum { MODE_DF = 0, MODE_SIGN = 1, MODE_CSR = 2 };

// Emit one distinct term of document d (MODE_CSR).
__device__ __forceinline__ void csr_emit(const SignArgs& sa, int64_t d, int64_t o, int t, unsigned tf, double nrm,
                                         int* tcount) {
    const float w = (float)((double)tf * (double)sa.tinfo[t].idf / nrm);
    const int r = sa.rank_of[t];
    if (r < sa.H) {
        sa.wh[d * sa.ldh + mrc_dev::mfma_col(r)] = w;
    } else {
        const int e = atomicAdd(tcount, 1);
        sa.ent_rank[o + e] = r;
        sa.ent_w[o + e] = w;
        atomicAdd(&sa.pcount[r - sa.H], 1u);
    }
}

// Offsets check before any token is read: offsets[0] = 0, non-decreasing,
// offsets[n] <= n_tokens. Sets kErrOffsets; the document kernels then return
// at once.
__global__ void k_validate_offsets(const int64_t* __restrict__ off, int64_t n, int64_t n_tokens,
                                   unsigned long long* __restrict__ err) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d > n) return;
    bool bad = false;
    if (d == 0) bad = off[0] != 0;
    else bad = off[d] < off[d - 1];
    if (d == n) bad = bad || off[n] > n_tokens || off[n] < 0;
    if (bad) atomicOr(err, kErrOffsets);
}

// LDS layout of one team: bins u64[kpad] | keys i32[SLOTS] | cnt i32[SLOTS] |
// used u16[SLOTS/2] | nused i32 | red (double[4])
__host__ __device__ constexpr size_t team_lds_bytes(int kpad, int slots) {
    return (size_t)kpad * 8 + (size_t)slots * 8 + (size_t)slots + 16 + 32;
}

// Documents d with lo_len < L_d <= hi_len are this kernel's; every kernel scans
// all offsets and skips the others (no lists, no atomics). df increments go to
// one of kDfReplicas copies of the [V] counters (chosen by document), so that
// frequent terms do not serialise on one address; the copies are summed later.
template <int MODE, int TEAM, int LOG2_SLOTS, int MAXPER>
__global__ __launch_bounds__(kBlock) void k_doc_lds(const int64_t* __restrict__ off, int64_t n_docs,
                                                    int lo_len, int hi_len,
                                                    const int32_t* __restrict__ tok,
                                                    int32_t V, uint32_t* __restrict__ df,
                                                    SignArgs sa, unsigned long long* __restrict__ err) {
    constexpr int SLOTS = 1 << LOG2_SLOTS;
    constexpr int TEAMS = kBlock / TEAM;
    extern __shared__ __align__(16) unsigned char smem[];
    const int kpad = MODE == MODE_SIGN ? ((sa.k + 1) & ~1) : 0;
    const size_t tbytes = team_lds_bytes(kpad, SLOTS);
    const int team = threadIdx.x / TEAM;
    const int tid = threadIdx.x % TEAM;
    unsigned char* base = smem + (size_t)team * tbytes;
    unsigned long long* bins = (unsigned long long*)base;
    int* keys = (int*)(base + (size_t)kpad * 8);
    int* cnt = keys + SLOTS;
    unsigned short* used = (unsigned short*)(cnt + SLOTS);
    int* nused = (int*)(used + SLOTS / 2);
    double* red = (double*)(base + tbytes - 32);

    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrOffsets) return;
    for (int s = tid; s < SLOTS; s += TEAM) {
        keys[s] = kEmpty;
        cnt[s] = 0;
    }
    for (int j = tid; j < kpad; j += TEAM) bins[j] = 0ull;
    if (tid == 0) *nused = 0;
    team_sync<TEAM>();

    for (int64_t d = (int64_t)blockIdx.x * TEAMS + team; d < n_docs; d += (int64_t)gridDim.x * TEAMS) {
        const int64_t o = off[d];
        const int64_t L64 = off[d + 1] - o;
        if (L64 <= lo_len || L64 > hi_len) {
            if (!(lo_len == 0 && L64 == 0)) continue;
        }
        const int L = (int)L64;
        uint32_t* dfr = df ? df + (size_t)(d % kDfReplicas) * (size_t)V : nullptr;
        int slot_r[MAXPER];
        float idf_r[MAXPER];
#pragma unroll
        for (int r = 0; r < MAXPER; ++r) {
            slot_r[r] = -1;
            idf_r[r] = 0.f;
            const int p = tid + r * TEAM;
            if (p < L) {
                const int t = tok[o + p];
                if ((unsigned)t >= (unsigned)V) {
                    atomicOr(err, kErrToken);
                    continue;
                }
                int h = hash_slot(t, LOG2_SLOTS);
                bool won = false;
                while (true) {
                    int prev = atomicCAS(&keys[h], kEmpty, t);
                    if (prev == kEmpty) {
                        won = true;
                        break;
                    }
                    if (prev == t) break;
                    h = (h + 1) & (SLOTS - 1);
                }
                int old = atomicAdd(&cnt[h], 1);
                if (won) used[atomicAdd(nused, 1)] = (unsigned short)h;
                if constexpr (MODE == MODE_DF) {
                    if (old == 0) atomicAdd(&dfr[t], 1u);
                } else {
                    (void)old;
                    TermInfo ti = sa.tinfo[t];
                    slot_r[r] = h;
                    idf_r[r] = ti.idf;
                    if (MODE == MODE_SIGN && ti.part >= 0) {
                        float c = sa.ref_idf ? ti.idf * ti.idf : ti.idf;
                        atomicAdd(&bins[ti.part], mrc_dev::fixed32(c));
                    }
                }
            }
        }
        team_sync<TEAM>();
        double nrm = 0.0;
        if constexpr (MODE != MODE_DF) {
            float nacc = 0.f;
#pragma unroll
            for (int r = 0; r < MAXPER; ++r) {
                if (slot_r[r] >= 0) nacc += (float)cnt[slot_r[r]] * (idf_r[r] * idf_r[r]);
            }
            float n2 = team_sum<TEAM, float>(nacc, (float*)red);
            nrm = (double)sqrtf(n2);
        }
        if constexpr (MODE == MODE_SIGN) {
            float* out = sa.sig + (int64_t)d * sa.k;
            for (int j = tid; j < sa.k; j += TEAM) {
                double v = nrm > 0.0 ? mrc_dev::unfixed32(bins[j]) * sa.rinv[j] / nrm : 0.0;
                out[j] = (float)v;
            }
            if (tid == 0 && sa.norm) sa.norm[d] = (float)nrm;
        }
        team_sync<TEAM>();
        const int nu = *nused;
        if constexpr (MODE == MODE_CSR) {
            int* tcount = (int*)red;
            if (tid == 0) *tcount = 0;
            team_sync<TEAM>();
            for (int u = tid; u < nu; u += TEAM) {
                const int sl = used[u];
                csr_emit(sa, d, o, keys[sl], (unsigned)cnt[sl], nrm, tcount);
            }
            team_sync<TEAM>();
            if (tid == 0) sa.nnz_tail[d] = *tcount;
            team_sync<TEAM>();
        }
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

// Long documents: a [V] uint32 count table per workgroup in global memory
// (all zero between documents).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_doc_global(const int64_t* __restrict__ off, int64_t n_docs,
                                                       int lo_len,
                                                       const int32_t* __restrict__ tok,
                                                       int32_t V, uint32_t* __restrict__ df,
                                                       SignArgs sa, uint32_t* __restrict__ tables,
                                                       unsigned long long* __restrict__ err) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* bins = (unsigned long long*)smem;
    const int kpad = MODE == MODE_SIGN ? ((sa.k + 1) & ~1) : 0;
    double* red = (double*)(smem + (size_t)kpad * 8);
    uint32_t* cnt = tables + (size_t)blockIdx.x * (size_t)V;
    const int tid = threadIdx.x;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrOffsets) return;
    for (int j = tid; j < kpad; j += kBlock) bins[j] = 0ull;
    __syncthreads();
    for (int64_t d = blockIdx.x; d < n_docs; d += gridDim.x) {
        const int64_t o = off[d];
        const int64_t L = off[d + 1] - o;
        if (L <= lo_len) continue;
        uint32_t* dfr = df ? df + (size_t)(d % kDfReplicas) * (size_t)V : nullptr;
        for (int64_t p = tid; p < L; p += kBlock) {
            const int t = tok[o + p];
            if ((unsigned)t >= (unsigned)V) {
                atomicOr(err, kErrToken);
                continue;
            }
            unsigned old = atomicAdd(&cnt[t], 1u);
            if constexpr (MODE == MODE_DF) {
                if (old == 0) atomicAdd(&dfr[t], 1u);
            } else if constexpr (MODE == MODE_SIGN) {
                (void)old;
                TermInfo ti = sa.tinfo[t];
                if (ti.part >= 0) {
                    float c = sa.ref_idf ? ti.idf * ti.idf : ti.idf;
                    atomicAdd(&bins[ti.part], mrc_dev::fixed32(c));
                }
            }
        }
        __threadfence();
        __syncthreads();
        if constexpr (MODE != MODE_DF) {
            double nrm;
            if (L > kFp64NormMin) {
                double acc = 0.0;
                for (int64_t p = tid; p < L; p += kBlock) {
                    const int t = tok[o + p];
                    if ((unsigned)t >= (unsigned)V) continue;
                    unsigned tf = __hip_atomic_load(&cnt[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    double idf = (double)sa.tinfo[t].idf;
                    acc += (double)tf * idf * idf;
                }
                nrm = sqrt(team_sum<kBlock, double>(acc, red));
            } else {
                float acc = 0.f;
                for (int64_t p = tid; p < L; p += kBlock) {
                    const int t = tok[o + p];
                    if ((unsigned)t >= (unsigned)V) continue;
                    unsigned tf = __hip_atomic_load(&cnt[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    float idf = sa.tinfo[t].idf;
                    acc += (float)tf * (idf * idf);
                }
                nrm = (double)sqrtf(team_sum<kBlock, float>(acc, (float*)red));
            }
            if constexpr (MODE == MODE_SIGN) {
                float* out = sa.sig + (int64_t)d * sa.k;
                for (int j = tid; j < sa.k; j += kBlock) {
                    double v = nrm > 0.0 ? mrc_dev::unfixed32(bins[j]) * sa.rinv[j] / nrm : 0.0;
                    out[j] = (float)v;
                }
                if (tid == 0 && sa.norm) sa.norm[d] = (float)nrm;
            } else {
                // each distinct term once: the first occurrence to swap its count out emits it
                int* tcount = (int*)(red + 2);
                if (tid == 0) *tcount = 0;
                __syncthreads();
                for (int64_t p = tid; p < L; p += kBlock) {
                    const int t = tok[o + p];
                    if ((unsigned)t >= (unsigned)V) continue;
                    const unsigned tf = atomicExch(&cnt[t], 0u);
                    if (tf > 0) csr_emit(sa, d, o, t, tf, nrm, tcount);
                }
                __syncthreads();
                if (tid == 0) sa.nnz_tail[d] = *tcount;
            }
        }
        __syncthreads();
        for (int64_t p = tid; p < L; p += kBlock) {
            const int t = tok[o + p];
            if ((unsigned)t >= (unsigned)V) continue;
            __hip_atomic_store(&cnt[t], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int j = tid; j < kpad; j += kBlock) bins[j] = 0ull;
        __threadfence();
        __syncthreads();
    }
}

constexpr int kShortTeam = 64, kShortLog2 = 10, kShortPer = kShortMax / 64;      // 1024 slots
constexpr int kMedTeam = 256, kMedLog2 = 13, kMedPer = kMediumMax / 256;         // 8192 slots
static_assert((1 << kShortLog2) >= 2 * kShortMax, "short table load factor");
static_assert((1 << kMedLog2) >= 2 * kMediumMax, "medium table load factor");

int grid_for(int64_t n_items_upper, int teams_per_block, int cap) {
    int64_t g = ceil_div(n_items_upper, teams_per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

__global__ void k_df_reduce(const uint32_t* __restrict__ rep, int32_t V, uint32_t* __restrict__ df) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V) return;
    uint32_t s = 0;
#pragma unroll 8
    for (int r = 0; r < kDfReplicas; ++r) s += rep[(size_t)r * V + t];
    df[t] = s;
}

template <int MODE>
mrc_status run_docpass(mrc_ctx* ctx, const mrc_docs* docs, int32_t V, uint32_t* df, const SignArgs& sa,
                       hipStream_t s, const char* name) {
    const int64_t n = docs->n_docs;
    unsigned long long* err = (unsigned long long*)ctx->d_flags;
    MRC_TRY(launch_validate_offsets(ctx, docs, s));
    if (n == 0) return MRC_OK;
    const int kpad = MODE == MODE_SIGN ? ((sa.k + 1) & ~1) : 0;
    const size_t rep_bytes = (size_t)kDfReplicas * (size_t)V * sizeof(uint32_t);
    void* rep = nullptr;
    if (MODE == MODE_DF) {
        MRC_TRY(scratch(ctx, "df_replicas", rep_bytes, &rep));
        MRC_HIP_TRY(ctx, hipMemsetAsync(rep, 0, rep_bytes, s));
    }
    uint32_t* dfk = (uint32_t*)rep;
    ScopedTimer tm(ctx, name, s);
    {
        size_t lds = team_lds_bytes(kpad, 1 << kShortLog2) * (kBlock / kShortTeam);
        int grid = grid_for(n, kBlock / kShortTeam, 256 * 8);
        hipLaunchKernelGGL((k_doc_lds<MODE, kShortTeam, kShortLog2, kShortPer>), dim3(grid), dim3(kBlock),
                           lds, s, docs->offsets, n, 0, kShortMax, docs->tokens, V, dfk, sa, err);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    {
        size_t lds = team_lds_bytes(kpad, 1 << kMedLog2);
        int grid = grid_for(n, 1, 256 * 2);
        hipLaunchKernelGGL((k_doc_lds<MODE, kMedTeam, kMedLog2, kMedPer>), dim3(grid), dim3(kBlock), lds, s,
                           docs->offsets, n, kShortMax, kMediumMax, docs->tokens, V, dfk, sa, err);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    {
        const size_t table_bytes = (size_t)kLongBlocks * (size_t)V * sizeof(uint32_t);
        auto it = ctx->scratch.find("long_tables");
        bool fresh = it == ctx->scratch.end() || it->second.second < table_bytes;
        void* tables = nullptr;
        MRC_TRY(scratch(ctx, "long_tables", table_bytes, &tables));
        if (fresh) MRC_HIP_TRY(ctx, hipMemsetAsync(tables, 0, ctx->scratch["long_tables"].second, s));
        size_t lds = (size_t)kpad * 8 + 32;
        hipLaunchKernelGGL((k_doc_global<MODE>), dim3(kLongBlocks), dim3(kBlock), lds, s, docs->offsets, n,
                           kMediumMax, docs->tokens, V, dfk, sa, (uint32_t*)tables, err);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    if (MODE == MODE_DF) {
        hipLaunchKernelGGL(k_df_reduce, dim3((unsigned)ceil_div(V, 256)), dim3(256), 0, s, (const uint32_t*)rep,
                           V, df);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    return MRC_OK;
}

}  // namespace

namespace mrc {

mrc_status launch_validate_offsets(mrc_ctx* ctx, const mrc_docs* docs, hipStream_t s) {
    MRC_HIP_TRY(ctx, hipMemsetAsync(ctx->d_flags, 0, sizeof(int64_t), s));
    const int64_t n = docs->n_docs;
    if (n == 0) return MRC_OK;
    hipLaunchKernelGGL(k_validate_offsets, dim3((unsigned)ceil_div(n + 1, 256)), dim3(256), 0, s, docs->offsets, n,
                       docs->n_tokens, (unsigned long long*)ctx->d_flags);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_df(mrc_ctx* ctx, const mrc_docs* docs, int32_t vocab, uint32_t* d_df, hipStream_t s) {
    SignArgs sa{};
    return run_docpass<MODE_DF>(ctx, docs, vocab, d_df, sa, s, "df");
}

mrc_status launch_csr(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const CsrOut& c, hipStream_t s) {
    SignArgs sa{};
    sa.tinfo = m->d_tinfo;
    sa.rank_of = m->d_rank_of;
    sa.H = c.H;
    sa.ldh = c.ldh;
    sa.wh = c.wh;
    sa.ent_rank = c.ent_rank;
    sa.ent_w = c.ent_w;
    sa.nnz_tail = c.nnz_tail;
    sa.pcount = c.pcount;
    return run_docpass<MODE_CSR>(ctx, docs, m->vocab, nullptr, sa, s, "csr");
}

mrc_status launch_sign(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, float* sig_out,
                       float* norm_out, hipStream_t s) {
    SignArgs sa{};
    sa.tinfo = m->d_tinfo;
    sa.rinv = m->d_rinv;
    sa.k = m->k;
    sa.ref_idf = m->spec.ref_weight == MRC_REF_IDF ? 1 : 0;
    sa.sig = sig_out;
    sa.norm = norm_out;
    return run_docpass<MODE_SIGN>(ctx, docs, m->vocab, nullptr, sa, s, "sign");
}

}  // namespace mrc
