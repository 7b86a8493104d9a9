// Exact cosine comparator (Eq. 1 on the TF-IDF vectors): the ground truth of
// Section 5, every document compared with every other.
//
// The score of a pair is defined as the float32 multiply-add chain over the
// unit TF-IDF weights in ascending term rank: acc = 0; for each rank r,
// acc = fmaf(w_ir, w_jr, acc) (absent terms leave acc unchanged).
//  * Ranks below H (the most frequent terms, where almost all of the pair
//    mass lies) are dense: a Gram panel of the head matrix is computed on the
//    FP32 matrix cores, whose 16x16x4 steps perform exactly that chain.
//  * The remaining ranks are sparse: for row i the chain continues over i's
//    tail terms in ascending rank, each adding w_ir * w_jr into the row's
//    accumulators for every j in that term's posting list (one term at a
//    time, so each accumulator sees its terms in order).
#include <algorithm>
#include <type_traits>

#include "common.h"

using namespace mrc;

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kWT = 64;
constexpr int kSortCap = 16384;   // tail terms per document sorted in LDS (8 B each)

// Posting lists of the tail ranks: (document, weight) for every tail entry.
__global__ void k_postings(const int64_t* __restrict__ off, int64_t n, const int32_t* __restrict__ ent_rank,
                           const float* __restrict__ ent_w, const int32_t* __restrict__ nnz_tail, int H,
                           const uint32_t* __restrict__ poff, uint32_t* __restrict__ pcur,
                           int32_t* __restrict__ post_doc, float* __restrict__ post_w) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t d = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); d < n; d += waves) {
        const int64_t o = off[d];
        const int m = nnz_tail[d];
        for (int e = lane; e < m; e += 64) {
            const int r = ent_rank[o + e] - H;
            const uint32_t pos = poff[r] + atomicAdd(&pcur[r], 1u);
            post_doc[pos] = (int32_t)d;
            post_w[pos] = ent_w[o + e];
        }
    }
}

// Sort each document's tail entries by rank (distinct within a document):
// bitonic network in LDS over the next power of two, padded with INT_MAX.
__global__ __launch_bounds__(256) void k_sort_tail(const int64_t* __restrict__ off, int64_t n,
                                                   int32_t* __restrict__ ent_rank, float* __restrict__ ent_w,
                                                   const int32_t* __restrict__ nnz_tail,
                                                   unsigned long long* __restrict__ err) {
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t* key = (int32_t*)smem;
    float* val = (float*)(smem + kSortCap * 4);
    for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
        const int m = nnz_tail[d];
        if (m <= 1) continue;
        if (m > kSortCap) {
            if (threadIdx.x == 0) atomicOr(err, kErrTailCap);
            continue;
        }
        const int64_t o = off[d];
        int P = 2;
        while (P < m) P <<= 1;
        for (int i = threadIdx.x; i < P; i += 256) {
            key[i] = i < m ? ent_rank[o + i] : 0x7fffffff;
            val[i] = i < m ? ent_w[o + i] : 0.f;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P; i += 256) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const bool asc = (i & k) == 0;
                        if ((key[i] > key[ixj]) == asc) {
                            const int tk = key[i];
                            key[i] = key[ixj];
                            key[ixj] = tk;
                            const float tv = val[i];
                            val[i] = val[ixj];
                            val[ixj] = tv;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < m; i += 256) {
            ent_rank[o + i] = key[i];
            ent_w[o + i] = val[i];
        }
        __syncthreads();
    }
}

// Head Gram panel: rows [r0, r1) (multiples of 64) against all columns j > i,
// written to G[(i - r0) * ldg + j]. One wavefront per 64x64 tile; blockIdx.y
// is the tile row, blockIdx.x * 4 + wave the tile column.
template <int NC>
__global__ __launch_bounds__(256) void k_gram_head(const float* __restrict__ wh, int ldh, int n, int r0,
                                                   float* __restrict__ G, int64_t ldg) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bi = r0 / kWT + blockIdx.y;
    const int bj = blockIdx.x * 4 + wave;
    const int nb = (n + kWT - 1) / kWT;
    if (bj < bi || bj >= nb) return;
    const int li = lane & 15, lg = lane >> 4;
    const float* pa = wh + (int64_t)(bi * kWT + li) * ldh + 4 * lg;
    const float* pb = wh + (int64_t)(bj * kWT + li) * ldh + 4 * lg;
    f32x4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        a[0][x] = *(const f32x4*)(pa + (int64_t)16 * x * ldh);
        b[0][x] = *(const f32x4*)(pb + (int64_t)16 * x * ldh);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int cur = c & 1, nxt = cur ^ 1;
        if (c + 1 < NC) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[nxt][x] = *(const f32x4*)(pa + (int64_t)16 * x * ldh + 16 * (c + 1));
                b[nxt][x] = *(const f32x4*)(pb + (int64_t)16 * x * ldh + 16 * (c + 1));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cur][x][m], b[cur][y][m], acc[x][y], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * kWT + 16 * x + 4 * lg + r, j = bj * kWT + 16 * y + li;
                if (i < j && j < n) G[(int64_t)(i - r0) * ldg + j] = acc[x][y][r];
            }
}

// Row pass: the chain of row i continues over its (rank-sorted) tail terms,
// then every j > i with score >= tau is emitted. Terms are applied one at a
// time (a workgroup barrier after each keeps every accumulator's terms in
// rank order); their posting ranges and weights are staged in LDS 512 terms
// at a time, and each thread's posting entries are loaded kRing - 1 terms
// ahead (up to kPostQ per thread; a longer list loads the rest in place), so
// a term costs a barrier rather than three dependent global loads.
// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>) in order
// (compile-time ring slots).
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

constexpr int kRowChunk = 16384;
constexpr int kRowStage = 512;
constexpr int kMetaTerms = 512;
constexpr int kPostQ = 2;   // posting entries per thread and term in the ring
constexpr int kRing = 6;    // terms in flight: entries of term e + kRing - 1 load while term e is applied

__global__ __launch_bounds__(256) void k_exact_rows(const float* __restrict__ G, int64_t ldg, int r0, int n,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ ent_rank,
                                                    const float* __restrict__ ent_w,
                                                    const int32_t* __restrict__ nnz_tail, int H,
                                                    const uint32_t* __restrict__ poff,
                                                    const int32_t* __restrict__ post_doc,
                                                    const float* __restrict__ post_w, float tau, PairSink sink) {
    __shared__ float acc[kRowChunk];
    __shared__ mrc_pair stage[kRowStage];
    __shared__ uint32_t sm_p0[kMetaTerms], sm_len[kMetaTerms];
    __shared__ float sm_w[kMetaTerms];
    __shared__ int scount;
    __shared__ unsigned long long sbase;
    const int i = r0 + blockIdx.x;
    if (i >= n) return;
    const int tid = threadIdx.x;
    const int64_t o = off[i];
    const int m = nnz_tail[i];
    const float* grow = G + (int64_t)blockIdx.x * ldg;
    int dq[kRing][kPostQ];
    float wq[kRing][kPostQ];
    for (int c0 = i + 1; c0 < n; c0 += kRowChunk) {
        const int c1 = min(n, c0 + kRowChunk);
        for (int j = c0 + tid; j < c1; j += 256) acc[j - c0] = grow[j];
        if (tid == 0) scount = 0;
        __syncthreads();
        for (int eb = 0; eb < m; eb += kMetaTerms) {
            const int nb = min(kMetaTerms, m - eb);
            for (int e = tid; e < nb; e += 256) {
                const int r = ent_rank[o + eb + e] - H;
                const uint32_t p0 = poff[r];
                sm_p0[e] = p0;
                sm_len[e] = poff[r + 1] - p0;
                sm_w[e] = ent_w[o + eb + e];
            }
            __syncthreads();
            // term e's first kPostQ * 256 entries into ring slot S
            auto load = [&](int e, auto slot) __attribute__((always_inline)) {
                constexpr int S = decltype(slot)::value;
                const bool has = e < nb;
                const uint32_t p0 = has ? sm_p0[e] : 0u, len = has ? sm_len[e] : 0u;
#pragma unroll
                for (int q = 0; q < kPostQ; ++q) {
                    const uint32_t x = (uint32_t)(tid + 256 * q);
                    dq[S][q] = x < len ? post_doc[p0 + x] : -1;
                    wq[S][q] = x < len ? post_w[p0 + x] : 0.f;
                }
            };
            auto apply = [&](int e, auto slot) __attribute__((always_inline)) {
                constexpr int S = decltype(slot)::value;
                const float wi = sm_w[e];
#pragma unroll
                for (int q = 0; q < kPostQ; ++q) {
                    const int j = dq[S][q];
                    if (j >= c0 && j < c1) acc[j - c0] = __builtin_fmaf(wi, wq[S][q], acc[j - c0]);
                }
                const uint32_t len = sm_len[e];
                if (len > 256u * kPostQ) {  // the rest of a long list, in place
                    const uint32_t p0 = sm_p0[e];
                    for (uint32_t x = 256u * kPostQ + tid; x < len; x += 256) {
                        const int j = post_doc[p0 + x];
                        if (j >= c0 && j < c1) acc[j - c0] = __builtin_fmaf(wi, post_w[p0 + x], acc[j - c0]);
                    }
                }
                __syncthreads();
            };
            static_for<kRing - 1>([&](auto sl) { load(sl.value, sl); });
            for (int e = 0; e < nb; e += kRing) {
                bool done = false;
                static_for<kRing>([&](auto sl) {
                    constexpr int S = decltype(sl)::value;
                    if (done || e + S >= nb) {
                        done = true;
                        return;
                    }
                    load(e + S + kRing - 1, std::integral_constant<int, (S + kRing - 1) % kRing>{});
                    apply(e + S, sl);
                });
                if (done) break;
            }
        }
        for (int j = c0 + tid; j < c1; j += 256) {
            const float v = acc[j - c0];
            if (v >= tau) {
                const int slot = atomicAdd(&scount, 1);
                if (slot < kRowStage) {
                    stage[slot] = mrc_pair{i, j, v, 0};
                } else {
                    const unsigned long long g = atomicAdd(sink.counter, 1ull);
                    if ((int64_t)g < sink.capacity) sink.pairs[g] = mrc_pair{i, j, v, 0};
                }
            }
        }
        __syncthreads();
        const int cnt = min(scount, kRowStage);
        if (tid == 0 && cnt > 0) sbase = atomicAdd(sink.counter, (unsigned long long)cnt);
        __syncthreads();
        for (int e = tid; e < cnt; e += 256) {
            const int64_t dst = (int64_t)sbase + e;
            if (dst < sink.capacity) sink.pairs[dst] = stage[e];
        }
        __syncthreads();
    }
}

// Exclusive scan of n counts (one workgroup) into out[0..n], out[n] = total.
__global__ __launch_bounds__(1024) void k_scan_excl(const uint32_t* __restrict__ in, int n, uint32_t* __restrict__ out) {
    __shared__ uint32_t part[1024];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(n, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += in[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
        out[n] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        out[i] = run;
        run += in[i];
    }
}

}  // namespace

namespace mrc {

mrc_status launch_exact_cosine(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, float tau, PairSink sink,
                               hipStream_t s) {
    const int64_t n = docs->n_docs;
    const int V = m->vocab;
    const int H = V >= 512 ? 512 : (int)ceil_div(V, 32) * 32;
    const int NC = H / 16;
    const int64_t n_pad = ceil_div(n > 0 ? n : 1, 64) * 64;
    const int64_t nt = docs->n_tokens > 0 ? docs->n_tokens : 1;
    const int ntail = std::max(1, V - H);
    void *wh, *er, *ew, *nz, *pc, *po, *pu, *pd, *pw;
    MRC_TRY(scratch(ctx, "ex_wh", (size_t)n_pad * H * 4, &wh));
    MRC_TRY(scratch(ctx, "ex_ent_rank", (size_t)nt * 4, &er));
    MRC_TRY(scratch(ctx, "ex_ent_w", (size_t)nt * 4, &ew));
    MRC_TRY(scratch(ctx, "ex_nnz", (size_t)n_pad * 4, &nz));
    MRC_TRY(scratch(ctx, "ex_pcount", (size_t)(ntail + 1) * 4, &pc));
    MRC_TRY(scratch(ctx, "ex_poff", (size_t)(ntail + 1) * 4, &po));
    MRC_TRY(scratch(ctx, "ex_pcur", (size_t)(ntail + 1) * 4, &pu));
    MRC_TRY(scratch(ctx, "ex_post_doc", (size_t)nt * 4, &pd));
    MRC_TRY(scratch(ctx, "ex_post_w", (size_t)nt * 4, &pw));
    MRC_HIP_TRY(ctx, hipMemsetAsync(wh, 0, (size_t)n_pad * H * 4, s));
    MRC_HIP_TRY(ctx, hipMemsetAsync(nz, 0, (size_t)n_pad * 4, s));
    MRC_HIP_TRY(ctx, hipMemsetAsync(pc, 0, (size_t)(ntail + 1) * 4, s));
    MRC_HIP_TRY(ctx, hipMemsetAsync(pu, 0, (size_t)(ntail + 1) * 4, s));
    CsrOut co{H, H, (float*)wh, (int32_t*)er, (float*)ew, (int32_t*)nz, (uint32_t*)pc};
    MRC_TRY(launch_csr(ctx, m, docs, co, s));
    if (n < 2) return MRC_OK;
    ScopedTimer tm(ctx, "exact_cosine", s);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, (const uint32_t*)pc, ntail, (uint32_t*)po);
    hipLaunchKernelGGL(k_postings, dim3((unsigned)std::min<int64_t>(ceil_div(n, 4), 4096)), dim3(256), 0, s,
                       docs->offsets, n, (const int32_t*)er, (const float*)ew, (const int32_t*)nz, H,
                       (const uint32_t*)po, (uint32_t*)pu, (int32_t*)pd, (float*)pw);
    hipLaunchKernelGGL(k_sort_tail, dim3((unsigned)std::min<int64_t>(n, 4096)), dim3(256), (size_t)kSortCap * 8, s,
                       docs->offsets, n, (int32_t*)er, (float*)ew, (const int32_t*)nz,
                       (unsigned long long*)ctx->d_flags);
    MRC_HIP_TRY(ctx, hipGetLastError());
    // Gram panels of at most ~1.5 GB
    int64_t P = (int64_t)(1.5e9 / (4.0 * (double)n_pad)) / 64 * 64;
    P = std::max<int64_t>(64, std::min<int64_t>(P, n_pad));
    void* G = nullptr;
    MRC_TRY(scratch(ctx, "ex_gram", (size_t)P * n_pad * 4, &G));
    const int nb = (int)(n_pad / 64);
    for (int64_t r0 = 0; r0 < n; r0 += P) {
        const int64_t r1 = std::min<int64_t>(n_pad, r0 + P);
        dim3 grid((unsigned)ceil_div(nb, 4), (unsigned)((r1 - r0) / 64));
        switch (NC) {
#define MRC_GH(c) case c: hipLaunchKernelGGL(k_gram_head<c>, grid, dim3(256), 0, s, (const float*)wh, H, (int)n, (int)r0, (float*)G, n_pad); break;
            MRC_GH(2) MRC_GH(4) MRC_GH(6) MRC_GH(8) MRC_GH(10) MRC_GH(12) MRC_GH(14) MRC_GH(16) MRC_GH(18) MRC_GH(20)
            MRC_GH(22) MRC_GH(24) MRC_GH(26) MRC_GH(28) MRC_GH(30) MRC_GH(32)
#undef MRC_GH
            default: return fail(MRC_E_INVAL, "exact cosine: unsupported head width");
        }
        const int64_t rows = std::min<int64_t>(n, r1) - r0;
        hipLaunchKernelGGL(k_exact_rows, dim3((unsigned)rows), dim3(256), 0, s, (const float*)G, n_pad, (int)r0, (int)n,
                           docs->offsets, (const int32_t*)er, (const float*)ew, (const int32_t*)nz, H,
                           (const uint32_t*)po, (const int32_t*)pd, (const float*)pw, tau, sink);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    return MRC_OK;
}

}  // namespace mrc
