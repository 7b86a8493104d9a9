// Model tables from document frequencies (Section 4): the frequency-sorted
// term list (df descending, ties by ascending id, zero-frequency terms after
// all listed terms), the selected positions, the k contiguous parts, idf and
// the reference-part norms.
//
// The sort is a stable least-significant-digit radix sort of the keys
// N - df[t] with the ids as values, 8 bits per pass; starting from ids in
// ascending order, stability gives the ascending-id tie order. Each scatter
// block finds its output positions from the per-digit totals and the counts
// of earlier tiles (no separate scan). The first pass also counts the
// zero-frequency terms, from which the tables kernel derives V' and the
// selected positions.
#include "common.h"

using namespace mrc;

namespace {

constexpr int kTile = 2048;      // elements per radix block
constexpr int kThreads = 256;
constexpr int kPerThread = kTile / kThreads;

template <bool FIRST>
__device__ __forceinline__ uint32_t radix_key(const uint32_t* df, const uint32_t* keys_in, int e,
                                              uint32_t N) {
    return FIRST ? N - df[e] : keys_in[e];
}

// Digit counts of one tile, stored digit-major (hist[digit * nblk + block]),
// and added into the per-digit totals. The first pass also adds the tile's
// zero-df count to *zeros.
template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ df,
                                                         const uint32_t* __restrict__ keys_in, int V,
                                                         uint32_t N, int shift,
                                                         uint32_t* __restrict__ hist, int nblk,
                                                         uint32_t* __restrict__ totals,
                                                         unsigned long long* __restrict__ zeros) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t nz;
    h[threadIdx.x] = 0;
    if (threadIdx.x == 0) nz = 0;
    __syncthreads();
    const int b0 = blockIdx.x * kTile;
    uint32_t z = 0;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const int e = b0 + i * kThreads + threadIdx.x;
        if (e < V) {
            const uint32_t key = radix_key<FIRST>(df, keys_in, e, N);
            atomicAdd(&h[(key >> shift) & 255u], 1u);
            if (FIRST) z += df[e] == 0u;
        }
    }
    if (FIRST) {
        z = mrc_dev::wave_sum(z);
        if ((threadIdx.x & 63) == 0 && z) atomicAdd(&nz, z);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
    if (h[threadIdx.x]) atomicAdd(&totals[threadIdx.x], h[threadIdx.x]);
    if (FIRST && threadIdx.x == 0 && nz) atomicAdd(zeros, (unsigned long long)nz);
}

// Selected positions [lo, hi) of the frequency-sorted list of V' terms;
// false when the selection is invalid or holds fewer than k terms.
__device__ bool select_positions(int64_t Vp, const mrc_ref_spec& spec, int64_t* lo_out, int64_t* hi_out) {
    int64_t lo = 0, hi = Vp;
    switch (spec.mode) {
        case MRC_SEL_ALL: break;
        case MRC_SEL_REGION:
            lo = spec.lo;
            hi = spec.hi < 0 ? Vp : (spec.hi < Vp ? spec.hi : Vp);
            break;
        case MRC_SEL_RAREST: lo = Vp - spec.m; break;
        case MRC_SEL_DROP_TOP: lo = (Vp * spec.drop_top_ppm + 999999) / 1000000; break;
        default: lo = -1; break;
    }
    const bool ok = !(lo < 0 || hi > Vp || hi - lo < (int64_t)spec.k || spec.k < 1);
    *lo_out = ok ? lo : 0;
    *hi_out = ok ? hi : 0;
    return ok;
}

template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ df,
                                                            const uint32_t* __restrict__ keys_in,
                                                            const int32_t* __restrict__ vals_in,
                                                            uint32_t* __restrict__ keys_out,
                                                            int32_t* __restrict__ vals_out, int V,
                                                            uint32_t N, int shift,
                                                            const uint32_t* __restrict__ hist, int nblk,
                                                            const uint32_t* __restrict__ totals) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    __shared__ uint32_t wsum[kThreads / 64];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    // first output position of (digit tid, this tile): the counts of all
    // smaller digits plus those of digit tid in earlier tiles
    uint32_t pre = 0;
    const uint32_t* row = hist + (size_t)tid * nblk;
    int b = 0;
    for (; b + 16 <= (int)blockIdx.x; b += 16) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = row[b + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) pre += v[u];
    }
    for (; b < (int)blockIdx.x; ++b) pre += row[b];
    const uint32_t tot = totals[tid];
    uint32_t incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    for (int i = 0; i < kThreads / 64; ++i) wcnt[i][tid] = 0;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    base[tid] = before + incl - tot + pre;
    __syncthreads();
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int b0 = blockIdx.x * kTile;
    for (int c = 0; c < kPerThread; ++c) {
        const int e = b0 + c * kThreads + tid;
        const bool valid = e < V;
        uint32_t key = valid ? radix_key<FIRST>(df, keys_in, e, N) : 0u;
        int32_t val = valid ? (FIRST ? e : vals_in[e]) : 0;
        const uint32_t digit = (key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const unsigned long long bal = __ballot(set);
            peers &= set ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[w][digit] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[digit] + (uint32_t)rank;
            for (int i = 0; i < w; ++i) pos += wcnt[i][digit];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int i = 0; i < kThreads / 64; ++i) {
            add += wcnt[i][tid];
            wcnt[i][tid] = 0;
        }
        base[tid] += add;
        __syncthreads();
    }
}

__device__ __forceinline__ int part_of_position(int64_t p, int64_t lo, int64_t hi, int k) {
    if (p < lo || p >= hi) return -1;
    const int64_t m = hi - lo, q = m / k, r = m % k, pos = p - lo, big = r * (q + 1);
    return pos < big ? (int)(pos / (q + 1)) : (int)(r + (pos - big) / q);
}

__device__ __forceinline__ float term_idf(uint32_t df, int64_t N, int idf_mode) {
    double idf = 1.0;
    if (idf_mode == MRC_IDF_SMOOTH) idf = log((1.0 + (double)N) / (1.0 + (double)df)) + 1.0;
    return (float)idf;
}

// Blocks [0, k): |r_j| = sqrt(sum of rho_t^2 over part j's terms), fixed-order
// reduction. Blocks k..: rank, idf and (idf, part) of 256 list positions each.
// Every block derives V' = V - info[5] and the selection; block 0 records
// them (info: [0] error bits, [5] zero-df terms, [6] V', [7] lo, [8] hi).
__global__ __launch_bounds__(kThreads) void k_tables(const uint32_t* __restrict__ df,
                                                     const int32_t* __restrict__ term_at, int V, int64_t N,
                                                     int64_t* __restrict__ info, mrc_ref_spec spec,
                                                     int32_t* __restrict__ rank_of,
                                                     float* __restrict__ idf_out, TermInfo* __restrict__ tinfo,
                                                     double* __restrict__ rnorm, double* __restrict__ rinv) {
    const int k = spec.k, idf_mode = spec.idf_mode, ref_idf = spec.ref_weight == MRC_REF_IDF ? 1 : 0;
    const int64_t Vp = (int64_t)V - info[5];
    int64_t sel_lo, sel_hi;
    const bool sel_ok = select_positions(Vp, spec, &sel_lo, &sel_hi);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!sel_ok) info[0] |= kErrSelection;
        info[6] = Vp;
        info[7] = sel_lo;
        info[8] = sel_hi;
    }
    if ((int)blockIdx.x >= k) {
        const int p = ((int)blockIdx.x - k) * kThreads + threadIdx.x;
        if (p >= V) return;
        const int t = term_at[p];
        rank_of[t] = p;
        const float f = term_idf(df[t], N, idf_mode);
        idf_out[t] = f;
        TermInfo ti;
        ti.idf = f;
        ti.part = sel_ok ? part_of_position(p, sel_lo, sel_hi, k) : -1;
        tinfo[t] = ti;
        return;
    }
    __shared__ double red[kThreads / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    if (sel_ok) {
        const int64_t lo = sel_lo, hi = sel_hi, m = hi - lo, q = m / k, r = m % k;
        const int64_t start = lo + (j < r ? j * (q + 1) : r * (q + 1) + (j - r) * q);
        const int64_t size = q + (j < r ? 1 : 0);
        for (int64_t i = threadIdx.x; i < size; i += kThreads) {
            const double rho = ref_idf ? (double)term_idf(df[term_at[start + i]], N, idf_mode) : 1.0;
            s += rho * rho;
        }
    }
    s = mrc_dev::wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) t += red[i];
        const double nrm = sqrt(t);
        rnorm[j] = nrm;
        rinv[j] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

}  // namespace

namespace mrc {

mrc_status launch_model_tables(mrc_ctx* ctx, mrc_model* m, hipStream_t s) {
    const int V = m->vocab;
    const uint32_t N = (uint32_t)m->n_docs;
    const int nblk = (int)ceil_div(V, kTile);
    void *hist = nullptr, *ka = nullptr, *kb = nullptr, *vb = nullptr;
    MRC_TRY(scratch(ctx, "radix_hist", (size_t)256 * nblk * sizeof(uint32_t), &hist));
    MRC_TRY(scratch(ctx, "radix_keys_a", (size_t)V * sizeof(uint32_t), &ka));
    MRC_TRY(scratch(ctx, "radix_keys_b", (size_t)V * sizeof(uint32_t), &kb));
    MRC_TRY(scratch(ctx, "radix_vals_b", (size_t)V * sizeof(int32_t), &vb));
    int bits = 1;
    while (bits < 32 && (N >> bits) != 0) ++bits;
    const int passes = (bits + 7) / 8;
    int64_t* info = ctx->d_flags;
    void* totals = nullptr;
    MRC_TRY(scratch(ctx, "radix_totals", (size_t)4 * 256 * sizeof(uint32_t), &totals));
    MRC_TRY(clear_words(ctx, (int64_t*)totals, 4 * 256 / 2, s));
    MRC_TRY(clear_words(ctx, info + 5, 4, s));
    // Ping-pong so that the final pass writes m->d_term_at.
    uint32_t* keys[2] = {(uint32_t*)ka, (uint32_t*)kb};
    int32_t* vals[2] = {m->d_term_at, (int32_t*)vb};
    int out = (passes % 2 == 1) ? 0 : 1;  // buffer index written by pass 0
    {
        ScopedTimer tm(ctx, "rank_sort", s);
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = 8 * pass;
            const int in = 1 - out;
            uint32_t* tot = (uint32_t*)totals + 256 * pass;
            if (pass == 0) {
                hipLaunchKernelGGL(k_radix_hist<true>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   (const uint32_t*)nullptr, V, N, shift, (uint32_t*)hist, nblk, tot,
                                   (unsigned long long*)(info + 5));
                hipLaunchKernelGGL(k_radix_scatter<true>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   (const uint32_t*)nullptr, (const int32_t*)nullptr, keys[out], vals[out],
                                   V, N, shift, (const uint32_t*)hist, nblk, (const uint32_t*)tot);
            } else {
                hipLaunchKernelGGL(k_radix_hist<false>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   keys[in], V, N, shift, (uint32_t*)hist, nblk, tot, (unsigned long long*)nullptr);
                hipLaunchKernelGGL(k_radix_scatter<false>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   keys[in], vals[in], keys[out], vals[out], V, N, shift,
                                   (const uint32_t*)hist, nblk, (const uint32_t*)tot);
            }
            MRC_HIP_TRY(ctx, hipGetLastError());
            out = 1 - out;
        }
    }
    hipLaunchKernelGGL(k_tables, dim3((unsigned)(m->k + ceil_div(V, kThreads))), dim3(kThreads), 0, s, m->d_df,
                       m->d_term_at, V, (int64_t)N, info, m->spec, m->d_rank_of, m->d_idf, m->d_tinfo, m->d_rnorm,
                       m->d_rinv);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
