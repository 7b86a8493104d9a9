// Model tables from document frequencies (Section 4): the frequency-sorted
// term list (df descending, ties by ascending id, zero-frequency terms after
// all listed terms), the selected positions, the k contiguous parts, idf and
// the reference-part norms.
//
// The sort is a stable least-significant-digit radix sort of the keys
// N - df[t] with the ids as values, 8 bits per pass; starting from ids in
// ascending order, stability gives the ascending-id tie order.
#include "common.h"

using namespace mrc;

namespace {

constexpr int kTile = 4096;      // elements per radix block
constexpr int kThreads = 256;
constexpr int kPerThread = kTile / kThreads;

template <bool FIRST>
__device__ __forceinline__ uint32_t radix_key(const uint32_t* df, const uint32_t* keys_in, int e,
                                              uint32_t N) {
    return FIRST ? N - df[e] : keys_in[e];
}

template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ df,
                                                         const uint32_t* __restrict__ keys_in, int V,
                                                         uint32_t N, int shift,
                                                         uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int b0 = blockIdx.x * kTile;
    for (int i = 0; i < kPerThread; ++i) {
        int e = b0 + i * kThreads + threadIdx.x;
        if (e < V) atomicAdd(&h[(radix_key<FIRST>(df, keys_in, e, N) >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of n counts in place, one workgroup.
__global__ __launch_bounds__(kThreads) void k_scan(uint32_t* __restrict__ a, int n) {
    __shared__ uint32_t part[kThreads];
    const int per = (n + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * per;
    const int hi = min(n, lo + per);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < kThreads; ++i) {
            uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t* __restrict__ df,
                                                            const uint32_t* __restrict__ keys_in,
                                                            const int32_t* __restrict__ vals_in,
                                                            uint32_t* __restrict__ keys_out,
                                                            int32_t* __restrict__ vals_out, int V,
                                                            uint32_t N, int shift,
                                                            const uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    base[tid] = hist[tid * nblk + blockIdx.x];
    for (int i = 0; i < kThreads / 64; ++i) wcnt[i][tid] = 0;
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

// V' = number of terms with df > 0; then the selected positions [lo, hi).
__global__ void k_count_listed(const uint32_t* __restrict__ df, int V, unsigned long long* out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    bool listed = t < V && df[t] > 0;
    unsigned long long b = __ballot(listed);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
}

// info: [0] error bits, [6] n_listed (input), [7] lo, [8] hi
__global__ void k_select(int64_t* info, mrc_ref_spec spec) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t Vp = info[6];
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
    if (lo < 0 || hi > Vp || hi - lo < (int64_t)spec.k || spec.k < 1) {
        info[0] |= 4;
        lo = 0;
        hi = 0;
    }
    info[7] = lo;
    info[8] = hi;
}

__device__ __forceinline__ int part_of_position(int64_t p, int64_t lo, int64_t hi, int k) {
    if (p < lo || p >= hi) return -1;
    const int64_t m = hi - lo, q = m / k, r = m % k, pos = p - lo, big = r * (q + 1);
    return pos < big ? (int)(pos / (q + 1)) : (int)(r + (pos - big) / q);
}

__global__ void k_tables(const uint32_t* __restrict__ df, const int32_t* __restrict__ term_at, int V,
                         int64_t N, const int64_t* __restrict__ info, int k, int idf_mode,
                         int32_t* __restrict__ rank_of, float* __restrict__ idf_out,
                         TermInfo* __restrict__ tinfo) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= V) return;
    const int t = term_at[p];
    rank_of[t] = p;
    double idf = 1.0;
    if (idf_mode == MRC_IDF_SMOOTH) idf = log((1.0 + (double)N) / (1.0 + (double)df[t])) + 1.0;
    const float f = (float)idf;
    idf_out[t] = f;
    TermInfo ti;
    ti.idf = f;
    ti.part = (info[0] & 4) ? -1 : part_of_position(p, info[7], info[8], k);
    tinfo[t] = ti;
}

// |r_j| = sqrt(sum of rho_t^2 over the part's terms), one workgroup per part,
// fixed-order reduction.
__global__ __launch_bounds__(kThreads) void k_rnorm(const int32_t* __restrict__ term_at,
                                                    const float* __restrict__ idf,
                                                    const int64_t* __restrict__ info, int k,
                                                    int ref_idf, double* __restrict__ rnorm,
                                                    double* __restrict__ rinv) {
    __shared__ double red[kThreads / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    if (!(info[0] & 4)) {
        const int64_t lo = info[7], hi = info[8], m = hi - lo, q = m / k, r = m % k;
        const int64_t start = lo + (j < r ? j * (q + 1) : r * (q + 1) + (j - r) * q);
        const int64_t size = q + (j < r ? 1 : 0);
        for (int64_t i = threadIdx.x; i < size; i += kThreads) {
            double rho = ref_idf ? (double)idf[term_at[start + i]] : 1.0;
            s += rho * rho;
        }
    }
    s = mrc_dev::wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) t += red[i];
        double nrm = sqrt(t);
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
    // Ping-pong so that the final pass writes m->d_term_at.
    uint32_t* keys[2] = {(uint32_t*)ka, (uint32_t*)kb};
    int32_t* vals[2] = {m->d_term_at, (int32_t*)vb};
    int out = (passes % 2 == 1) ? 0 : 1;  // buffer index written by pass 0
    {
        ScopedTimer tm(ctx, "rank_sort", s);
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = 8 * pass;
            const int in = 1 - out;
            if (pass == 0) {
                hipLaunchKernelGGL(k_radix_hist<true>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   (const uint32_t*)nullptr, V, N, shift, (uint32_t*)hist, nblk);
            } else {
                hipLaunchKernelGGL(k_radix_hist<false>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   keys[in], V, N, shift, (uint32_t*)hist, nblk);
            }
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(kThreads), 0, s, (uint32_t*)hist, 256 * nblk);
            if (pass == 0) {
                hipLaunchKernelGGL(k_radix_scatter<true>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   (const uint32_t*)nullptr, (const int32_t*)nullptr, keys[out], vals[out],
                                   V, N, shift, (const uint32_t*)hist, nblk);
            } else {
                hipLaunchKernelGGL(k_radix_scatter<false>, dim3(nblk), dim3(kThreads), 0, s, m->d_df,
                                   keys[in], vals[in], keys[out], vals[out], V, N, shift,
                                   (const uint32_t*)hist, nblk);
            }
            MRC_HIP_TRY(ctx, hipGetLastError());
            out = 1 - out;
        }
    }
    int64_t* info = ctx->d_flags;
    MRC_HIP_TRY(ctx, hipMemsetAsync(info + 6, 0, 3 * sizeof(int64_t), s));
    hipLaunchKernelGGL(k_count_listed, dim3((unsigned)ceil_div(V, 256)), dim3(256), 0, s, m->d_df, V,
                       (unsigned long long*)(info + 6));
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, info, m->spec);
    hipLaunchKernelGGL(k_tables, dim3((unsigned)ceil_div(V, 256)), dim3(256), 0, s, m->d_df, m->d_term_at,
                       V, (int64_t)N, (const int64_t*)info, m->k, m->spec.idf_mode, m->d_rank_of, m->d_idf,
                       m->d_tinfo);
    hipLaunchKernelGGL(k_rnorm, dim3(m->k), dim3(kThreads), 0, s, m->d_term_at, m->d_idf,
                       (const int64_t*)info, m->k, m->spec.ref_weight == MRC_REF_IDF ? 1 : 0, m->d_rnorm,
                       m->d_rinv);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
