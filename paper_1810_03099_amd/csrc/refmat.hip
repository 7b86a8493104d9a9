// Signatures against general reference vectors: the k columns of a dense
// V x k matrix R (Section 4's construction with Section 6's weighted
// vector-space models; a column may weight its terms, and columns may share
// terms). For each document d and reference j,
//   sig_dj = (sum over the document's terms t of w_dt R[t][j]) / (|w_d| |r_j|),
// w_dt = tf_dt * idf_t (the model's float idf), |w_d| as in every signing
// pass (exact fixed-point sum, exact_sums.h), |r_j| the column norm of R.
//
// The document's distinct terms come from the count pass (term, tf lists at
// its token offset). One wavefront per document, lane c of k-tile q owning
// output column 64 q + c: each term of the document contributes one
// contiguous row segment R[t][64 q .. 64 q + 63] (a 256-byte load across the
// wavefront). The H most frequent terms of the model (H = 8192 / k rows, at
// most 256) have their rows of R staged in LDS once per workgroup: their
// entries read LDS instead of memory. Sums run in float64, in the count
// list's order, rounded once to float.
#include <algorithm>

#include "common.h"
#include "exact_sums.h"

using namespace mrc;
using namespace mrc_exact;

namespace {

constexpr int kHotFloats = 8192;  // LDS floats of staged rows per workgroup (32 KB)
constexpr int kBatch = 8;         // memory rows in flight per lane

// Column sums of squares of R over row slabs: partial[slab][c] (float64), in
// a fixed order (each lane walks its column over the slab's rows).
__global__ __launch_bounds__(256) void k_col_sq(const float* __restrict__ R, int64_t V, int k, int64_t slab,
                                                double* __restrict__ partial) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= k) return;
    const int64_t r0 = (int64_t)blockIdx.y * slab, r1 = std::min<int64_t>(V, r0 + slab);
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double v = R[r * k + c];
        acc = fma(v, v, acc);
    }
    partial[(int64_t)blockIdx.y * k + c] = acc;
}

// rinv[c] = 1 / |r_c| (0 for a zero column), summing the slabs in order.
__global__ void k_col_rinv(const double* __restrict__ partial, int slabs, int k, double* __restrict__ rinv) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double s = 0.0;
    for (int b = 0; b < slabs; ++b) s += partial[(int64_t)b * k + c];
    rinv[c] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
}

struct RefArgs {
    const int64_t* off;
    int64_t n;
    const int32_t* term;   // count lists (term, tf) at each document's token offset
    const int32_t* tf;
    const int32_t* nnz;
    const float* idf;      // [V]
    const int32_t* rank_of;
    const int32_t* term_at;
    const float* R;        // [V][k]
    int64_t V;
    int k;
    int hot;               // staged rows (the model's `hot` most frequent terms)
    const double* rinv;    // [k]
    float* sig;
    float* norm;
};

// NT k-tiles of 64 columns (k <= 64 NT).
template <int NT>
__global__ __launch_bounds__(256) void k_sign_matrix(RefArgs a, const unsigned long long* __restrict__ err) {
    extern __shared__ __align__(16) float hot_rows[];  // [hot][k]
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kErrOffsets | kErrDocLen)) return;
    const int k = a.k;
    for (int64_t i = threadIdx.x; i < (int64_t)a.hot * k; i += 256) {
        const int h = (int)(i / k), c = (int)(i % k);
        hot_rows[i] = a.R[(int64_t)a.term_at[h] * k + c];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int64_t d = (int64_t)blockIdx.x * 4 + wave; d < a.n; d += (int64_t)gridDim.x * 4) {
        const int64_t o = a.off[d];
        const int m = a.nnz[d];
        double acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = 0.0;
        u128 nsq = 0;
        for (int e0 = 0; e0 < m; e0 += 64) {
            // this lane's entry of the chunk: term, weight, staged row (-1: none)
            const bool valid = e0 + lane < m;
            int t = 0, h = -1;
            double w = 0.0;
            if (valid) {
                t = a.term[o + e0 + lane];
                const uint32_t f = (uint32_t)a.tf[o + e0 + lane];
                const float idf = a.idf[t];
                const int r = a.rank_of[t];
                h = r < a.hot ? r : -1;
                w = (double)f * (double)idf;
                nsq += term_sq_fixed(f, idf);
            }
            uint64_t hot_m = __ballot(valid && h >= 0);
            uint64_t cold_m = __ballot(valid && h < 0);
            // staged rows: LDS reads
            while (hot_m) {
                const int e = __ffsll((long long)hot_m) - 1;
                hot_m &= hot_m - 1;
                const int he = __builtin_amdgcn_readlane(h, e);
                const double we = __shfl(w, e, 64);
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int c = 64 * q + lane;
                    if (c < k) acc[q] = fma(we, (double)hot_rows[he * k + c], acc[q]);
                }
            }
            // the others: row segments of R, kBatch entries in flight
            while (cold_m) {
                int te[kBatch];
                double we[kBatch];
                int nb = 0;
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    te[u] = 0;
                    we[u] = 0.0;
                    if (cold_m) {
                        const int e = __ffsll((long long)cold_m) - 1;
                        cold_m &= cold_m - 1;
                        te[u] = __builtin_amdgcn_readlane(t, e);
                        we[u] = __shfl(w, e, 64);
                        nb = u + 1;
                    }
                }
                float v[kBatch][NT];
#pragma unroll
                for (int u = 0; u < kBatch; ++u)
#pragma unroll
                    for (int q = 0; q < NT; ++q) {
                        const int c = 64 * q + lane;
                        v[u][q] = (u < nb && c < k) ? a.R[(int64_t)te[u] * k + c] : 0.f;
                    }
#pragma unroll
                for (int u = 0; u < kBatch; ++u)
                    if (u < nb) {
#pragma unroll
                        for (int q = 0; q < NT; ++q) acc[q] = fma(we[u], (double)v[u][q], acc[q]);
                    }
            }
        }
        const double nrm = norm_from_fixed(wave_sum_u128(nsq));
        float* out = a.sig + d * k;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int c = 64 * q + lane;
            if (c < k) out[c] = (float)(nrm > 0.0 ? acc[q] * a.rinv[c] / nrm : 0.0);
        }
        if (lane == 0 && a.norm) a.norm[d] = (float)nrm;
    }
}

template <int NT>
mrc_status launch_nt(mrc_ctx* ctx, const RefArgs& a, size_t lds, hipStream_t s) {
    const int64_t grid = persistent_grid(ctx, (const void*)k_sign_matrix<NT>, 256, ceil_div(a.n, 4));
    hipLaunchKernelGGL(k_sign_matrix<NT>, dim3((unsigned)grid), dim3(256), lds, s, a,
                       (const unsigned long long*)ctx->d_flags);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace

namespace mrc {

mrc_status launch_sign_matrix(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const float* R, int32_t k,
                              float* sig_out, float* norm_out, hipStream_t s) {
    const int64_t n = docs->n_docs;
    const int64_t V = m->vocab;
    // column norms of R
    const int64_t slab = 4096;
    const int slabs = (int)ceil_div(V, slab);
    void *partial = nullptr, *rinv = nullptr;
    MRC_TRY(scratch(ctx, "refmat_partial", (size_t)slabs * k * sizeof(double), &partial));
    MRC_TRY(scratch(ctx, "refmat_rinv", (size_t)k * sizeof(double), &rinv));
    {
        ScopedTimer tm(ctx, "refmat_norms", s);
        hipLaunchKernelGGL(k_col_sq, dim3((unsigned)ceil_div(k, 256), (unsigned)slabs), dim3(256), 0, s, R, V, k,
                           slab, (double*)partial);
        hipLaunchKernelGGL(k_col_rinv, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, (const double*)partial,
                           slabs, k, (double*)rinv);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    // the documents' distinct terms and counts
    CountLists c;
    MRC_TRY(count_scratch(ctx, docs, &c));
    MRC_TRY(launch_counts(ctx, docs, (int32_t)V, c, s));
    if (n == 0) return MRC_OK;
    RefArgs a{};
    a.off = docs->offsets;
    a.n = n;
    a.term = c.term;
    a.tf = c.tf;
    a.nnz = c.nnz;
    a.idf = m->d_idf;
    a.rank_of = m->d_rank_of;
    a.term_at = m->d_term_at;
    a.R = R;
    a.V = V;
    a.k = k;
    a.hot = (int)std::min<int64_t>({256, kHotFloats / k, m->n_listed});
    a.rinv = (const double*)rinv;
    a.sig = sig_out;
    a.norm = norm_out;
    const size_t lds = (size_t)a.hot * k * sizeof(float);
    ScopedTimer tm(ctx, "sign_matrix", s);
    const int nt = (int)ceil_div(k, 64);
    switch (nt) {
        case 1: return launch_nt<1>(ctx, a, lds, s);
        case 2: return launch_nt<2>(ctx, a, lds, s);
        case 3: case 4: return launch_nt<4>(ctx, a, lds, s);
        case 5: case 6: case 7: case 8: return launch_nt<8>(ctx, a, lds, s);
        default: return launch_nt<16>(ctx, a, lds, s);
    }
}

}  // namespace mrc
