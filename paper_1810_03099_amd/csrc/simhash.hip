// Simhash comparator (Section 3): hash every token to 64 bits, add +1 to bit
// column b when bit b of the hash is 1 and -1 when it is 0, keep bit b of the
// result when the column sum is greater than 0; documents are compared by the
// Hamming distance of their 64-bit words.
//
// Token hash: the first 8 bytes (little-endian) of MD5 over the term id as 4
// little-endian bytes. MD5 follows the RFC 1321 algorithm: one 512-bit block
// (message, 0x80, zero fill, bit length), four rounds of 16 steps.
#include <cmath>

#include "common.h"

using namespace mrc;

namespace {

struct Md5Consts {
    uint32_t k[64];  // floor(|sin(i + 1)| * 2^32)
};

__device__ __forceinline__ uint32_t rotl(uint32_t x, int s) { return (x << s) | (x >> (32 - s)); }

__device__ uint64_t md5_first8(uint32_t t, const Md5Consts& c) {
    uint32_t m[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) m[i] = 0;
    m[0] = t;            // 4 message bytes, little-endian
    m[1] = 0x80u;        // padding bit right after the message
    m[14] = 32u;         // message length in bits (low word)
    const int sh[4][4] = {{7, 12, 17, 22}, {5, 9, 14, 20}, {4, 11, 16, 23}, {6, 10, 15, 21}};
    uint32_t a = 0x67452301u, b = 0xefcdab89u, cc = 0x98badcfeu, d = 0x10325476u;
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        uint32_t f;
        int g;
        const int round = i >> 4;
        if (round == 0) {
            f = (b & cc) | (~b & d);
            g = i;
        } else if (round == 1) {
            f = (d & b) | (~d & cc);
            g = (5 * i + 1) & 15;
        } else if (round == 2) {
            f = b ^ cc ^ d;
            g = (3 * i + 5) & 15;
        } else {
            f = cc ^ (b | ~d);
            g = (7 * i) & 15;
        }
        const uint32_t tmp = d;
        d = cc;
        cc = b;
        b = b + rotl(a + f + c.k[i] + m[g], sh[round][i & 3]);
        a = tmp;
    }
    const uint32_t h0 = 0x67452301u + a, h1 = 0xefcdab89u + b;
    return (uint64_t)h0 | ((uint64_t)h1 << 32);
}

__global__ void k_term_hashes(int32_t V, Md5Consts c, uint64_t* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < V) out[t] = md5_first8((uint32_t)t, c);
}

// One wavefront per document, 64 tokens per round, one token per lane. The sum
// over valid tokens of +1 / -1 for bit b of their hashes is 2 c_b - v, with c_b
// the number of valid tokens whose bit b is set and v the number of valid
// tokens. A round's 64 hashes (0 for invalid tokens) are a 64x64 bit matrix;
// six exchange stages between lanes l and l ^ j (j = 32 .. 1) transpose it
// (each stage swaps the off-diagonal j x j blocks of every 2j x 2j block), so
// that lane b holds bit b of every token and c_b grows by its popcount; bit b
// of the word is the sign of 2 c_b - v > 0.
__global__ __launch_bounds__(256) void k_simhash(const int64_t* __restrict__ off, int64_t n,
                                                 const int32_t* __restrict__ tok, int32_t V,
                                                 const uint64_t* __restrict__ hash, uint64_t* __restrict__ out,
                                                 unsigned long long* __restrict__ err) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1ull) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t d = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); d < n; d += waves) {
        const int64_t o = off[d], L = off[d + 1] - o;
        int cnt = 0, nvalid = 0;
        for (int64_t p0 = 0; p0 < L; p0 += 64) {
            const int64_t p = p0 + lane;
            uint64_t h = 0;
            bool valid = false;
            if (p < L) {
                const int t = tok[o + p];
                if ((unsigned)t < (unsigned)V) {
                    h = hash[t];
                    valid = true;
                } else {
                    atomicOr(err, kErrToken);
                }
            }
            nvalid += __popcll(__ballot(valid));
            uint64_t w = h;
#pragma unroll
            for (int j = 32; j >= 1; j >>= 1) {
                // the low j bits of every 2j-bit group
                const uint64_t m = j == 32 ? 0x00000000FFFFFFFFull
                                 : j == 16 ? 0x0000FFFF0000FFFFull
                                 : j == 8  ? 0x00FF00FF00FF00FFull
                                 : j == 4  ? 0x0F0F0F0F0F0F0F0Full
                                 : j == 2  ? 0x3333333333333333ull
                                           : 0x5555555555555555ull;
                const uint64_t p = __shfl_xor(w, j, 64);
                const bool first = (lane & j) == 0;  // the pair's lower lane
                const uint64_t t = (((first ? w : p) >> j) ^ (first ? p : w)) & m;
                w ^= first ? (t << j) : t;
            }
            cnt += __popcll(w);
        }
        const unsigned long long bits = __ballot(2 * cnt - nvalid > 0);
        if (lane == 0) out[d] = bits;
    }
}

// All pairs i < j with popcount(x_i ^ x_j) <= max_dist. A workgroup takes a
// 256x256 tile of the upper triangle, one row per thread; the column words
// are read by scalar loads (the same for the whole wavefront); hits are staged
// in LDS and reserved with one atomic per tile.
constexpr int kHT = 256;
constexpr int kHStage = 4096;

__global__ __launch_bounds__(256) void k_hamming(const uint64_t* __restrict__ sim, int n, int max_dist, int nb,
                                                 PairSink sink) {
    __shared__ mrc_pair stage[kHStage];
    __shared__ int scount;
    __shared__ unsigned long long sbase;
    // upper-triangle tile t -> (bi, bj), row-major
    const int64_t t = blockIdx.x;
    double a = 2.0 * nb + 1.0;
    int bi = (int)((a - sqrt(a * a - 8.0 * (double)t)) * 0.5);
    bi = max(0, min(nb - 1, bi));
    auto start = [nb](int64_t r) { return r * nb - r * (r - 1) / 2; };
    while (bi > 0 && start(bi) > t) --bi;
    while (bi + 1 < nb && start(bi + 1) <= t) ++bi;
    const int bj = bi + (int)(t - start(bi));
    const int i = bi * kHT + threadIdx.x;
    const int j0 = bj * kHT;
    if (threadIdx.x == 0) scount = 0;
    __syncthreads();
    // a hit (row i, column j0 + c): staged in LDS, or straight to the output
    // when the tile has more hits than the stage holds
    auto put = [&](int c, int dist) {
        const int j = j0 + c;
        const int slot = atomicAdd(&scount, 1);
        if (slot < kHStage) {
            stage[slot] = mrc_pair{i, j, (float)dist, 0};
        } else {
            const unsigned long long g = atomicAdd(sink.counter, 1ull);
            if ((int64_t)g < sink.capacity) sink.pairs[g] = mrc_pair{i, j, (float)dist, 0};
        }
    };
    if (i < n) {
        // the column words are the same for every thread: scalar loads, 16
        // columns per group, the distances' tests gathered into a mask
        const uint64_t x = sim[i];
        const int jmax = min(kHT, n - j0);
        const bool diag = bi == bj;  // only there can j <= i occur
        int c0 = 0;
        for (; c0 + 16 <= jmax; c0 += 16) {
            // bit u: the sign of max_dist - distance (distances and max_dist are
            // small non-negative integers), shifted in by a funnel shift
            uint32_t far = 0;
#pragma unroll
            for (int u = 15; u >= 0; --u)
                far = __builtin_amdgcn_alignbit(far, (uint32_t)(max_dist - __popcll(x ^ sim[j0 + c0 + u])), 31);
            uint32_t hit = ~far & 0xFFFFu;
            while (hit) {
                const int u = __builtin_ctz(hit);
                hit &= hit - 1;
                if (!diag || j0 + c0 + u > i) put(c0 + u, __popcll(x ^ sim[j0 + c0 + u]));
            }
        }
        for (int c = c0; c < jmax; ++c) {
            const int dist = __popcll(x ^ sim[j0 + c]);
            if (dist <= max_dist && (!diag || j0 + c > i)) put(c, dist);
        }
    }
    __syncthreads();
    const int cnt = min(scount, kHStage);
    if (threadIdx.x == 0 && cnt > 0) sbase = atomicAdd(sink.counter, (unsigned long long)cnt);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += 256) {
        const int64_t dst = (int64_t)sbase + e;
        if (dst < sink.capacity) sink.pairs[dst] = stage[e];
    }
}

}  // namespace

namespace mrc {

mrc_status launch_term_hashes(mrc_ctx* ctx, int32_t vocab, uint64_t* out, hipStream_t s) {
    Md5Consts c;
    for (int i = 0; i < 64; ++i) c.k[i] = (uint32_t)std::floor(std::fabs(std::sin((double)(i + 1))) * 4294967296.0);
    hipLaunchKernelGGL(k_term_hashes, dim3((unsigned)ceil_div(vocab, 256)), dim3(256), 0, s, vocab, c, out);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_simhash(mrc_ctx* ctx, const mrc_docs* docs, int32_t vocab, const uint64_t* d_hash, uint64_t* out,
                          hipStream_t s) {
    const int64_t n = docs->n_docs;
    MRC_TRY(launch_validate_offsets(ctx, docs, s));
    if (n == 0) return MRC_OK;
    ScopedTimer tm(ctx, "simhash", s);
    const int64_t grid = std::min<int64_t>(ceil_div(n, 4), 256 * 16);
    hipLaunchKernelGGL(k_simhash, dim3((unsigned)grid), dim3(256), 0, s, docs->offsets, n, docs->tokens, vocab, d_hash,
                       out, (unsigned long long*)ctx->d_flags);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_hamming(mrc_ctx* ctx, const uint64_t* sim, int64_t n, int32_t max_dist, PairSink sink,
                          hipStream_t s) {
    if (n < 2) return MRC_OK;
    const int nb = (int)ceil_div(n, kHT);
    const int64_t tiles = (int64_t)nb * (nb + 1) / 2;
    if (tiles > 0x7FFFFFFFLL) return fail(MRC_E_INVAL, "too many tiles for one launch");
    ScopedTimer tm(ctx, "hamming", s);
    hipLaunchKernelGGL(k_hamming, dim3((unsigned)tiles), dim3(256), 0, s, sim, (int)n, max_dist, nb, sink);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
