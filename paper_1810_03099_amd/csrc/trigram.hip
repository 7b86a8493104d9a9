// Character 3-gram front end (Sections 3-4: documents and the reference are
// vectors over character 3-grams). Raw bytes in, term ids out, in the token
// CSR that the rest of the library reads.
//
// Alphabet: the 26 ASCII letters, case-folded, are symbols 0-25; every other
// byte (space, digit, punctuation, control, any byte >= 0x80) is the one
// separator symbol 26. Every window of three consecutive bytes of a document
// is one 3-gram, id = 729 s0 + 27 s1 + s2 in [0, 19683); a document of L bytes
// gives max(L - 2, 0) ids, in text order.
//
// Passes: per-document id counts with a block total (also checks the
// offsets), an exclusive scan of the block totals (one workgroup), the
// output offsets; then the map itself, one wavefront per document, each lane
// loading eight aligned words of text per round and writing the ids that
// start in them.
#include "common.h"

using namespace mrc;

namespace {

constexpr int kTriBlock = 256;
constexpr int kTriPer = 8;                          // documents per thread in the offset passes
constexpr int kTriDocs = kTriBlock * kTriPer;       // documents per workgroup

__device__ __forceinline__ int tri_sym(unsigned b) {
    const unsigned l = (b | 0x20u) - (unsigned)'a';
    return l < 26u ? (int)l : 26;
}

__device__ __forceinline__ int64_t tri_count(const int64_t* __restrict__ off, int64_t d, int64_t n, int64_t n_bytes,
                                             bool* bad) {
    const int64_t a = off[d], b = off[d + 1];
    if (b < a || (d == 0 && a != 0) || (d == n - 1 && b != n_bytes)) *bad = true;
    const int64_t L = b - a;
    return L > 2 ? L - 2 : 0;
}

// Inclusive workgroup scan of one value per thread (four wavefronts).
__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t* lds_wave) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) lds_wave[w] = v;
    __syncthreads();
    int64_t base = 0;
    for (int i = 0; i < w; ++i) base += lds_wave[i];
    return v + base;
}

__global__ __launch_bounds__(kTriBlock) void k_tri_block_sums(const int64_t* __restrict__ off, int64_t n,
                                                              int64_t n_bytes, int64_t* __restrict__ bsum,
                                                              unsigned long long* __restrict__ err) {
    __shared__ int64_t wsum[kTriBlock / 64];
    const int64_t d0 = (int64_t)blockIdx.x * kTriDocs + (int64_t)threadIdx.x * kTriPer;
    bool bad = false;
    int64_t s = 0;
    for (int i = 0; i < kTriPer; ++i)
        if (d0 + i < n) s += tri_count(off, d0 + i, n, n_bytes, &bad);
    if (bad) atomicOr(err, kErrOffsets);
    const int64_t incl = block_incl_scan(s, wsum);
    if (threadIdx.x == kTriBlock - 1) bsum[blockIdx.x] = incl;
}

// Exclusive scan of nb block totals in place (one workgroup); the grand total
// goes to *total.
__global__ __launch_bounds__(kTriBlock) void k_tri_scan_sums(int64_t* __restrict__ bsum, int64_t nb,
                                                             int64_t* __restrict__ total) {
    __shared__ int64_t wsum[kTriBlock / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kTriBlock) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? bsum[b] : 0;
        const int64_t incl = block_incl_scan(v, wsum);
        const int64_t c = carry;
        if (b < nb) bsum[b] = c + incl - v;
        __syncthreads();  // every thread has read carry and wsum
        if (threadIdx.x == kTriBlock - 1) carry = c + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kTriBlock) void k_tri_offsets(const int64_t* __restrict__ off, int64_t n, int64_t n_bytes,
                                                           const int64_t* __restrict__ bsum,
                                                           int64_t* __restrict__ tok_off) {
    __shared__ int64_t wsum[kTriBlock / 64];
    const int64_t d0 = (int64_t)blockIdx.x * kTriDocs + (int64_t)threadIdx.x * kTriPer;
    bool bad = false;
    int64_t c[kTriPer];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kTriPer; ++i) {
        c[i] = d0 + i < n ? tri_count(off, d0 + i, n, n_bytes, &bad) : 0;
        s += c[i];
    }
    int64_t run = bsum[blockIdx.x] + block_incl_scan(s, wsum) - s;
#pragma unroll
    for (int i = 0; i < kTriPer; ++i) {
        if (d0 + i < n) tok_off[d0 + i] = run;
        run += c[i];
        if (d0 + i == n - 1) tok_off[n] = run;
    }
}

// Four bytes at the 4-byte-aligned address x, as a little-endian word; a word
// that reaches outside [lo, hi) is assembled from its bytes inside it (zero
// elsewhere), so no access leaves the caller's buffer.
// (The loads go through `text` itself, the buffer's first byte at address
// lo, so that they are global loads: through a pointer made from an integer
// they would be FLAT, after which every wait drains all loads in flight.)
__device__ __forceinline__ uint32_t tri_word(const uint8_t* __restrict__ text, uintptr_t x, uintptr_t lo,
                                             uintptr_t hi) {
    if (x >= lo && x + 4 <= hi) return *(const uint32_t*)(text + (x - lo));
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (x + i >= lo && x + i < hi) w |= (uint32_t)text[x + i - lo] << (8 * i);
    return w;
}

// One wavefront per document (grid-stride). A round covers 256 kTriWords
// window starts from a 4-byte-aligned address r: lane l loads the aligned
// words at r + 256 j + 4 l, j < kTriWords, all before any is used (so that a
// wavefront keeps 256 kTriWords bytes of text in flight). The ids are formed
// in store order: for each group of 256 window starts, store k has lane l
// write the window at 64 k + l, whose bytes it takes by shuffle from the two
// words that hold them (the last word's successor is the next group's first
// word, or lane 63's load past the round), so that every store instruction
// writes 256 contiguous bytes. A word is loaded only if it holds a byte some
// window needs. The next document's offsets are loaded before this one's text.
constexpr int kTriWords = 8;

__global__ __launch_bounds__(kTriBlock) void k_trigrams(const uint8_t* __restrict__ text, int64_t n_bytes,
                                                       const int64_t* __restrict__ off, int64_t n,
                                                       const int64_t* __restrict__ tok_off,
                                                       int32_t* __restrict__ out) {
    const int lane = __lane_id();
    const int64_t waves = (int64_t)gridDim.x * (kTriBlock / 64);
    const uintptr_t lo = (uintptr_t)text, hi = lo + (uintptr_t)n_bytes;
    int64_t d = (int64_t)blockIdx.x * (kTriBlock / 64) + (threadIdx.x >> 6);
    int64_t a = 0, e = 0, t0 = 0;
    if (d < n) {
        a = off[d];
        e = off[d + 1];
        t0 = tok_off[d];
    }
    for (; d < n; d += waves) {
        const int64_t dn = d + waves;
        int64_t an = 0, en = 0, tn = 0;
        if (dn < n) {
            an = off[dn];
            en = off[dn + 1];
            tn = tok_off[dn];
        }
        if (e - a >= 3) {
            const uintptr_t pa = lo + (uintptr_t)a, plast = lo + (uintptr_t)(e - 3);  // first / last window start
            const uintptr_t pend = plast + 2;                                            // last byte any window reads
            int32_t* __restrict__ o = out + t0;
            for (uintptr_t r = pa & ~(uintptr_t)3; r <= plast; r += 256 * kTriWords) {
                uint32_t w[kTriWords];
#pragma unroll
                for (int j = 0; j < kTriWords; ++j) {
                    const uintptr_t x = r + 256 * j + 4 * (uintptr_t)lane;
                    w[j] = x <= pend ? tri_word(text, x, lo, hi) : 0u;
                }
                const uintptr_t xt = r + 256 * kTriWords;
                const uint32_t tail = (lane == 63 && xt <= pend) ? tri_word(text, xt, lo, hi) : 0u;
                const uint32_t tail_all = __shfl(tail, 63, 64);
#pragma unroll
                for (int j = 0; j < kTriWords; ++j) {
                    // the word after this quarter's last one, on every lane
                    const uint32_t next_first =
                        j < kTriWords - 1 ? __shfl(w[j < kTriWords - 1 ? j + 1 : j], 0, 64) : tail_all;
                    // store instruction k writes window starts r + 256 j + 64 k + lane: the
                    // window's first byte is byte (lane mod 4) of lane 16 k + lane / 4's word
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int src = 16 * k + (lane >> 2);
                        const uint32_t wa = __shfl(w[j], src, 64);
                        const uint32_t wb0 = __shfl(w[j], (src + 1) & 63, 64);
                        const uint32_t wb = src == 63 ? next_first : wb0;
                        const uint64_t b = ((uint64_t)wa | ((uint64_t)wb << 32)) >> (8 * (lane & 3));
                        const uintptr_t q = r + 256 * j + 64 * k + (uintptr_t)lane;
                        if (q >= pa && q <= plast) {
                            const int s0 = tri_sym((unsigned)b & 0xffu);
                            const int s1 = tri_sym((unsigned)(b >> 8) & 0xffu);
                            const int s2 = tri_sym((unsigned)(b >> 16) & 0xffu);
                            o[q - pa] = s0 * 729 + s1 * 27 + s2;
                        }
                    }
                }
            }
        }
        a = an;
        e = en;
        t0 = tn;
    }
}

}  // namespace

namespace mrc {

// Offsets pass into tok_off (device, n + 1) and the id total into
// ctx->d_flags[1]; offset errors into ctx->d_flags[0].
mrc_status launch_trigram_offsets(mrc_ctx* ctx, const int64_t* off, int64_t n, int64_t n_bytes, int64_t* tok_off,
                                  hipStream_t s) {
    MRC_TRY(clear_words(ctx, ctx->d_flags, 2, s));
    if (n == 0) return MRC_OK;
    const int64_t nb = ceil_div(n, kTriDocs);
    void* bs = nullptr;
    MRC_TRY(scratch(ctx, "tri_bsum", (size_t)nb * 8, &bs));
    hipLaunchKernelGGL(k_tri_block_sums, dim3((unsigned)nb), dim3(kTriBlock), 0, s, off, n, n_bytes, (int64_t*)bs,
                       (unsigned long long*)ctx->d_flags);
    hipLaunchKernelGGL(k_tri_scan_sums, dim3(1), dim3(kTriBlock), 0, s, (int64_t*)bs, nb, ctx->d_flags + 1);
    hipLaunchKernelGGL(k_tri_offsets, dim3((unsigned)nb), dim3(kTriBlock), 0, s, off, n, n_bytes,
                       (const int64_t*)bs, tok_off);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

mrc_status launch_trigrams(mrc_ctx* ctx, const uint8_t* text, int64_t n_bytes, const int64_t* off, int64_t n,
                           const int64_t* tok_off, int32_t* out, hipStream_t s) {
    if (n == 0) return MRC_OK;
    ScopedTimer tm(ctx, "trigrams", s);
    const int64_t grid = std::min<int64_t>(ceil_div(n, kTriBlock / 64), 16384);
    hipLaunchKernelGGL(k_trigrams, dim3((unsigned)grid), dim3(kTriBlock), 0, s, text, n_bytes, off, n, tok_off, out);
    MRC_HIP_TRY(ctx, hipGetLastError());
    return MRC_OK;
}

}  // namespace mrc
