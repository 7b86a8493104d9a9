// Internal definitions shared by the HIP translation units of libmrc.
// Host-side: context, model and database objects, scratch arena, error and
// timing helpers. Device-side: wavefront reductions and small utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrc.h"

namespace mrc {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
mrc_status fail(mrc_status code, const std::string& msg);

#define MRC_HIP_TRY(ctx, expr)                                                         \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) return ::mrc::hip_fail((ctx), _e, #expr, __FILE__, __LINE__); \
    } while (0)

#define MRC_TRY(expr)                    \
    do {                                 \
        mrc_status _s = (expr);          \
        if (_s != MRC_OK) return _s;     \
    } while (0)

// ---------------------------------------------------------------- objects

// Per-term record the signing kernels gather once per token occurrence.
struct TermInfo {
    float idf;     // idf_t rounded to float
    int32_t part;  // reference part of t, -1 when t is not in the selection
};

struct KernelTimer {
    double total_ms = 0.0;
    int64_t launches = 0;
};

}  // namespace mrc

struct mrc_ctx {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;             // bytes held by scratch + owned objects
    mrc_status sticky = MRC_OK;  // a HIP failure poisons the context
    std::map<std::string, std::pair<void*, size_t>> scratch;
    // buffers a scratch entry outgrew: queued work may still use them, so they
    // are freed at teardown (or all at once, after one device-wide wait, when
    // they pass kRetiredMax) rather than each behind a device-wide wait
    std::vector<std::pair<void*, size_t>> retired;
    size_t retired_bytes = 0;
    int64_t* d_flags = nullptr;  // small device word array: counters + error flags
    int64_t* h_flags = nullptr;  // pinned host mirror
    bool timing = false;
    std::map<std::string, mrc::KernelTimer> timers;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> event_pool;
    std::mutex mu;               // guards `used` (databases may be touched by server threads)
    int tile_order_nb = -1;      // the band table in scratch "tile_order" is for this many tile rows
    int tile_order_bh = -1;      // ... and this band height
    int scan_form = 0;           // MRC_SCAN_GRID or MRC_SCAN_PERSISTENT (query collection)
    int query_attempts = 0;
    int64_t lowp_candidates = 0;  // candidates of the last low-precision mrc_compare (structured log)      // collection passes of the last mrc_query (above 1: capacity grew)
    void* model_spare = nullptr; // table block of the last destroyed model, kept for the next build
    size_t model_spare_bytes = 0;
    // Models and databases hold their context: destroyed while any of them
    // lives, the context is only marked (closing) and the last one released
    // frees it, so handles may be destroyed in any order.
    int live = 0;
    bool closing = false;
};

struct mrc_model {
    mrc_ctx* ctx = nullptr;
    int64_t n_docs = 0;
    int32_t vocab = 0;
    mrc_ref_spec spec{};
    int32_t k = 0;
    int64_t n_listed = 0, lo = 0, hi = 0;
    uint32_t* d_df = nullptr;        // [V]
    float* d_idf = nullptr;          // [V]
    int32_t* d_term_at = nullptr;    // [V]
    int32_t* d_rank_of = nullptr;    // [V]
    mrc::TermInfo* d_tinfo = nullptr;  // [V]
    double* d_rnorm = nullptr;       // [k]
    double* d_rinv = nullptr;        // [k]  1 / |r_j|
    uint64_t* d_hash = nullptr;      // [V]  MD5 term hashes (built on first use)
    size_t bytes = 0;                // the one device block holding d_df .. d_rinv (at d_df)
    mutable int users = 0;           // servers using the model (guarded by ctx->mu)
    mutable bool closing = false;    // destroyed while in use: freed when the last server stops
};

struct mrc_db {
    mrc_ctx* ctx = nullptr;
    int64_t capacity = 0;
    int64_t cap_pad = 0;         // capacity rounded up to 64 rows (padding rows stay zero)
    int32_t k = 0;
    uint32_t precisions = 0;
    int64_t size = 0;            // committed rows
    float* d_unit = nullptr;     // [cap_pad][kp] unit signatures, FP32 matrix-core layout
    uint16_t* d_bf16 = nullptr;  // [cap_pad][ldb]
    uint8_t* d_fp8 = nullptr;    // [cap_pad][ld8]
    float* d_scale = nullptr;    // [cap_pad]
    float* d_err = nullptr;      // [2][cap_pad]: bf16 then fp8 row error bounds
    float* d_errmax = nullptr;   // [2]: largest bf16 / fp8 row error bound of the committed rows
    size_t bytes = 0;
    std::mutex mu;
    int users = 0;               // servers using the database (guarded by ctx->mu)
    bool closing = false;        // destroyed while in use: freed when the last server stops
};

namespace mrc {

mrc_status hip_fail(mrc_ctx* ctx, hipError_t e, const char* what, const char* file, int line);
// Entry-point check of a context: not NULL, not poisoned; makes its device current.
mrc_status check_ctx(mrc_ctx* ctx, const char* fn);
// Resolves the device address of the fixed scratch array of the no-allocation
// comparison for `device` (current), once per device.
mrc_status noalloc_setup(int device);

// Context lifetime (see mrc_ctx::live): an object that holds the context
// retains it when created and releases it when freed; the release that ends
// a closing context frees it.
void ctx_retain(mrc_ctx* ctx);
void ctx_release(mrc_ctx* ctx);
void free_model(mrc_model* m);
void free_db(mrc_db* db);

// Device allocation accounted against the context budget.
mrc_status dev_alloc(mrc_ctx* ctx, void** p, size_t bytes);
void dev_free(mrc_ctx* ctx, void* p, size_t bytes);

// Named, grow-only scratch buffer owned by the context.
mrc_status scratch(mrc_ctx* ctx, const char* name, size_t bytes, void** p);

// Kernel timing around launches (no-ops when timing is off).
void timer_begin(mrc_ctx* ctx, const char* name, hipStream_t s, hipEvent_t* ev_pair);
void timer_end(mrc_ctx* ctx, const char* name, hipStream_t s, hipEvent_t* ev_pair);
void timer_collect(mrc_ctx* ctx);

// Structured log: env MRC_LOG = 0 (off, default) .. 3 and MRC_LOG_FILE (a path,
// default stderr), read once per process. One JSON object per line, each with
// "t_ms" (milliseconds since the library's first log line) and "event".
// Level 1: one line per main entry point call (status, sizes, counts, wall
// time); 2: also the call's per-kernel device times; 3: also one line per
// serving batch and the server's totals at stop.
int log_level();
void log_line(const std::string& event, const std::string& fields);  // fields: `"k": v, ...` or empty

// The log record of one entry point call (nothing unless MRC_LOG >= 1).
// Level 2 turns the context's kernel timers on for the call and reports what
// its kernels took.
struct CallLog {
    mrc_ctx* ctx;
    const char* name;
    bool on = false, timers = false, timing_was = false;
    double t0 = 0.0;
    std::map<std::string, KernelTimer> before;
    std::string fields;
    CallLog(mrc_ctx* c, const char* n);
    void add(const char* key, int64_t v);
    void add(const char* key, double v);
    mrc_status done(mrc_status st);  // writes the line; returns st
};

struct ScopedTimer {
    mrc_ctx* ctx;
    const char* name;
    hipStream_t s;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ScopedTimer(mrc_ctx* c, const char* n, hipStream_t st) : ctx(c), name(n), s(st) {
        timer_begin(ctx, name, s, ev);
    }
    ~ScopedTimer() { timer_end(ctx, name, s, ev); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- stage launchers
// Each returns MRC_OK or an error; all work is enqueued on `s`.

// Zero n 64-bit words at p with one small kernel (no fill-kernel split for
// unaligned ranges).
mrc_status clear_words(mrc_ctx* ctx, int64_t* p, int n, hipStream_t s);

// Clear the error word and check offsets on the device (kErrOffsets = bit 0);
// the document kernels return at once when it is set. With `lists`
// (kClasses n int32) it also lists the documents above kShortMax tokens by
// length class, their counts in ctx->d_flags[kClassCount + c] (it clears
// words 0 .. kClassCount + kClasses - 1 first).
mrc_status launch_validate_offsets(mrc_ctx* ctx, const mrc_docs* docs, hipStream_t s, int32_t* lists = nullptr);

// Distinct terms of each document of a corpus with their counts, at the
// document's token offset: term[off[d] + e], tf[off[d] + e] for e < nnz[d].
struct CountLists {
    int32_t* term;
    int32_t* tf;
    int32_t* nnz;
};
// Context scratch sized for `docs`.
mrc_status count_scratch(mrc_ctx* ctx, const mrc_docs* docs, CountLists* c);

// df over a corpus: the count lists, then one count per distinct (document,
// term). Also checks offsets and token ids (error bits in ctx->d_flags[0]).
mrc_status launch_df(mrc_ctx* ctx, const mrc_docs* docs, int32_t vocab, uint32_t* d_df, const CountLists& c,
                     hipStream_t s);

// The count pass alone: the distinct terms of each document with their counts
// (also checks offsets and token ids, error bits in ctx->d_flags[0]).
mrc_status launch_counts(mrc_ctx* ctx, const mrc_docs* docs, int32_t vocab, const CountLists& c, hipStream_t s);

// Signatures against the k columns of a dense [V][k] reference matrix R.
mrc_status launch_sign_matrix(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const float* R, int32_t k,
                              float* sig_out, float* norm_out, hipStream_t s);

// Signatures of the corpus whose count lists `c` holds (bit-identical to
// launch_sign on the same documents).
mrc_status launch_sign_counts(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const CountLists& c,
                              float* sig_out, float* norm_out, hipStream_t s);

// Unit TF-IDF vectors of a batch for the exact-cosine comparator: ranks < H in
// a dense [n_pad][ldh] matrix (matrix-core layout), the rest listed per
// document at its token offset.
struct CsrOut {
    int H, ldh;
    float* wh;
    int32_t* ent_rank;
    float* ent_w;
    int32_t* nnz_tail;
    uint32_t* pcount;   // [V - H] entries per tail rank
};
mrc_status launch_csr(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, const CsrOut& c, hipStream_t s);

// Model tables from df: idf, stable rank sort, selection, parts, reference norms.
mrc_status launch_model_tables(mrc_ctx* ctx, mrc_model* m, hipStream_t s);

// Signatures with a frozen model. unit_out optional: also write unit signatures.
mrc_status launch_sign(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, float* sig_out,
                       float* norm_out, hipStream_t s);

// Normalise + quantise rows.
// umfma (optional): unit signatures in the matrix-core layout, [roundup(n,64)][roundup(k,16)]
// with transposed 4x4 sub-blocks in each 16-column block and zero padding.
mrc_status launch_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit,
                            uint16_t* bf16, uint8_t* fp8, float* scale, float* err,
                            hipStream_t s, float* umfma = nullptr, int64_t* clear = nullptr, int n_clear = 0);

// Pair output buffer shared by the all-pairs kernels.
struct PairSink {
    mrc_pair* pairs;          // may be null when capacity == 0
    int64_t capacity;
    unsigned long long* counter;  // device: number of pairs found
};

// `table` (optional): device words for the tile order's band table (at least
// n / 64 / TileOrder::kBand + 2 of them), else the context's scratch holds it.
mrc_status launch_compare_f32(mrc_ctx* ctx, const float* umfma, int64_t n, int32_t k, float tau,
                              PairSink sink, hipStream_t s, int64_t* table = nullptr);
// 64x64-tile form of the same (allpairs_f32_small.hip; k <= 64 or k > 512).
mrc_status launch_compare_f32_small(mrc_ctx* ctx, const float* umfma, int64_t n, int32_t k, float tau,
                                    PairSink sink, hipStream_t s, int64_t* table = nullptr);

// Even number of 16x16 matrix-core steps (32 BF16 or 128 FP8 components)
// covering k: the column padding of the query kernels' code layouts.
int lowp_steps(int precision, int k);
// err: the rows' errors of the form's codes (FP8: each 32-row block's
// candidate threshold comes from its rows' largest error); tau, nominal: the
// comparison's threshold and nominal band.
mrc_status launch_compare_lowp(mrc_ctx* ctx, int32_t precision, const uint8_t* q, int ldq_bytes,
                               const float* scale, int64_t n, int32_t k, const float* d_lo_thr,
                               const float* err, float tau, float nominal, PairSink cand, hipStream_t s);
float lowp_acc_unit(int precision, int k);
mrc_status launch_lowp_threshold(mrc_ctx* ctx, int precision, const float* err, int64_t n, float tau,
                                 float nominal, int k, unsigned int* d_emax, float* d_out, hipStream_t s);
mrc_status launch_rescore2(mrc_ctx* ctx, int precision, const mrc_pair* cand, const unsigned long long* n_cand,
                           int64_t cand_cap, const float* unit, int32_t k, const float* err, float tau, float nominal,
                           PairSink out, unsigned long long* stats, hipStream_t s);
// Normalise with explicit layouts (see compare.hip).
// Outputs of the normalisation kernel. umfma holds the unit signatures for the
// FP32 matrix cores: with frag == 0 row-major (ld_mfma floats per row, 4x4
// sub-blocks of each 16-column block transposed, see mfma_col); with
// frag != 0 fragment-major: fragment (16-row block rb, 16-column chunk c) is
// 64 lanes x 4 floats at ((rb * ld_mfma / 16 + c) * 64 + lane) * 4, lane
// l = li + 16 g holding components 16c + 4m + g (m = 0..3) of row 16rb + li,
// so each operand load of the all-pairs kernel reads 1 KB contiguously.
struct NormLayout {
    float* unit;      int ld_unit;
    uint16_t* bf16;   int ld_bf16;
    uint8_t* fp8;     int ld_fp8;
    float* scale;
    float* err;       int64_t ld_err;
    float* umfma;     int ld_mfma;
    int64_t n_pad;
    int frag = 0;
    int errs = 3;     // row errors formed: bit 0 BF16, bit 1 FP8 (the other half of err is 0)
    int64_t* clear = nullptr;  // words (at most 256) zeroed by the normalising launch: the
    int n_clear = 0;           // counters of the kernels that follow it on the stream
};

// Offset of component c of row r in the fragment-major FP32 layout with nc
// 16-column chunks.
__host__ __device__ __forceinline__ int64_t frag_offset(int64_t r, int c, int nc) {
    return (((r >> 4) * nc + (c >> 4)) * 64 + (r & 15) + 16 * (c & 3)) * 4 + ((c >> 2) & 3);
}
mrc_status launch_normalise_rows(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, const NormLayout& o,
                                 hipStream_t s);
mrc_status launch_score_pairs(mrc_ctx* ctx, const float* unit, int32_t k, const int32_t* ii,
                              const int32_t* jj, int64_t n_pairs, float* out, hipStream_t s);

// Comparators.
mrc_status launch_term_hashes(mrc_ctx* ctx, int32_t vocab, uint64_t* out, hipStream_t s);
mrc_status launch_simhash(mrc_ctx* ctx, const mrc_docs* docs, int32_t vocab, const uint64_t* d_hash,
                          uint64_t* out, hipStream_t s);
mrc_status launch_hamming(mrc_ctx* ctx, const uint64_t* sim, int64_t n, int32_t max_dist,
                          PairSink sink, hipStream_t s);
mrc_status launch_exact_cosine(mrc_ctx* ctx, const mrc_model* m, const mrc_docs* docs, float tau,
                               PairSink sink, hipStream_t s);
// Character 3-grams: output offsets (and the id total in ctx->d_flags[1]),
// then the ids themselves.
mrc_status launch_trigram_offsets(mrc_ctx* ctx, const int64_t* off, int64_t n, int64_t n_bytes, int64_t* tok_off,
                                  hipStream_t s);
mrc_status launch_trigrams(mrc_ctx* ctx, const uint8_t* text, int64_t n_bytes, const int64_t* off, int64_t n,
                           const int64_t* tok_off, int32_t* out, hipStream_t s);

// Leading dimensions (elements) of the database / query layouts for k.
struct DbLayout {
    int kp;    // FP32 matrix-core layout
    int ldb;   // BF16 codes
    int ld8;   // FP8 codes
};
DbLayout db_layout(int32_t k);

// Query top-k against a database.
mrc_status run_query(mrc_ctx* ctx, const mrc_db* db, int64_t db_rows, const mrc_model* m,
                     const mrc_docs* q, int32_t topk, float tau, int32_t precision,
                     mrc_hit* topk_out, int32_t* n_hits, hipStream_t s);

// Normalise and append unit signatures to a database.
mrc_status db_append(mrc_db* db, const float* sig, int64_t n, int64_t first, hipStream_t s);
// Raise errmax[0] / errmax[1] to the largest of the n row error bounds e16[i] /
// e8[i] (non-negative floats).
mrc_status launch_err_max(mrc_ctx* ctx, const float* e16, const float* e8, int64_t n, float* errmax, hipStream_t s);

// Upper-triangle tile schedule for the all-pairs kernels. Tile rows are grouped
// in bands of kBand rows; a band lists its tiles column by column (inside a
// column, row by row), so consecutive tiles share the column panel and a band
// reuses its row panels. Workgroups are dispatched round-robin over the 8
// XCDs; the schedule gives each XCD a contiguous range of the band order, so
// the panels a range touches stay in that XCD's L2.
struct TileOrder {
    int nb;                 // tile rows (= tile columns)
    int n_bands;
    int per_block;          // tiles per workgroup
    int64_t n_tiles;
    int64_t blocks;         // workgroups that carry tiles
    int64_t per_xcd;        // ceil(blocks / 8)
    const int64_t* band_start;  // device [n_bands + 1]: first tile index of each band
    int bh;                     // tile rows per band (the last band may hold fewer)
    static constexpr int kBand = 8;  // default band height

    // Position of one wavefront in the band order: its current band and the
    // band's first and one-past-last tile indices (all wavefront-uniform).
    struct Cursor {
        int band;
        int64_t start, next;
    };

    // Cursor at tile t (binary search over the band starts; once per wavefront).
    __device__ __forceinline__ Cursor seek(int64_t t) const {
        int lo = 0, hi = n_bands - 1;                   // band: last start <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (band_start[mid] <= t) lo = mid; else hi = mid - 1;
        }
        return Cursor{lo, band_start[lo], band_start[lo + 1]};
    }

    // Coordinates of tile t >= the cursor's tile (the cursor moves forward).
    // Call with a wavefront-uniform t: everything here is then scalar, and
    // memory is only read when t enters a later band.
    __device__ __forceinline__ void tile(Cursor& c, int64_t t, int* bi, int* bj) const {
        while (t >= c.next) {
            ++c.band;
            c.start = c.next;
            c.next = band_start[c.band + 1];
        }
        const int r0 = c.band * bh;
        const int h = min(bh, nb - r0);
        int q = (int)(t - c.start);                     // < kBand * nb
        const int tri = h * (h + 1) / 2;
        if (q < tri) {                                  // columns r0 .. r0+h-1: J - r0 + 1 tiles each
            int col = 0;
            while ((col + 1) * (col + 2) / 2 <= q) ++col;
            *bj = r0 + col;
            *bi = r0 + (q - col * (col + 1) / 2);
        } else {
            q -= tri;
            const int col = q / h;
            *bj = r0 + h + col;
            *bi = r0 + (q - col * h);
        }
    }
};

// The band table goes to `table` (device, n_bands + 1 words) when given, else
// to context scratch (kept for the next call with the same tile count).
mrc_status make_tile_order(mrc_ctx* ctx, int nb, int per_block, TileOrder* ord, int64_t* grid, hipStream_t s,
                           int64_t* table = nullptr, int band_h = TileOrder::kBand);
// Low-precision candidate kernels (lds_allpairs.hip, LDS-tiled 256x256 blocks),
// called by launch_compare_lowp. The codes need ceil(n / 256) * 256 rows of
// ldq_bytes = 128 * lowp_lds_chunks(precision, k) bytes, zero padded; the FP8
// row scales are powers of two.
int lowp_lds_chunks(int precision, int k);  // -1: k too large for the form
mrc_status launch_compare_bf16(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, int64_t n, const float* d_lo_thr,
                               PairSink cand, hipStream_t s);
// Candidate threshold of a 32x32 block of FP8 scores (rows of block x, columns
// of block y): min(t_nom, c - g (1 + E_x)(1 + E_y)), E = the block's largest
// row error. (1 + a)(1 + e_i)(1 + e_j) - 1 + 2^-20 is the pair band's bound
// term, so with E >= e and the margin folded into c and t_nom it is at most
// every pair's own lower threshold tau - band(e_i, e_j).
struct BlockBand {
    const float* blk_err;  // device [rows of the codes / 32]: largest row error per block (0 past the last row)
    float c;               // tau + 1 - 2^-20 - margin
    float t_nom;           // tau - nominal - margin
    float g;               // 1 + accumulation allowance
};
mrc_status launch_compare_fp8(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, const float* scale, int64_t n,
                              const float* d_lo_thr, BlockBand bb, PairSink cand, hipStream_t s);
// Workgroups of a persistent launch: as many as are resident at once on the
// device (occupancy x CUs), rounded down to a multiple of the 8 XCDs and at most
// `cap`.
int64_t persistent_grid(mrc_ctx* ctx, const void* kernel, int block, int64_t cap);

// Number of 16-column chunks of the FP32 matrix-core layout for k components
// (rounded up to an instantiated count); the layout has 16 * mfma_chunks(k) columns.
int mfma_chunks(int k);

// Sizes of the length classes the document kernels use.
constexpr int kShortMax = 512;    // one wavefront per document, LDS hash table
constexpr int kMidMax = 2048;     // one 256-thread workgroup per document: 4096-slot table
constexpr int kMedMax = 4096;     //   ... 8192-slot table
constexpr int kMediumMax = 8192;  //   ... 16384-slot table; longer documents: global tables
// Documents above kShortMax are listed by length class (c = 0: up to kMidMax,
// 1: kMedMax, 2: kMediumMax, 3: longer) in lists[c n ..), with the class
// counts in context words kClassCount + c.
constexpr int kClasses = 4;
constexpr int kClassCount = 9;
// Largest signature length of queries against a database (the query scans are
// instantiated up to 32 FP32 / 16 BF16 chunks).
constexpr int kQueryMaxK = 512;
constexpr int kLongBlocks = 64;   // workgroups of the long-document pass (each owns a [V] table)
constexpr int64_t kMaxDocLen = 1 << 22;  // longest document (exact 64/128-bit sums below this)

// Error bits of ctx->d_flags[0], set by kernels and decoded after the call.
constexpr unsigned long long kErrOffsets = 1, kErrToken = 2, kErrSelection = 4, kErrTailCap = 8,
                             kErrQueryCap = 16, kErrDocLen = 32;
// Context word of the query collection's capacity signal (kErrQueryCap): kept
// apart from word 0, whose input-error bits the query's signing pass sets.
constexpr int kQueryCapWord = 40;

}  // namespace mrc

// ---------------------------------------------------------------- device helpers

namespace mrc_dev {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Column position of component c in the FP32 matrix-core layout: inside each
// block of 16 components the 4x4 sub-blocks are transposed, so that lane group
// g loading 4 consecutive floats at 4g feeds MFMA step m with component 4m + g.
__host__ __device__ __forceinline__ int mfma_col(int c) { return (c & ~15) | ((c & 3) << 2) | ((c >> 2) & 3); }

// Fixed-order wavefront sum (butterfly over 64 lanes). Every lane receives
// the same value, computed by the same tree regardless of data.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Exact fixed-point form of a non-negative float c with 2^-9 <= c < 2^24:
// c * 2^32 is then an integer below 2^56, returned as uint64. Sums of such
// values are exact and independent of order.
__device__ __forceinline__ unsigned long long fixed32(float c) {
    unsigned int hi = (unsigned int)c;          // truncation, exact integer part
    float frac = c - (float)hi;                 // exact (same binade or below)
    unsigned int lo = (unsigned int)(frac * 4294967296.0f);  // exact: power-of-two scale
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ double unfixed32(unsigned long long v) {
    return (double)v * 2.3283064365386963e-10;  // 2^-32
}

// Reserve `mine` consecutive output slots per lane with one atomic per
// wavefront. Returns this lane's first slot. All 64 lanes must call it.
__device__ __forceinline__ int64_t wave_reserve(unsigned long long* counter, int mine) {
    const int lane = __lane_id();
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (total > 0 && lane == 63) base = atomicAdd(counter, (unsigned long long)total);
    base = __shfl(base, 63, 64);
    return (int64_t)base + incl - mine;
}

}  // namespace mrc_dev
