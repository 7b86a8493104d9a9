/*
 * mrc.h - C ABI of the Multi-reference Cosine (MRC) near-duplicate engine for
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Mohammadi & Nikoukaran, "Multi-reference Cosine: A New Approach
 * to Text Similarity Measurement in Large Collections", arXiv 1810.03099):
 *   - a document is a vector of term counts, compared by cosine (Section 3,
 *     Eq. 1); here terms are integer ids and counts are TF-IDF weighted (the
 *     weighted vector-space model of Section 6);
 *   - a reference is the frequency-sorted term list without zero-frequency
 *     terms, optionally cut to a frequency region or the rarest terms, split
 *     into k equal parts; a document's signature is its cosine against each
 *     part (Section 4);
 *   - signatures are compared by cosine to flag duplicates and near
 *     duplicates, and each new document is compared with the whole signature
 *     database (Section 1);
 *   - Simhash with Hamming distance is the rival method (Section 3) and exact
 *     cosine the ground truth (Section 5).
 *
 * Conventions for every call:
 *   - Pointers marked "device" are device memory of the context's GPU, owned
 *     by the caller; the library never frees caller memory. Pointers marked
 *     "host" are host memory owned by the caller.
 *   - hip_stream is a hipStream_t (NULL = the default stream). Device work of
 *     a call is ordered on that stream. Unless stated otherwise a call
 *     synchronises the stream before it returns, so that its status (and any
 *     count it returns) covers all of its device work.
 *   - Return value: MRC_OK or a negative status. mrc_last_error() returns a
 *     thread-local message for the last failure of the calling thread.
 *   - A context is used by one host thread at a time (the serving API runs its
 *     own threads on its own internal state).
 *   - No exception crosses this boundary.
 */
#ifndef MRC_H
#define MRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mrc_status;

#define MRC_OK 0
#define MRC_E_INVAL (-1)    /* bad argument or bad input data (token id out of range, ...) */
#define MRC_E_NOMEM (-2)    /* device allocation failed or would exceed the context budget */
#define MRC_E_OVERFLOW (-3) /* output capacity too small; the exact required count is returned */
#define MRC_E_HIP (-4)      /* a HIP runtime error; sticky on the context */
#define MRC_E_BUSY (-5)     /* serving admission refused (budget or queue full) */
#define MRC_E_STATE (-6)    /* call not valid in the object's current state */

/* Reference selection over the frequency-sorted term list (Section 4). V' is
 * the number of terms with non-zero document frequency. */
#define MRC_SEL_ALL 0       /* positions [0, V'): every listed term */
#define MRC_SEL_REGION 1    /* positions [lo, hi), hi < 0 means V' (a frequency region) */
#define MRC_SEL_RAREST 2    /* positions [V' - m, V'): the m least frequent terms */
#define MRC_SEL_DROP_TOP 3  /* positions [ceil(V' * drop_top_ppm / 1e6), V') */

#define MRC_IDF_SMOOTH 0    /* idf = ln((1 + N) / (1 + df)) + 1, rounded once to float */
#define MRC_IDF_NONE 1      /* idf = 1: raw term counts, the paper's unweighted vectors */

#define MRC_REF_ONE 0       /* reference part = indicator vector of its terms */
#define MRC_REF_IDF 1       /* reference part carries its terms' idf */

#define MRC_PREC_FP32 0     /* plain path: float32 multiply-add chain in ascending component order,
                               run on the FP32 matrix cores (16x16x4 steps keep that order) */
#define MRC_PREC_BF16 1     /* bfloat16 matrix cores, FP32 accumulate, band rescored in FP32 */
#define MRC_PREC_FP8 2      /* float8 e4m3fn with per-row FP32 scale, band rescored in FP32 */

typedef struct mrc_ctx mrc_ctx;
typedef struct mrc_model mrc_model;
typedef struct mrc_db mrc_db;
typedef struct mrc_server mrc_server;

/* A batch of documents as a token CSR: document d owns
 * tokens[offsets[d] .. offsets[d+1]). offsets: device int64 [n_docs + 1],
 * offsets[0] = 0, non-decreasing, offsets[n_docs] <= n_tokens. tokens: device
 * int32 term ids, n_tokens entries readable. Offsets are validated on the
 * device before any token is read (MRC_E_INVAL when malformed). */
typedef struct {
    int64_t n_docs;
    const int64_t* offsets;
    const int32_t* tokens;
    int64_t n_tokens;
} mrc_docs;

/* How the reference is chosen and split (Section 4). k parts of equal length
 * over the selected m positions; the first m mod k parts hold one extra term.
 * Ties in the frequency-sorted list are broken by ascending term id. */
typedef struct {
    int32_t k;
    int32_t mode;          /* MRC_SEL_* */
    int64_t lo, hi;        /* MRC_SEL_REGION */
    int64_t m;             /* MRC_SEL_RAREST */
    int64_t drop_top_ppm;  /* MRC_SEL_DROP_TOP, parts per million of V' */
    int32_t idf_mode;      /* MRC_IDF_* */
    int32_t ref_weight;    /* MRC_REF_* */
} mrc_ref_spec;

/* Options of the all-pairs comparison. */
typedef struct {
    float tau;             /* a pair i < j is flagged when its similarity >= tau */
    int32_t precision;     /* MRC_PREC_* */
    float band;            /* nominal rescoring half-width for BF16/FP8 (e.g. 0.02); the
                              FP8 form widens it per pair to its proven error bound */
    int32_t reserved;      /* must be 0 */
} mrc_compare_opts;

/* One flagged pair, i < j. s is the reported similarity: the FP32 plain score
 * for MRC_PREC_FP32 and for rescored pairs, else the low-precision score.
 * flags bit 0: the pair was rescored in FP32. */
typedef struct {
    int32_t i;
    int32_t j;
    float s;
    int32_t flags;
} mrc_pair;

/* One query hit: database id and similarity. */
typedef struct {
    int64_t id;
    float s;
    int32_t flags;
} mrc_hit;

/* Counters of one comparison (all pairs i < j). */
typedef struct {
    int64_t n_pairs_compared;   /* n (n - 1) / 2 */
    int64_t n_flagged;          /* pairs with final decision >= tau */
    int64_t n_band;             /* low-precision pairs rescored in FP32 */
    int64_t n_band_nominal;     /* of those, pairs within the nominal band */
    int64_t n_flip_outside_nominal; /* rescored pairs outside the nominal band whose
                                       decision the low-precision score would have
                                       got wrong: the flips a fixed +-band would miss */
    float max_abs_err;          /* max |low-precision score - FP32 score| over rescored pairs */
    float mean_abs_err;         /* mean of the same */
} mrc_compare_stats;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`. hbm_budget_bytes caps the device
 * memory the context itself allocates (scratch, models, databases); 0 means
 * 80% of the device's memory. */
mrc_status mrc_ctx_create(mrc_ctx** out, int32_t device, size_t hbm_budget_bytes);
/* Destroy a context. Models and databases created on it keep it alive: with
 * any of them left, the context is freed when the last one is destroyed (no
 * further calls on the context itself are allowed after this one). */
mrc_status mrc_ctx_destroy(mrc_ctx* ctx);
/* Device bytes currently allocated by the context (scratch + owned objects). */
mrc_status mrc_ctx_memory(const mrc_ctx* ctx, size_t* used, size_t* budget);
/* Kernel timing: when enabled, the library records HIP events around each of
 * its kernels on the launch stream and accumulates per-kernel durations.
 * mrc_ctx_kernel_time fetches (and with reset != 0 clears) the totals for a
 * kernel name; unknown names give count 0. */
mrc_status mrc_ctx_set_timing(mrc_ctx* ctx, int32_t enabled);
mrc_status mrc_ctx_kernel_time(mrc_ctx* ctx, const char* kernel, double* total_ms,
                               int64_t* launches, int32_t reset);

/* Form of the query collection pass (Section 1: each new document against
 * the whole signature database) used by mrc_query and by servers started on
 * this context afterwards. MRC_SCAN_GRID (default): each workgroup strides
 * over the database tiles of one query block. MRC_SCAN_PERSISTENT: as many
 * workgroups as are resident at once take (query block, 16-tile range) items
 * in order from a device work counter until none is left. Both give the same
 * results. Errors: MRC_E_INVAL for another form. */
#define MRC_SCAN_GRID 0
#define MRC_SCAN_PERSISTENT 1
mrc_status mrc_ctx_set_scan(mrc_ctx* ctx, int32_t form);

/* Thread-local message of the last failed call on this thread. */
const char* mrc_last_error(void);

/* ------------------------------------------------------------------ model */

/* Build the model of a corpus (Section 4): term counts per document, document
 * frequency df over the corpus, idf, the frequency-sorted list of terms with
 * df > 0 (df descending, id ascending), the selection and its k parts.
 * vocab_size: term ids must lie in [0, vocab_size), vocab_size <= 2^24.
 * Errors: MRC_E_INVAL for a bad spec, a selection with fewer than k terms, an
 * out-of-range token, malformed offsets or a document longer than 2^22
 * tokens. */
mrc_status mrc_build_vocab_idf(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size,
                               const mrc_ref_spec* spec, mrc_model** out, void* hip_stream);
/* Destroy a model (waits for the device). A model that a running server
 * uses is freed when the last such server stops. */
mrc_status mrc_model_destroy(mrc_model* model);
/* Shape of a model: number of model documents, vocabulary, k, V' (listed
 * terms) and the selected positions [lo, hi). Any output may be NULL. */
mrc_status mrc_model_info(const mrc_model* model, int64_t* n_docs, int32_t* vocab, int32_t* k,
                          int64_t* n_listed, int64_t* lo, int64_t* hi);
/* Copy model tables to host memory (any pointer may be NULL):
 * df uint32 [V], idf float [V], term_at int32 [V] (the sorted list; entries
 * at positions >= V' are the df = 0 terms in ascending id), rank_of int32 [V]
 * (inverse of term_at), part_of int32 [V] (reference part, -1 if not
 * selected), rnorm double [k] (|r_j|). */
mrc_status mrc_model_get(const mrc_model* model, uint32_t* df, float* idf, int32_t* term_at,
                         int32_t* rank_of, int32_t* part_of, double* rnorm);
/* Serialise a model to / from a host file (versioned header + checksum). */
mrc_status mrc_model_save(const mrc_model* model, const char* path);
mrc_status mrc_model_load(mrc_ctx* ctx, const char* path, mrc_model** out);

/* ------------------------------------------------------------------ signing */

/* MRC signatures (Section 4) with the frozen model:
 * sig[d][j] = (sum over terms t of part j of w_dt * rho_t) / (|w_d| * |r_j|),
 * w_dt = tf * idf_t, 0 for an empty document. Terms with df = 0 in the model
 * corpus count in |w_d| (with their smoothed idf) but belong to no part.
 * sig_out: device float [n_docs][k] row-major. norm_out: device float [n_docs]
 * (|w_d|) or NULL. The part sums and |w_d|^2 are accumulated exactly (integer
 * fixed point), so a document's signature does not depend on the batch it is
 * signed in. Documents may hold at most 2^22 tokens. Errors: MRC_E_INVAL for a
 * token outside [0, V), bad offsets or a longer document. */
mrc_status mrc_sign(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, float* sig_out,
                    float* norm_out, void* hip_stream);

/* Signatures against k general reference vectors (Section 4's construction
 * with the weighted vector-space models of Section 6): the columns of a dense
 * matrix R, whose entries may weight their terms and whose columns may share
 * terms. sig[d][j] = (sum over the document's terms t of w_dt R[t][j]) /
 * (|w_d| |r_j|), with w_dt = tf * idf_t under `model` (its idf and frequency
 * order only; its own parts play no role) and |r_j| the Euclidean norm of
 * column j; 0 when either norm is 0. The model's parts as columns (R[t][part
 * of t] = rho_t) give mrc_sign's signature.
 * R: device float [V][k] row-major (row t = term t's weight in every
 * reference), V = the model's vocabulary; caller-owned, read only. k in
 * [1, 1024]. sig_out: device float [n_docs][k]; norm_out as mrc_sign (the
 * same exact |w_d|). The numerators are float64 sums in the order of each
 * document's distinct-term list, rounded once to float. Errors: those of
 * mrc_sign; MRC_E_INVAL for k outside [1, 1024] or a NULL R. */
mrc_status mrc_sign_matrix(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, const float* R,
                           int32_t k, float* sig_out, float* norm_out, void* hip_stream);

/* Build the model of a corpus and sign that corpus (Sections 1 and 4: the
 * signature database of a collection) in one call, reusing the per-document
 * term counts of the build. Same result as mrc_build_vocab_idf followed by
 * mrc_sign on the same documents, bit for bit. sig_out: device float
 * [n_docs][k] (may be NULL only for an empty corpus); norm_out as mrc_sign.
 * Errors: those of mrc_build_vocab_idf and mrc_sign. */
mrc_status mrc_build_and_sign(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size,
                              const mrc_ref_spec* spec, mrc_model** out, float* sig_out, float* norm_out,
                              void* hip_stream);

/* ------------------------------------------------------------------ comparison */

/* All-pairs signature comparison: MRC(i, j) = cosine of the two signatures
 * (Eq. 1 on signatures; the similarity Eq. 2 calls multi reference cosine),
 * 0 when either is zero. Flags every pair i < j with MRC(i, j) >= tau.
 * sig: device float [n][k] (raw or normalised signatures). pairs_out: device
 * mrc_pair [capacity] (may be NULL when capacity is 0); pairs are written in
 * unspecified order. n_found: host, receives the number of flagged pairs. If
 * it exceeds capacity the call returns MRC_E_OVERFLOW, writes the first
 * `capacity` pairs found and the exact count: call again with a larger buffer.
 * stats: host, may be NULL.
 * FP32: the score is acc = 0; acc = fmaf(u_ic, u_jc, acc) for c = 0..k-1 over
 * the unit signatures u = sig / |sig| (float32). BF16 and FP8 score on the
 * matrix cores and rescore in FP32 every pair within their error band of tau,
 * so their decisions equal the FP32 decisions. */
mrc_status mrc_compare(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k,
                       const mrc_compare_opts* opts, mrc_pair* pairs_out, int64_t capacity,
                       int64_t* n_found, mrc_compare_stats* stats, void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc. The FP32 form
 * of mrc_compare (same kernels, same pairs and scores, bit for bit) with its
 * working memory (pair counter, tile-order table, unit signatures in the
 * matrix-core layout) in a fixed device array of the library, one per GPU,
 * held from the first mrc_ctx_create on that GPU until the process ends. The
 * call allocates nothing; the caller passes inputs and outputs as for
 * mrc_compare (sig device float [n][k]; pairs_out device mrc_pair [capacity];
 * n_found host).
 * Limit: ceil(n / 128) * 128 rows x 16 * mfma_chunks(k) columns x 4 bytes
 * (columns = k rounded up to 32, 64, 96, 128, 192, 256, 384, 512, 768 or
 * 1024) must not exceed MRC_NOALLOC_MAX_UNIT_BYTES (32 MiB), e.g.
 * n <= 131,072 at k = 64 and n <= 32,768 at k = 256; larger inputs return
 * MRC_E_INVAL before any device work. The array is that plus 8 KiB.
 * Every call on one GPU uses that GPU's array, so calls that overlap on one
 * GPU (several streams or threads) race; the array keeps the last call's
 * contents (the call clears what must start at zero). Synchronises the stream
 * (it returns the count). Errors: MRC_E_INVAL (sizes, NULL buffers, NaN tau),
 * MRC_E_OVERFLOW (two-call protocol as mrc_compare), MRC_E_STATE (the array
 * was not set up on this GPU), MRC_E_HIP. */
#define MRC_NOALLOC_MAX_UNIT_BYTES ((size_t)32 << 20)
mrc_status mrc_compare_f32_noalloc(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float tau,
                                   mrc_pair* pairs_out, int64_t capacity, int64_t* n_found, void* hip_stream);

/* Unit signatures and their low-precision forms, as mrc_compare uses them.
 * unit_out: device float [n][k] (may be NULL); bf16_out: device uint16 [n][k]
 * (bfloat16 bits, round to nearest even; may be NULL); fp8_out: device uint8
 * [n][k] (float8 e4m3fn bits of u / scale, round to nearest even; may be
 * NULL); scale_out: device float [n] with scale = the smallest power of two
 * >= max_c |u_c| / 448 (the quotient in float32; an E8M0 operand scale of the
 * matrix cores; may be NULL); err_out: device float [2][n]: per-row |u - dequantised|_2 bounds for
 * bf16 then fp8 (may be NULL). */
mrc_status mrc_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit_out,
                         uint16_t* bf16_out, uint8_t* fp8_out, float* scale_out, float* err_out,
                         void* hip_stream);

/* FP32 plain score of listed pairs over unit signatures (the rescoring chain).
 * unit: device float [n][k]; ii, jj: device int32 [n_pairs]; out: device float. */
mrc_status mrc_score_pairs(mrc_ctx* ctx, const float* unit, int64_t n, int32_t k,
                           const int32_t* ii, const int32_t* jj, int64_t n_pairs, float* out,
                           void* hip_stream);

/* ------------------------------------------------------------------ text front end */

/* Character 3-grams of raw text (Sections 3-4: documents and the reference
 * are vectors over character 3-grams), as token ids for the other calls.
 * Case-folded ASCII letters are symbols 0-25; every other byte is the
 * separator symbol 26. Each window of three consecutive bytes of a document
 * gives id 729 s0 + 27 s1 + s2 in [0, 19683), in text order: a document of L
 * bytes gives max(L - 2, 0) ids (vocab_size 19683 for the model calls).
 *   text:            device bytes [n_bytes].
 *   text_offsets:    device int64 [n_docs + 1], nondecreasing, first 0, last n_bytes.
 *   tok_offsets_out: device int64 [n_docs + 1], written: the ids' CSR offsets.
 *   tokens_out:      device int32 [capacity]; may be NULL when capacity is 0.
 *   n_tokens:        host; receives the total number of ids.
 * Two-call protocol: if the total exceeds capacity the call writes the
 * offsets and *n_tokens, writes no ids and returns MRC_E_OVERFLOW. Malformed
 * offsets: MRC_E_INVAL, nothing usable written. The caller owns every buffer;
 * the ids are ready when the stream reaches the end of the call's work. */
mrc_status mrc_trigrams(mrc_ctx* ctx, const uint8_t* text, const int64_t* text_offsets, int64_t n_docs,
                        int64_t n_bytes, int64_t* tok_offsets_out, int32_t* tokens_out, int64_t capacity,
                        int64_t* n_tokens, void* hip_stream);

/* ------------------------------------------------------------------ comparators */

/* Simhash-64 of each document (Section 3): term t hashes to the first 8 bytes
 * (little-endian) of MD5 over its 4-byte little-endian id; every occurrence
 * adds +1 to column b if bit b of its hash is 1, else -1; bit b of the result
 * is 1 iff the column sum is > 0. out: device uint64 [n_docs]. */
mrc_status mrc_simhash(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, uint64_t* out,
                       void* hip_stream);
/* MD5 term-hash table of the model's vocabulary. out: device uint64 [V]. */
mrc_status mrc_term_hashes(mrc_ctx* ctx, const mrc_model* model, uint64_t* out, void* hip_stream);
/* All pairs i < j with Hamming(sim_i, sim_j) <= max_dist (Section 3).
 * Two-call protocol and outputs as mrc_compare; s holds the distance. */
mrc_status mrc_hamming_pairs(mrc_ctx* ctx, const uint64_t* sim, int64_t n, int32_t max_dist,
                             mrc_pair* pairs_out, int64_t capacity, int64_t* n_found,
                             void* hip_stream);
/* Exact cosine (Eq. 1) of the TF-IDF vectors of all pairs i < j, flagged at
 * >= tau: the ground truth of Section 5. Two-call protocol as mrc_compare. */
mrc_status mrc_exact_cosine(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, float tau,
                            mrc_pair* pairs_out, int64_t capacity, int64_t* n_found,
                            void* hip_stream);

/* ------------------------------------------------------------------ database + query */

/* A resident signature database (Section 1: each new page is compared with
 * all pages through their signatures). Holds unit signatures in FP32 and the
 * low-precision copies selected by `precisions` (bit MRC_PREC_BF16 -> 1<<1,
 * MRC_PREC_FP8 -> 1<<2; FP32 is always kept, it is the rescoring source).
 * Ids are assigned in insertion order from 0; the database is append-only. */
mrc_status mrc_db_create(mrc_ctx* ctx, int64_t capacity, int32_t k, uint32_t precisions,
                         mrc_db** out);
/* Destroy a database (waits for the device). A database that a running
 * server uses is freed when the last such server stops. */
mrc_status mrc_db_destroy(mrc_db* db);
/* Append n signatures (device float [n][k], raw or unit). first_id: host, may
 * be NULL. Errors: MRC_E_OVERFLOW when capacity would be exceeded. */
mrc_status mrc_db_insert(mrc_db* db, const float* sig, int64_t n, int64_t* first_id,
                         void* hip_stream);
/* Sign documents with the model and append them. */
mrc_status mrc_db_insert_docs(mrc_db* db, const mrc_model* model, const mrc_docs* docs,
                              int64_t* first_id, void* hip_stream);
mrc_status mrc_db_size(const mrc_db* db, int64_t* n, int32_t* k);
mrc_status mrc_db_save(const mrc_db* db, const char* path);
mrc_status mrc_db_load(mrc_ctx* ctx, const char* path, uint32_t precisions, mrc_db** out);

/* Query a batch of documents against the database: sign them with the model,
 * then for each query return the topk rows of highest MRC (score descending,
 * id ascending) and the number of rows with MRC >= tau.
 * topk_out: device mrc_hit [n_queries][topk] (rows beyond the database size
 * get id -1); n_hits: device int32 [n_queries]. precision as in mrc_compare:
 * BF16/FP8 candidates are rescored in FP32 so results equal the FP32 ones.
 * The database snapshot is its size at call time. topk in [1, 16]; the
 * database's k at most 512 (MRC_E_INVAL above, here and in mrc_serve_start). */
mrc_status mrc_query(mrc_ctx* ctx, const mrc_db* db, const mrc_model* model, const mrc_docs* q,
                     int32_t topk, float tau, int32_t precision, mrc_hit* topk_out,
                     int32_t* n_hits, void* hip_stream);

/* ------------------------------------------------------------------ serving */

#define MRC_REQ_QUERY 0
#define MRC_REQ_INSERT 1

typedef struct {
    int32_t max_batch;        /* max documents per device batch (1..4096) */
    int32_t n_streams;        /* device streams batches overlap on (1..4) */
    int32_t topk;             /* hits per query (<= 64) */
    float tau;
    int32_t precision;        /* MRC_PREC_* */
    int32_t max_queue;        /* pending requests beyond which submit returns MRC_E_BUSY */
    double hbm_frac;          /* admission cap as a fraction of the context budget */
    int64_t max_batch_tokens; /* token budget of one batch */
    int32_t max_wait_us;      /* how long a partial batch may wait for more arrivals */
} mrc_serve_opts;

typedef struct {
    int32_t status;           /* MRC_OK, or the error of the batch this request ran in */
    int32_t kind;             /* MRC_REQ_* */
    int64_t id;               /* INSERT: the database id assigned */
    int32_t n_hits;           /* QUERY: rows with MRC >= tau */
    int32_t n_top;            /* QUERY: entries filled in top[] */
    mrc_hit top[64];          /* QUERY: best rows, score descending, id ascending */
    double t_submit_ms, t_start_ms, t_done_ms; /* host clock, ms since server start */
} mrc_result;

/* Start a server over a database and model; it owns its streams and worker
 * thread. Requests are admitted while the memory they need fits the cap and
 * are batched continuously: batches form while earlier ones run on the GPU. */
mrc_status mrc_serve_start(mrc_ctx* ctx, mrc_db* db, const mrc_model* model,
                           const mrc_serve_opts* opts, mrc_server** out);
/* Submit one document (host int32 tokens, copied before return). */
mrc_status mrc_serve_submit(mrc_server* srv, const int32_t* tokens, int64_t len, int32_t kind,
                            uint64_t* ticket);
/* Submit n documents in one call (a front end that receives several at once):
 * host CSR arrays, document i being tokens[offsets[i], offsets[i + 1]), int64
 * offsets[n + 1], int32 tokens; all copied before return. They are queued in
 * order while the queue has room; *n_accepted (always written) says how many
 * went in, and tickets[0, *n_accepted) are theirs. Returns MRC_OK when all
 * were queued, MRC_E_BUSY when the queue filled first, MRC_E_INVAL (nothing
 * queued) for bad offsets or a token id outside [0, vocab). */
mrc_status mrc_serve_submit_many(mrc_server* srv, const int64_t* offsets, const int32_t* tokens, int64_t n,
                                 int32_t kind, uint64_t* tickets, int64_t* n_accepted);
/* Fetch a result: MRC_OK with the result when done, MRC_E_BUSY while pending,
 * MRC_E_INVAL for an unknown ticket. wait_ms > 0 blocks up to that long. */
mrc_status mrc_serve_poll(mrc_server* srv, uint64_t ticket, mrc_result* out, int32_t wait_ms);
/* Drain outstanding requests and stop; frees the database and model too if
 * they were destroyed while the server ran. */
mrc_status mrc_serve_stop(mrc_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MRC_H */
