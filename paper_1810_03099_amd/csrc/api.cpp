// C ABI entry points of libmrc: argument checks, object life cycle, stage
// sequencing on the caller's stream, and status reporting.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>

#include "common.h"

using namespace mrc;

namespace mrc {

mrc_status check_ctx(mrc_ctx* ctx, const char* fn) {
    if (!ctx) return fail(MRC_E_INVAL, std::string(fn) + ": ctx is NULL");
    if (ctx->sticky != MRC_OK)
        return fail(MRC_E_HIP, std::string(fn) + ": context unusable after an earlier HIP error");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice", __FILE__, __LINE__);
    // Drop an error another library left in the thread's last-error slot, so
    // that the launch checks below report only this call's launches.
    (void)hipGetLastError();
    return MRC_OK;
}

}  // namespace mrc

namespace {

mrc_status check_docs(const mrc_docs* d, const char* fn) {
    if (!d) return fail(MRC_E_INVAL, std::string(fn) + ": docs is NULL");
    if (d->n_docs < 0 || d->n_docs > 0x7FFFFFFFLL)
        return fail(MRC_E_INVAL, std::string(fn) + ": n_docs out of range");
    if (!d->offsets) return fail(MRC_E_INVAL, std::string(fn) + ": offsets is NULL");
    if (d->n_docs > 0 && !d->tokens && d->n_tokens > 0) return fail(MRC_E_INVAL, std::string(fn) + ": tokens is NULL");
    if (d->n_tokens < 0) return fail(MRC_E_INVAL, std::string(fn) + ": n_tokens < 0");
    return MRC_OK;
}

// Read the context flag words back after the stream drains; report input errors.
mrc_status sync_flags(mrc_ctx* ctx, hipStream_t s, int n_words, const char* fn) {
    MRC_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, n_words * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    const uint64_t err = (uint64_t)ctx->h_flags[0];
    if (err & kErrOffsets) return fail(MRC_E_INVAL, std::string(fn) + ": malformed offsets");
    if (err & kErrDocLen)
        return fail(MRC_E_INVAL, std::string(fn) + ": a document is longer than 2^22 tokens");
    if (err & kErrToken) return fail(MRC_E_INVAL, std::string(fn) + ": token id outside [0, vocab)");
    if (err & kErrSelection)
        return fail(MRC_E_INVAL, std::string(fn) + ": reference selection holds fewer terms than k");
    if (err & kErrTailCap)
        return fail(MRC_E_INVAL, std::string(fn) + ": a document has more than 16384 distinct terms past the dense head");
    return MRC_OK;
}

// The model's tables live in one device block (offsets 256-byte aligned), so
// a build costs one allocation and a destroy one free.
size_t model_layout(size_t V, size_t k, size_t off[7]) {
    const size_t sizes[7] = {V * 4, V * 4, V * 4, V * 4, V * sizeof(TermInfo), k * 8, k * 8};
    size_t total = 0;
    for (int i = 0; i < 7; ++i) {
        off[i] = total;
        total += (sizes[i] + 255) & ~size_t(255);
    }
    return total;
}

}  // namespace

namespace mrc {

// The context keeps the table block of one destroyed model for the next build
// of the same size, so that rebuilding a model costs no device allocation or
// free. The kept block still counts against the budget; the context frees it
// when a build of another size needs the room, and on destroy. Callers
// synchronise the device before handing a block back.
void free_model(mrc_model* m) {
    if (!m) return;
    mrc_ctx* c = m->ctx;
    void* old = nullptr;
    size_t old_bytes = 0;
    {
        std::lock_guard<std::mutex> g(c->mu);
        if (m->d_df) {
            old = c->model_spare;
            old_bytes = c->model_spare_bytes;
            c->model_spare = m->d_df;
            c->model_spare_bytes = m->bytes;
        }
    }
    dev_free(c, old, old_bytes);
    dev_free(c, m->d_hash, (size_t)m->vocab * 8);
    delete m;
    ctx_release(c);
}

}  // namespace mrc

namespace {

mrc_status alloc_model(mrc_ctx* ctx, int32_t V, int32_t k, mrc_model** out) {
    mrc_model* m = new mrc_model();
    m->ctx = ctx;
    m->vocab = V;
    m->k = k;
    size_t off[7];
    m->bytes = model_layout((size_t)V, (size_t)k, off);
    char* base = nullptr;
    void* spare = nullptr;
    size_t spare_bytes = 0;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        spare = ctx->model_spare;
        spare_bytes = ctx->model_spare_bytes;
        ctx->model_spare = nullptr;
        ctx->model_spare_bytes = 0;
    }
    mrc_status st = MRC_OK;
    if (spare && spare_bytes == m->bytes) {
        base = (char*)spare;
    } else {
        dev_free(ctx, spare, spare_bytes);
        st = dev_alloc(ctx, (void**)&base, m->bytes);
    }
    if (st != MRC_OK) {
        delete m;
        return st;
    }
    m->d_df = (uint32_t*)(base + off[0]);
    m->d_idf = (float*)(base + off[1]);
    m->d_term_at = (int32_t*)(base + off[2]);
    m->d_rank_of = (int32_t*)(base + off[3]);
    m->d_tinfo = (TermInfo*)(base + off[4]);
    m->d_rnorm = (double*)(base + off[5]);
    m->d_rinv = (double*)(base + off[6]);
    ctx_retain(ctx);
    *out = m;
    return MRC_OK;
}

mrc_status check_spec(const mrc_ref_spec* spec, int32_t V) {
    if (!spec) return fail(MRC_E_INVAL, "spec is NULL");
    if (spec->k < 1 || spec->k > 1024) return fail(MRC_E_INVAL, "k must lie in [1, 1024]");
    if (spec->mode < MRC_SEL_ALL || spec->mode > MRC_SEL_DROP_TOP) return fail(MRC_E_INVAL, "bad selection mode");
    if (spec->idf_mode != MRC_IDF_SMOOTH && spec->idf_mode != MRC_IDF_NONE) return fail(MRC_E_INVAL, "bad idf mode");
    if (spec->ref_weight != MRC_REF_ONE && spec->ref_weight != MRC_REF_IDF) return fail(MRC_E_INVAL, "bad reference weight");
    if (spec->mode == MRC_SEL_REGION && spec->lo < 0) return fail(MRC_E_INVAL, "region lo < 0");
    if (spec->mode == MRC_SEL_RAREST && spec->m < 1) return fail(MRC_E_INVAL, "rarest m < 1");
    if (spec->mode == MRC_SEL_DROP_TOP && (spec->drop_top_ppm < 0 || spec->drop_top_ppm > 1000000))
        return fail(MRC_E_INVAL, "drop_top_ppm outside [0, 1e6]");
    if (spec->k > V) return fail(MRC_E_INVAL, "k exceeds the vocabulary");
    return MRC_OK;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------ model

namespace {

// Model build shared by mrc_build_vocab_idf and mrc_build_and_sign; with
// sig_out set, the corpus is also signed from its count lists.
mrc_status build_model(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size, const mrc_ref_spec* spec,
                       mrc_model** out, float* sig_out, float* norm_out, hipStream_t s, const char* fn) {
    MRC_TRY(check_ctx(ctx, fn));
    MRC_TRY(check_docs(corpus, fn));
    if (!out) return fail(MRC_E_INVAL, std::string(fn) + ": out is NULL");
    *out = nullptr;
    if (vocab_size < 1 || vocab_size > (1 << 24)) return fail(MRC_E_INVAL, "vocab_size must lie in [1, 2^24]");
    MRC_TRY(check_spec(spec, vocab_size));
    mrc_model* m = nullptr;
    MRC_TRY(alloc_model(ctx, vocab_size, spec->k, &m));
    m->n_docs = corpus->n_docs;
    m->spec = *spec;
    auto bail = [&](mrc_status st) {
        (void)hipStreamSynchronize(s);
        free_model(m);
        return st;
    };
    CountLists cl{};
    mrc_status st = count_scratch(ctx, corpus, &cl);
    if (st == MRC_OK) st = launch_df(ctx, corpus, vocab_size, m->d_df, cl, s);
    if (st == MRC_OK) st = launch_model_tables(ctx, m, s);
    if (st == MRC_OK && sig_out) st = launch_sign_counts(ctx, m, corpus, cl, sig_out, norm_out, s);
    if (st == MRC_OK) st = sync_flags(ctx, s, 9, fn);
    if (st != MRC_OK) return bail(st);
    m->n_listed = ctx->h_flags[6];
    m->lo = ctx->h_flags[7];
    m->hi = ctx->h_flags[8];
    *out = m;
    return MRC_OK;
}

}  // namespace

static mrc_status build_vocab_idf_impl(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size,
                                       const mrc_ref_spec* spec, mrc_model** out, void* hip_stream) {
    return build_model(ctx, corpus, vocab_size, spec, out, nullptr, nullptr, (hipStream_t)hip_stream,
                       "mrc_build_vocab_idf");
}

static mrc_status build_and_sign_impl(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size,
                                      const mrc_ref_spec* spec, mrc_model** out, float* sig_out, float* norm_out,
                                      void* hip_stream) {
    if (corpus && corpus->n_docs > 0 && !sig_out) return fail(MRC_E_INVAL, "mrc_build_and_sign: sig_out is NULL");
    float* sig = sig_out;
    float dummy = 0.f;
    if (!sig) sig = &dummy;  // empty corpus: nothing is written
    return build_model(ctx, corpus, vocab_size, spec, out, sig, norm_out, (hipStream_t)hip_stream,
                       "mrc_build_and_sign");
}

mrc_status mrc_model_destroy(mrc_model* model) {
    if (!model) return MRC_OK;
    {
        std::lock_guard<std::mutex> g(model->ctx->mu);
        if (model->users > 0) {  // a server still uses it: the last one to stop frees it
            model->closing = true;
            return MRC_OK;
        }
    }
    (void)hipSetDevice(model->ctx->device);
    (void)hipDeviceSynchronize();
    free_model(model);
    return MRC_OK;
}

mrc_status mrc_model_info(const mrc_model* m, int64_t* n_docs, int32_t* vocab, int32_t* k,
                          int64_t* n_listed, int64_t* lo, int64_t* hi) {
    if (!m) return fail(MRC_E_INVAL, "mrc_model_info: model is NULL");
    if (n_docs) *n_docs = m->n_docs;
    if (vocab) *vocab = m->vocab;
    if (k) *k = m->k;
    if (n_listed) *n_listed = m->n_listed;
    if (lo) *lo = m->lo;
    if (hi) *hi = m->hi;
    return MRC_OK;
}

mrc_status mrc_model_get(const mrc_model* m, uint32_t* df, float* idf, int32_t* term_at, int32_t* rank_of,
                         int32_t* part_of, double* rnorm) {
    if (!m) return fail(MRC_E_INVAL, "mrc_model_get: model is NULL");
    mrc_ctx* ctx = m->ctx;
    MRC_TRY(check_ctx(ctx, "mrc_model_get"));
    const size_t V = (size_t)m->vocab;
    if (df) MRC_HIP_TRY(ctx, hipMemcpy(df, m->d_df, V * 4, hipMemcpyDeviceToHost));
    if (idf) MRC_HIP_TRY(ctx, hipMemcpy(idf, m->d_idf, V * 4, hipMemcpyDeviceToHost));
    if (term_at) MRC_HIP_TRY(ctx, hipMemcpy(term_at, m->d_term_at, V * 4, hipMemcpyDeviceToHost));
    if (rank_of) MRC_HIP_TRY(ctx, hipMemcpy(rank_of, m->d_rank_of, V * 4, hipMemcpyDeviceToHost));
    if (part_of) {
        std::vector<TermInfo> ti(V);
        MRC_HIP_TRY(ctx, hipMemcpy(ti.data(), m->d_tinfo, V * sizeof(TermInfo), hipMemcpyDeviceToHost));
        for (size_t t = 0; t < V; ++t) part_of[t] = ti[t].part;
    }
    if (rnorm) MRC_HIP_TRY(ctx, hipMemcpy(rnorm, m->d_rnorm, (size_t)m->k * 8, hipMemcpyDeviceToHost));
    return MRC_OK;
}

// File layout: magic "MRCMODEL", u32 version, header fields, then df[V],
// idf[V], term_at[V], rank_of[V], tinfo[V], rnorm[k], rinv[k], u64 FNV-1a
// checksum of everything before it.
mrc_status mrc_model_save(const mrc_model* m, const char* path) {
    if (!m || !path) return fail(MRC_E_INVAL, "mrc_model_save: NULL argument");
    mrc_ctx* ctx = m->ctx;
    MRC_TRY(check_ctx(ctx, "mrc_model_save"));
    const size_t V = (size_t)m->vocab, k = (size_t)m->k;
    std::vector<char> buf;
    auto put = [&](const void* p, size_t n) {
        const char* c = (const char*)p;
        buf.insert(buf.end(), c, c + n);
    };
    const char magic[8] = {'M', 'R', 'C', 'M', 'O', 'D', 'E', 'L'};
    const uint32_t version = 1;
    put(magic, 8);
    put(&version, 4);
    put(&m->n_docs, 8);
    put(&m->vocab, 4);
    put(&m->spec, sizeof(mrc_ref_spec));
    put(&m->k, 4);
    put(&m->n_listed, 8);
    put(&m->lo, 8);
    put(&m->hi, 8);
    std::vector<char> tmp(V * sizeof(TermInfo));
    struct Arr { const void* d; size_t n; } arrs[] = {
        {m->d_df, V * 4}, {m->d_idf, V * 4}, {m->d_term_at, V * 4}, {m->d_rank_of, V * 4},
        {m->d_tinfo, V * sizeof(TermInfo)}, {m->d_rnorm, k * 8}, {m->d_rinv, k * 8}};
    for (auto& a : arrs) {
        MRC_HIP_TRY(ctx, hipMemcpy(tmp.data(), a.d, a.n, hipMemcpyDeviceToHost));
        put(tmp.data(), a.n);
    }
    uint64_t h = fnv1a(buf.data(), buf.size());
    put(&h, 8);
    std::ofstream f(path, std::ios::binary);
    if (!f) return fail(MRC_E_INVAL, std::string("mrc_model_save: cannot open ") + path);
    f.write(buf.data(), (std::streamsize)buf.size());
    if (!f) return fail(MRC_E_INVAL, "mrc_model_save: write failed");
    return MRC_OK;
}

mrc_status mrc_model_load(mrc_ctx* ctx, const char* path, mrc_model** out) {
    MRC_TRY(check_ctx(ctx, "mrc_model_load"));
    if (!path || !out) return fail(MRC_E_INVAL, "mrc_model_load: NULL argument");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(MRC_E_INVAL, std::string("mrc_model_load: cannot open ") + path);
    std::vector<char> buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    size_t pos = 0;
    auto get = [&](void* p, size_t n) {
        if (pos + n > buf.size()) return false;
        memcpy(p, buf.data() + pos, n);
        pos += n;
        return true;
    };
    char magic[8];
    uint32_t version = 0;
    int64_t n_docs = 0, n_listed = 0, lo = 0, hi = 0;
    int32_t vocab = 0, k = 0;
    mrc_ref_spec spec{};
    if (!get(magic, 8) || memcmp(magic, "MRCMODEL", 8) != 0) return fail(MRC_E_INVAL, "mrc_model_load: not a model file");
    if (!get(&version, 4) || version != 1) return fail(MRC_E_INVAL, "mrc_model_load: unsupported version");
    bool ok = get(&n_docs, 8) && get(&vocab, 4) && get(&spec, sizeof spec) && get(&k, 4) && get(&n_listed, 8) &&
              get(&lo, 8) && get(&hi, 8);
    if (!ok || vocab < 1 || vocab > (1 << 24) || k < 1 || k > 1024 || spec.k != k)
        return fail(MRC_E_INVAL, "mrc_model_load: corrupt header");
    const size_t V = (size_t)vocab;
    const size_t body = V * 16 + V * sizeof(TermInfo) + (size_t)k * 16;
    if (buf.size() != pos + body + 8) return fail(MRC_E_INVAL, "mrc_model_load: truncated file");
    uint64_t h_stored = 0;
    memcpy(&h_stored, buf.data() + pos + body, 8);
    if (fnv1a(buf.data(), pos + body) != h_stored) return fail(MRC_E_INVAL, "mrc_model_load: checksum mismatch");
    mrc_model* m = nullptr;
    MRC_TRY(alloc_model(ctx, vocab, k, &m));
    m->n_docs = n_docs;
    m->spec = spec;
    m->n_listed = n_listed;
    m->lo = lo;
    m->hi = hi;
    struct Arr { void* d; size_t n; } arrs[] = {
        {m->d_df, V * 4}, {m->d_idf, V * 4}, {m->d_term_at, V * 4}, {m->d_rank_of, V * 4},
        {m->d_tinfo, V * sizeof(TermInfo)}, {m->d_rnorm, (size_t)k * 8}, {m->d_rinv, (size_t)k * 8}};
    for (auto& a : arrs) {
        hipError_t e = hipMemcpy(a.d, buf.data() + pos, a.n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_model(m);
            return hip_fail(ctx, e, "model upload", __FILE__, __LINE__);
        }
        pos += a.n;
    }
    *out = m;
    return MRC_OK;
}

// ------------------------------------------------------------------ signing

static mrc_status sign_impl(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, float* sig_out,
                            float* norm_out, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_sign"));
    MRC_TRY(check_docs(docs, "mrc_sign"));
    if (!model) return fail(MRC_E_INVAL, "mrc_sign: model is NULL");
    if (model->ctx->device != ctx->device) return fail(MRC_E_INVAL, "mrc_sign: model lives on another device");
    if (docs->n_docs > 0 && !sig_out) return fail(MRC_E_INVAL, "mrc_sign: sig_out is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(launch_sign(ctx, model, docs, sig_out, norm_out, s));
    return sync_flags(ctx, s, 1, "mrc_sign");
}

static mrc_status sign_matrix_impl(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, const float* R,
                                   int32_t k, float* sig_out, float* norm_out, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_sign_matrix"));
    MRC_TRY(check_docs(docs, "mrc_sign_matrix"));
    if (!model) return fail(MRC_E_INVAL, "mrc_sign_matrix: model is NULL");
    if (model->ctx->device != ctx->device) return fail(MRC_E_INVAL, "mrc_sign_matrix: model lives on another device");
    if (k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_sign_matrix: k must lie in [1, 1024]");
    if (!R) return fail(MRC_E_INVAL, "mrc_sign_matrix: R is NULL");
    if (docs->n_docs > 0 && !sig_out) return fail(MRC_E_INVAL, "mrc_sign_matrix: sig_out is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(launch_sign_matrix(ctx, model, docs, R, k, sig_out, norm_out, s));
    return sync_flags(ctx, s, 1, "mrc_sign_matrix");
}

// ------------------------------------------------------------------ comparison

mrc_status mrc_normalise(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float* unit_out,
                         uint16_t* bf16_out, uint8_t* fp8_out, float* scale_out, float* err_out,
                         void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_normalise"));
    if (n < 0 || k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_normalise: bad n or k");
    if (n > 0 && !sig) return fail(MRC_E_INVAL, "mrc_normalise: sig is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(launch_normalise(ctx, sig, n, k, unit_out, bf16_out, fp8_out, scale_out, err_out, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    return MRC_OK;
}

mrc_status mrc_score_pairs(mrc_ctx* ctx, const float* unit, int64_t n, int32_t k, const int32_t* ii,
                           const int32_t* jj, int64_t n_pairs, float* out, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_score_pairs"));
    if (n < 0 || k < 1 || n_pairs < 0) return fail(MRC_E_INVAL, "mrc_score_pairs: bad sizes");
    if (n_pairs > 0 && (!unit || !ii || !jj || !out)) return fail(MRC_E_INVAL, "mrc_score_pairs: NULL buffer");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(launch_score_pairs(ctx, unit, k, ii, jj, n_pairs, out, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    return MRC_OK;
}

static mrc_status compare_impl(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, const mrc_compare_opts* opts,
                               mrc_pair* pairs_out, int64_t capacity, int64_t* n_found, mrc_compare_stats* stats,
                               void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_compare"));
    if (!opts || !n_found) return fail(MRC_E_INVAL, "mrc_compare: NULL opts or n_found");
    if (n < 0 || n > 0x7FFFFFFFLL || k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_compare: bad n or k");
    if (n > 0 && !sig) return fail(MRC_E_INVAL, "mrc_compare: sig is NULL");
    if (capacity < 0 || (capacity > 0 && !pairs_out)) return fail(MRC_E_INVAL, "mrc_compare: bad output buffer");
    if (!(opts->tau == opts->tau) || opts->reserved != 0) return fail(MRC_E_INVAL, "mrc_compare: bad options");
    if (opts->precision < MRC_PREC_FP32 || opts->precision > MRC_PREC_FP8)
        return fail(MRC_E_INVAL, "mrc_compare: bad precision");
    if (opts->precision != MRC_PREC_FP32 && !(opts->band >= 0.f))
        return fail(MRC_E_INVAL, "mrc_compare: band must be >= 0");
    hipStream_t s = (hipStream_t)hip_stream;
    *n_found = 0;
    mrc_compare_stats st{};
    st.n_pairs_compared = n * (n - 1) / 2;
    unsigned long long* counter = (unsigned long long*)(ctx->d_flags + 4);
    if (opts->precision == MRC_PREC_FP32) {
        const int64_t n_pad = ceil_div(n > 0 ? n : 1, 128) * 128, kp = 16 * (int64_t)mfma_chunks(k);  // 128-row tiles
        void* umfma = nullptr;
        MRC_TRY(scratch(ctx, "cmp_unit_mfma", (size_t)(n_pad * kp) * sizeof(float), &umfma));
        // (the normalising launch also zeroes the flag words the comparison counts into)
        MRC_TRY(launch_normalise(ctx, sig, n, k, nullptr, nullptr, nullptr, nullptr, nullptr, s, (float*)umfma,
                                 ctx->d_flags, 16));
        PairSink sink{pairs_out, capacity, counter};
        MRC_TRY(launch_compare_f32(ctx, (const float*)umfma, n, k, opts->tau, sink, s));
        MRC_TRY(sync_flags(ctx, s, 16, "mrc_compare"));
        const int64_t found = ctx->h_flags[4];
        *n_found = found;
        st.n_flagged = found;
        if (stats) *stats = st;
        if (found > capacity) return fail(MRC_E_OVERFLOW, "mrc_compare: more pairs than capacity");
        return MRC_OK;
    }
    // BF16 / FP8: candidates on the matrix cores, then exact decisions by rescoring.
    const int prec = opts->precision;
    const int ebytes = prec == MRC_PREC_BF16 ? 2 : 1;
    const int chunks = lowp_lds_chunks(prec, k);
    if (chunks < 0) return fail(MRC_E_INVAL, "mrc_compare: k too large for the low-precision form");
    const int ldq = chunks * 128 / ebytes;  // components per row (whole 128-byte chunks)
    const int64_t n_pad = ceil_div(n > 0 ? n : 1, 256) * 256;  // 256-row blocks
    void *unit = nullptr, *q = nullptr, *scale = nullptr, *err = nullptr;
    MRC_TRY(scratch(ctx, "lp_unit", (size_t)(n > 0 ? n : 1) * k * sizeof(float), &unit));
    MRC_TRY(scratch(ctx, "lp_codes", (size_t)n_pad * ldq * ebytes, &q));
    MRC_TRY(scratch(ctx, "lp_scale", (size_t)n_pad * sizeof(float), &scale));
    MRC_TRY(scratch(ctx, "lp_err", (size_t)2 * n_pad * sizeof(float), &err));
    int64_t cand_cap = std::max<int64_t>(1 << 20, 16 * n);
    auto it = ctx->scratch.find("lp_cand");
    if (it != ctx->scratch.end()) cand_cap = std::max<int64_t>(cand_cap, (int64_t)(it->second.second / sizeof(mrc_pair)));
    for (int attempt = 0; attempt < 2; ++attempt) {
        void* cand = nullptr;
        MRC_TRY(scratch(ctx, "lp_cand", (size_t)cand_cap * sizeof(mrc_pair), &cand));
        NormLayout o{(float*)unit, k, prec == MRC_PREC_BF16 ? (uint16_t*)q : nullptr, ldq,
                     prec == MRC_PREC_FP8 ? (uint8_t*)q : nullptr, ldq, (float*)scale, (float*)err, n_pad,
                     nullptr, 0, n_pad, 0, prec == MRC_PREC_BF16 ? 1 : 2};
        o.clear = ctx->d_flags;  // (zeroed by the normalising launch: the candidate and pair counters)
        o.n_clear = 32;
        MRC_TRY(launch_normalise_rows(ctx, sig, n, k, o, s));
        const float* err_p = (const float*)err + (prec == MRC_PREC_BF16 ? 0 : n_pad);
        float* d_lo = (float*)(ctx->d_flags + 22);
        if (n >= 2) {
            // (word 23: zeroed with the others above, the largest row error)
            MRC_TRY(launch_lowp_threshold(ctx, prec, err_p, n, opts->tau, opts->band, k,
                                          (unsigned int*)(ctx->d_flags + 23), d_lo, s));
            PairSink cs{(mrc_pair*)cand, cand_cap, (unsigned long long*)(ctx->d_flags + 16)};
            MRC_TRY(launch_compare_lowp(ctx, prec, (const uint8_t*)q, ldq * ebytes, (const float*)scale, n, k, d_lo,
                                        err_p, opts->tau, opts->band, cs, s));
            PairSink out{pairs_out, capacity, counter};
            MRC_TRY(launch_rescore2(ctx, prec, (const mrc_pair*)cand, (const unsigned long long*)(ctx->d_flags + 16),
                                    cand_cap, (const float*)unit, k, err_p, opts->tau, opts->band, out,
                                    (unsigned long long*)(ctx->d_flags + 17), s));
        }
        MRC_TRY(sync_flags(ctx, s, 32, "mrc_compare"));
        const int64_t n_cand = ctx->h_flags[16];
        ctx->lowp_candidates = n_cand;
        if (n_cand > cand_cap && attempt == 0) {
            cand_cap = n_cand + n_cand / 4;
            continue;
        }
        if (n_cand > cand_cap) return fail(MRC_E_NOMEM, "mrc_compare: candidate list overflow");
        const int64_t found = ctx->h_flags[4];
        *n_found = found;
        st.n_flagged = found;
        st.n_band = ctx->h_flags[17];
        st.n_band_nominal = ctx->h_flags[18];
        st.n_flip_outside_nominal = ctx->h_flags[19];
        uint32_t mx = (uint32_t)ctx->h_flags[20];
        memcpy(&st.max_abs_err, &mx, 4);
        double sum = 0.0;
        memcpy(&sum, &ctx->h_flags[21], 8);
        st.mean_abs_err = st.n_band ? (float)(sum / (double)st.n_band) : 0.f;
        if (stats) *stats = st;
        if (found > capacity) return fail(MRC_E_OVERFLOW, "mrc_compare: more pairs than capacity");
        return MRC_OK;
    }
    return fail(MRC_E_STATE, "mrc_compare: unreachable");
}

// ------------------------------------------------------------------ comparators

static mrc_status ensure_hashes(mrc_ctx* ctx, const mrc_model* model, hipStream_t s) {
    mrc_model* m = const_cast<mrc_model*>(model);
    if (m->d_hash) return MRC_OK;
    MRC_TRY(dev_alloc(ctx, (void**)&m->d_hash, (size_t)m->vocab * 8));
    return launch_term_hashes(ctx, m->vocab, m->d_hash, s);
}

mrc_status mrc_term_hashes(mrc_ctx* ctx, const mrc_model* model, uint64_t* out, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_term_hashes"));
    if (!model || !out) return fail(MRC_E_INVAL, "mrc_term_hashes: NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(ensure_hashes(ctx, model, s));
    MRC_HIP_TRY(ctx, hipMemcpyAsync(out, model->d_hash, (size_t)model->vocab * 8, hipMemcpyDeviceToDevice, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    return MRC_OK;
}

mrc_status mrc_trigrams(mrc_ctx* ctx, const uint8_t* text, const int64_t* text_offsets, int64_t n_docs,
                        int64_t n_bytes, int64_t* tok_offsets_out, int32_t* tokens_out, int64_t capacity,
                        int64_t* n_tokens, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_trigrams"));
    if (!n_tokens || n_docs < 0 || n_bytes < 0 || capacity < 0 || (capacity > 0 && !tokens_out) ||
        !text_offsets || !tok_offsets_out || (n_bytes > 0 && !text) || (n_docs == 0 && n_bytes != 0))
        return fail(MRC_E_INVAL, "mrc_trigrams: bad argument");
    hipStream_t s = (hipStream_t)hip_stream;
    *n_tokens = 0;
    if (n_docs == 0) {
        MRC_TRY(clear_words(ctx, tok_offsets_out, 1, s));
        return MRC_OK;
    }
    MRC_TRY(launch_trigram_offsets(ctx, text_offsets, n_docs, n_bytes, tok_offsets_out, s));
    MRC_TRY(sync_flags(ctx, s, 2, "mrc_trigrams"));
    *n_tokens = ctx->h_flags[1];
    if (*n_tokens > capacity) return fail(MRC_E_OVERFLOW, "mrc_trigrams: more ids than capacity");
    return launch_trigrams(ctx, text, n_bytes, text_offsets, n_docs, tok_offsets_out, tokens_out, s);
}

mrc_status mrc_simhash(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, uint64_t* out, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_simhash"));
    MRC_TRY(check_docs(docs, "mrc_simhash"));
    if (!model || (docs->n_docs > 0 && !out)) return fail(MRC_E_INVAL, "mrc_simhash: NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(ensure_hashes(ctx, model, s));
    MRC_TRY(launch_simhash(ctx, docs, model->vocab, model->d_hash, out, s));
    return sync_flags(ctx, s, 1, "mrc_simhash");
}

mrc_status mrc_hamming_pairs(mrc_ctx* ctx, const uint64_t* sim, int64_t n, int32_t max_dist, mrc_pair* pairs_out,
                             int64_t capacity, int64_t* n_found, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_hamming_pairs"));
    if (!n_found || n < 0 || n > 0x7FFFFFFFLL || (n > 0 && !sim) || max_dist < 0 || capacity < 0 ||
        (capacity > 0 && !pairs_out))
        return fail(MRC_E_INVAL, "mrc_hamming_pairs: bad argument");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(clear_words(ctx, ctx->d_flags, 8, s));
    PairSink sink{pairs_out, capacity, (unsigned long long*)(ctx->d_flags + 4)};
    MRC_TRY(launch_hamming(ctx, sim, n, max_dist, sink, s));
    MRC_TRY(sync_flags(ctx, s, 8, "mrc_hamming_pairs"));
    *n_found = ctx->h_flags[4];
    if (*n_found > capacity) return fail(MRC_E_OVERFLOW, "mrc_hamming_pairs: more pairs than capacity");
    return MRC_OK;
}

mrc_status mrc_exact_cosine(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, float tau, mrc_pair* pairs_out,
                            int64_t capacity, int64_t* n_found, void* hip_stream) {
    MRC_TRY(check_ctx(ctx, "mrc_exact_cosine"));
    MRC_TRY(check_docs(docs, "mrc_exact_cosine"));
    if (!model || !n_found || capacity < 0 || (capacity > 0 && !pairs_out) || !(tau == tau))
        return fail(MRC_E_INVAL, "mrc_exact_cosine: bad argument");
    hipStream_t s = (hipStream_t)hip_stream;
    MRC_TRY(clear_words(ctx, ctx->d_flags, 8, s));
    PairSink sink{pairs_out, capacity, (unsigned long long*)(ctx->d_flags + 4)};
    MRC_TRY(launch_exact_cosine(ctx, model, docs, tau, sink, s));
    MRC_TRY(sync_flags(ctx, s, 8, "mrc_exact_cosine"));
    *n_found = ctx->h_flags[4];
    if (*n_found > capacity) return fail(MRC_E_OVERFLOW, "mrc_exact_cosine: more pairs than capacity");
    return MRC_OK;
}

// ------------------------------------------------------------------ logged entry points
// (each records one line when MRC_LOG >= 1; the work is in the *_impl above)

static void log_docs(CallLog& L, const mrc_docs* d) {
    L.add("n_docs", d ? d->n_docs : (int64_t)-1);
    L.add("tokens", d ? d->n_tokens : (int64_t)-1);
}

mrc_status mrc_build_vocab_idf(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size,
                               const mrc_ref_spec* spec, mrc_model** out, void* hip_stream) {
    CallLog L(ctx, "mrc_build_vocab_idf");
    log_docs(L, corpus);
    L.add("vocab", (int64_t)vocab_size);
    L.add("k", (int64_t)(spec ? spec->k : -1));
    const mrc_status st = build_vocab_idf_impl(ctx, corpus, vocab_size, spec, out, hip_stream);
    if (st == MRC_OK && out && *out) L.add("n_listed", (*out)->n_listed);
    return L.done(st);
}

mrc_status mrc_build_and_sign(mrc_ctx* ctx, const mrc_docs* corpus, int32_t vocab_size, const mrc_ref_spec* spec,
                              mrc_model** out, float* sig_out, float* norm_out, void* hip_stream) {
    CallLog L(ctx, "mrc_build_and_sign");
    log_docs(L, corpus);
    L.add("vocab", (int64_t)vocab_size);
    L.add("k", (int64_t)(spec ? spec->k : -1));
    const mrc_status st = build_and_sign_impl(ctx, corpus, vocab_size, spec, out, sig_out, norm_out, hip_stream);
    if (st == MRC_OK && out && *out) L.add("n_listed", (*out)->n_listed);
    return L.done(st);
}

mrc_status mrc_sign(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, float* sig_out,
                    float* norm_out, void* hip_stream) {
    CallLog L(ctx, "mrc_sign");
    log_docs(L, docs);
    L.add("k", (int64_t)(model ? model->k : -1));
    return L.done(sign_impl(ctx, model, docs, sig_out, norm_out, hip_stream));
}

mrc_status mrc_sign_matrix(mrc_ctx* ctx, const mrc_model* model, const mrc_docs* docs, const float* R, int32_t k,
                           float* sig_out, float* norm_out, void* hip_stream) {
    CallLog L(ctx, "mrc_sign_matrix");
    log_docs(L, docs);
    L.add("k", (int64_t)k);
    return L.done(sign_matrix_impl(ctx, model, docs, R, k, sig_out, norm_out, hip_stream));
}

mrc_status mrc_compare(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, const mrc_compare_opts* opts,
                       mrc_pair* pairs_out, int64_t capacity, int64_t* n_found, mrc_compare_stats* stats,
                       void* hip_stream) {
    CallLog L(ctx, "mrc_compare");
    L.add("n", n);
    L.add("k", (int64_t)k);
    L.add("precision", (int64_t)(opts ? opts->precision : -1));
    L.add("tau", (double)(opts ? opts->tau : 0.f));
    mrc_compare_stats local{};
    const mrc_status st =
        compare_impl(ctx, sig, n, k, opts, pairs_out, capacity, n_found, stats ? stats : &local, hip_stream);
    const mrc_compare_stats& cs = stats ? *stats : local;
    if (st == MRC_OK || st == MRC_E_OVERFLOW) {
        L.add("flagged", cs.n_flagged);
        L.add("band_pairs", cs.n_band);
        L.add("band_pairs_nominal", cs.n_band_nominal);
        L.add("flips_outside_nominal", cs.n_flip_outside_nominal);
        L.add("max_abs_err", (double)cs.max_abs_err);
        if (opts && opts->precision != MRC_PREC_FP32) L.add("candidates", ctx->lowp_candidates);
    }
    return L.done(st);
}

}  // extern "C"
