// Resident signature database: unit signatures in the FP32 matrix-core layout
// plus optional BF16 / FP8 copies, append-only ids, save / load, and the
// batched query entry point.
#include <algorithm>
#include <cstdio>
#include <fstream>

#include "common.h"

using namespace mrc;

namespace {

mrc_status ctx_ready(mrc_ctx* ctx, const char* fn) {
    if (!ctx) return fail(MRC_E_INVAL, std::string(fn) + ": ctx is NULL");
    if (ctx->sticky != MRC_OK) return fail(MRC_E_HIP, std::string(fn) + ": context unusable after an earlier HIP error");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice", __FILE__, __LINE__);
    (void)hipGetLastError();
    return MRC_OK;
}

}  // namespace

namespace mrc {

void free_db(mrc_db* db) {
    if (!db) return;
    mrc_ctx* c = db->ctx;
    const DbLayout L = db_layout(db->k);
    dev_free(c, db->d_unit, (size_t)db->cap_pad * L.kp * 4);
    dev_free(c, db->d_bf16, (size_t)db->cap_pad * L.ldb * 2);
    dev_free(c, db->d_fp8, (size_t)db->cap_pad * L.ld8);
    dev_free(c, db->d_scale, (size_t)db->cap_pad * 4);
    dev_free(c, db->d_err, (size_t)db->cap_pad * 8);
    dev_free(c, db->d_errmax, 8);
    delete db;
    ctx_release(c);
}

}  // namespace mrc

namespace {

mrc_status alloc_db(mrc_ctx* ctx, int64_t capacity, int32_t k, uint32_t precisions, mrc_db** out) {
    if (capacity < 1 || k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_db_create: bad capacity or k");
    if (capacity > 0x7FFFFFFFLL - 64) return fail(MRC_E_INVAL, "mrc_db_create: capacity above 2^31 rows");
    mrc_db* db = new mrc_db();
    db->ctx = ctx;
    ctx_retain(ctx);
    db->capacity = capacity;
    db->cap_pad = ceil_div(capacity, 64) * 64;
    db->k = k;
    db->precisions = precisions;
    const DbLayout L = db_layout(k);
    mrc_status st = dev_alloc(ctx, (void**)&db->d_unit, (size_t)db->cap_pad * L.kp * 4);
    if (st == MRC_OK && (precisions & (1u << MRC_PREC_BF16)))
        st = dev_alloc(ctx, (void**)&db->d_bf16, (size_t)db->cap_pad * L.ldb * 2);
    if (st == MRC_OK && (precisions & (1u << MRC_PREC_FP8)))
        st = dev_alloc(ctx, (void**)&db->d_fp8, (size_t)db->cap_pad * L.ld8);
    if (st == MRC_OK) st = dev_alloc(ctx, (void**)&db->d_scale, (size_t)db->cap_pad * 4);
    if (st == MRC_OK) st = dev_alloc(ctx, (void**)&db->d_err, (size_t)db->cap_pad * 8);
    if (st == MRC_OK) st = dev_alloc(ctx, (void**)&db->d_errmax, 8);
    if (st != MRC_OK) {
        free_db(db);
        return st;
    }
    hipError_t e = hipMemset(db->d_unit, 0, (size_t)db->cap_pad * L.kp * 4);
    if (e == hipSuccess && db->d_bf16) e = hipMemset(db->d_bf16, 0, (size_t)db->cap_pad * L.ldb * 2);
    if (e == hipSuccess && db->d_fp8) e = hipMemset(db->d_fp8, 0, (size_t)db->cap_pad * L.ld8);
    if (e == hipSuccess) e = hipMemset(db->d_scale, 0, (size_t)db->cap_pad * 4);
    if (e == hipSuccess) e = hipMemset(db->d_err, 0, (size_t)db->cap_pad * 8);
    if (e == hipSuccess) e = hipMemset(db->d_errmax, 0, 8);
    if (e != hipSuccess) {
        free_db(db);
        return hip_fail(ctx, e, "database clear", __FILE__, __LINE__);
    }
    *out = db;
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

namespace mrc {

// Normalise n signatures into rows [first, first + n) of the database.
mrc_status db_append(mrc_db* db, const float* sig, int64_t n, int64_t first, hipStream_t s) {
    const DbLayout L = db_layout(db->k);
    NormLayout o{nullptr, 0, db->d_bf16 ? db->d_bf16 + first * L.ldb : nullptr, L.ldb,
                 db->d_fp8 ? db->d_fp8 + first * L.ld8 : nullptr, L.ld8, db->d_scale + first,
                 db->d_err + first, db->cap_pad, db->d_unit + first * L.kp, L.kp, n};
    MRC_TRY(launch_normalise_rows(db->ctx, sig, n, db->k, o, s));
    // the queries' rescoring band uses the largest row error, kept up to date here
    // (before the rows are committed) so that a query never scans the database for it
    return launch_err_max(db->ctx, db->d_err + first, db->d_err + db->cap_pad + first, n, db->d_errmax, s);
}

}  // namespace mrc

extern "C" {

mrc_status mrc_db_create(mrc_ctx* ctx, int64_t capacity, int32_t k, uint32_t precisions, mrc_db** out) {
    MRC_TRY(ctx_ready(ctx, "mrc_db_create"));
    if (!out) return fail(MRC_E_INVAL, "mrc_db_create: out is NULL");
    *out = nullptr;
    return alloc_db(ctx, capacity, k, precisions, out);
}

mrc_status mrc_db_destroy(mrc_db* db) {
    if (!db) return MRC_OK;
    {
        std::lock_guard<std::mutex> g(db->ctx->mu);
        if (db->users > 0) {  // a server still uses it: the last one to stop frees it
            db->closing = true;
            return MRC_OK;
        }
    }
    (void)hipSetDevice(db->ctx->device);
    (void)hipDeviceSynchronize();
    free_db(db);
    return MRC_OK;
}

mrc_status mrc_db_size(const mrc_db* db, int64_t* n, int32_t* k) {
    if (!db) return fail(MRC_E_INVAL, "mrc_db_size: db is NULL");
    if (n) *n = __atomic_load_n(&db->size, __ATOMIC_ACQUIRE);
    if (k) *k = db->k;
    return MRC_OK;
}

static mrc_status db_insert_impl(mrc_db* db, const float* sig, int64_t n, int64_t* first_id, void* hip_stream) {
    if (!db) return fail(MRC_E_INVAL, "mrc_db_insert: db is NULL");
    MRC_TRY(ctx_ready(db->ctx, "mrc_db_insert"));
    if (n < 0 || (n > 0 && !sig)) return fail(MRC_E_INVAL, "mrc_db_insert: bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> g(db->mu);
    if (db->size + n > db->capacity) return fail(MRC_E_OVERFLOW, "mrc_db_insert: database capacity exceeded");
    const int64_t first = db->size;
    MRC_TRY(db_append(db, sig, n, first, s));
    mrc_ctx* ctx = db->ctx;
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    __atomic_store_n(&db->size, first + n, __ATOMIC_RELEASE);
    if (first_id) *first_id = first;
    return MRC_OK;
}

mrc_status mrc_db_insert_docs(mrc_db* db, const mrc_model* model, const mrc_docs* docs, int64_t* first_id,
                              void* hip_stream) {
    if (!db || !model || !docs) return fail(MRC_E_INVAL, "mrc_db_insert_docs: NULL argument");
    mrc_ctx* ctx = db->ctx;
    MRC_TRY(ctx_ready(ctx, "mrc_db_insert_docs"));
    if (model->k != db->k) return fail(MRC_E_INVAL, "mrc_db_insert_docs: model and database differ in k");
    if (docs->n_docs < 0 || !docs->offsets) return fail(MRC_E_INVAL, "mrc_db_insert_docs: bad docs");
    hipStream_t s = (hipStream_t)hip_stream;
    void* sig = nullptr;
    MRC_TRY(scratch(ctx, "ins_sig", (size_t)std::max<int64_t>(1, docs->n_docs) * db->k * 4, &sig));
    MRC_TRY(launch_sign(ctx, model, docs, (float*)sig, nullptr, s));
    MRC_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, 8, hipMemcpyDeviceToHost, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->h_flags[0])
        return fail(MRC_E_INVAL, "mrc_db_insert_docs: malformed offsets, token ids or document lengths");
    return mrc_db_insert(db, (const float*)sig, docs->n_docs, first_id, hip_stream);
}

// File: magic "MRCDBASE", u32 version, i64 size, i32 k, then the FP32 rows
// [size][kp] in the matrix-core layout, u64 FNV-1a checksum. Low-precision
// copies are rebuilt from the rows on load.
mrc_status mrc_db_save(const mrc_db* db, const char* path) {
    if (!db || !path) return fail(MRC_E_INVAL, "mrc_db_save: NULL argument");
    mrc_ctx* ctx = db->ctx;
    MRC_TRY(ctx_ready(ctx, "mrc_db_save"));
    const DbLayout L = db_layout(db->k);
    const int64_t n = db->size;
    std::vector<char> buf(8 + 4 + 8 + 4 + (size_t)n * L.kp * 4);
    size_t pos = 0;
    auto put = [&](const void* p, size_t m) {
        memcpy(buf.data() + pos, p, m);
        pos += m;
    };
    const uint32_t version = 1;
    put("MRCDBASE", 8);
    put(&version, 4);
    put(&n, 8);
    put(&db->k, 4);
    if (n > 0) MRC_HIP_TRY(ctx, hipMemcpy(buf.data() + pos, db->d_unit, (size_t)n * L.kp * 4, hipMemcpyDeviceToHost));
    pos += (size_t)n * L.kp * 4;
    const uint64_t h = fnv1a(buf.data(), pos);
    std::ofstream f(path, std::ios::binary);
    if (!f) return fail(MRC_E_INVAL, std::string("mrc_db_save: cannot open ") + path);
    f.write(buf.data(), (std::streamsize)pos);
    f.write((const char*)&h, 8);
    if (!f) return fail(MRC_E_INVAL, "mrc_db_save: write failed");
    return MRC_OK;
}

// Undo the matrix-core layout of FP32 rows (component c sits at mfma_col(c)).
static void unpermute_rows(const std::vector<float>& src, int64_t n, int k, int kp, std::vector<float>& dst) {
    dst.assign((size_t)n * k, 0.f);
    for (int64_t r = 0; r < n; ++r)
        for (int c = 0; c < k; ++c) dst[(size_t)r * k + c] = src[(size_t)r * kp + mrc_dev::mfma_col(c)];
}

mrc_status mrc_db_load(mrc_ctx* ctx, const char* path, uint32_t precisions, mrc_db** out) {
    MRC_TRY(ctx_ready(ctx, "mrc_db_load"));
    if (!path || !out) return fail(MRC_E_INVAL, "mrc_db_load: NULL argument");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(MRC_E_INVAL, std::string("mrc_db_load: cannot open ") + path);
    std::vector<char> buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (buf.size() < 32 || memcmp(buf.data(), "MRCDBASE", 8) != 0) return fail(MRC_E_INVAL, "mrc_db_load: not a database file");
    uint32_t version = 0;
    int64_t n = 0;
    int32_t k = 0;
    memcpy(&version, buf.data() + 8, 4);
    memcpy(&n, buf.data() + 12, 8);
    memcpy(&k, buf.data() + 20, 4);
    if (version != 1 || n < 0 || k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_db_load: corrupt header");
    const DbLayout L = db_layout(k);
    const size_t body = (size_t)n * L.kp * 4;
    if (buf.size() != 24 + body + 8) return fail(MRC_E_INVAL, "mrc_db_load: truncated file");
    uint64_t h = 0;
    memcpy(&h, buf.data() + 24 + body, 8);
    if (fnv1a(buf.data(), 24 + body) != h) return fail(MRC_E_INVAL, "mrc_db_load: checksum mismatch");
    mrc_db* db = nullptr;
    MRC_TRY(alloc_db(ctx, std::max<int64_t>(n, 1), k, precisions, &db));
    if (n > 0) {
        // FP32 rows go back verbatim; the unit rows in natural order feed the
        // quantisers (u / |u| of a unit row can move its last bit, so the FP32
        // copy is restored after).
        std::vector<float> rows((size_t)n * L.kp), nat;
        memcpy(rows.data(), buf.data() + 24, body);
        unpermute_rows(rows, n, k, L.kp, nat);
        void* d = nullptr;
        mrc_status st = scratch(ctx, "db_load", (size_t)n * k * 4, &d);
        hipError_t e = hipSuccess;
        if (st == MRC_OK) e = hipMemcpy(d, nat.data(), (size_t)n * k * 4, hipMemcpyHostToDevice);
        if (st == MRC_OK && e == hipSuccess) st = db_append(db, (const float*)d, n, 0, nullptr);
        if (st == MRC_OK && e == hipSuccess) e = hipDeviceSynchronize();
        if (st == MRC_OK && e == hipSuccess) e = hipMemcpy(db->d_unit, rows.data(), body, hipMemcpyHostToDevice);
        if (st != MRC_OK || e != hipSuccess) {
            free_db(db);
            return st != MRC_OK ? st : hip_fail(ctx, e, "database upload", __FILE__, __LINE__);
        }
    }
    db->size = n;
    *out = db;
    return MRC_OK;
}

static mrc_status query_impl(mrc_ctx* ctx, const mrc_db* db, const mrc_model* model, const mrc_docs* q, int32_t topk,
                             float tau, int32_t precision, mrc_hit* topk_out, int32_t* n_hits, void* hip_stream) {
    MRC_TRY(ctx_ready(ctx, "mrc_query"));
    if (!db || !model || !q || !q->offsets) return fail(MRC_E_INVAL, "mrc_query: NULL argument");
    if (model->k != db->k) return fail(MRC_E_INVAL, "mrc_query: model and database differ in k");
    if (topk < 1 || topk > 16) return fail(MRC_E_INVAL, "mrc_query: topk must lie in [1, 16]");
    if (db->k > kQueryMaxK) return fail(MRC_E_INVAL, "mrc_query: queries support k <= 512");
    if (precision < MRC_PREC_FP32 || precision > MRC_PREC_FP8) return fail(MRC_E_INVAL, "mrc_query: bad precision");
    if (q->n_docs < 0 || q->n_docs > (1 << 20)) return fail(MRC_E_INVAL, "mrc_query: n_docs outside [0, 2^20]");
    if (q->n_docs > 0 && (!topk_out || !n_hits)) return fail(MRC_E_INVAL, "mrc_query: NULL output");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t rows = __atomic_load_n(&db->size, __ATOMIC_ACQUIRE);
    MRC_TRY(run_query(ctx, db, rows, model, q, topk, tau, precision, topk_out, n_hits, s));
    MRC_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_flags, ctx->d_flags, 8, hipMemcpyDeviceToHost, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->h_flags[0] & (kErrOffsets | kErrToken | kErrDocLen))
        return fail(MRC_E_INVAL, "mrc_query: malformed offsets, token ids or document lengths");
    return MRC_OK;
}

// ------------------------------------------------------------------ logged entry points

mrc_status mrc_db_insert(mrc_db* db, const float* sig, int64_t n, int64_t* first_id, void* hip_stream) {
    CallLog L(db ? db->ctx : nullptr, "mrc_db_insert");
    L.add("n", n);
    const mrc_status st = db_insert_impl(db, sig, n, first_id, hip_stream);
    if (st == MRC_OK && db) L.add("rows", (int64_t)__atomic_load_n(&db->size, __ATOMIC_ACQUIRE));
    return L.done(st);
}

mrc_status mrc_query(mrc_ctx* ctx, const mrc_db* db, const mrc_model* model, const mrc_docs* q, int32_t topk, float tau,
                     int32_t precision, mrc_hit* topk_out, int32_t* n_hits, void* hip_stream) {
    CallLog L(ctx, "mrc_query");
    L.add("n_queries", q ? q->n_docs : (int64_t)-1);
    L.add("tokens", q ? q->n_tokens : (int64_t)-1);
    L.add("rows", db ? (int64_t)__atomic_load_n(&db->size, __ATOMIC_ACQUIRE) : (int64_t)-1);
    L.add("topk", (int64_t)topk);
    L.add("precision", (int64_t)precision);
    L.add("scan", (int64_t)(ctx ? ctx->scan_form : -1));
    if (ctx) ctx->query_attempts = 0;
    const mrc_status st = query_impl(ctx, db, model, q, topk, tau, precision, topk_out, n_hits, hip_stream);
    L.add("collect_attempts", (int64_t)(ctx ? ctx->query_attempts : -1));
    return L.done(st);
}

}  // extern "C"
