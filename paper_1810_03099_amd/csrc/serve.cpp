// Serving loop on the GPU: the continuous-batching scheduler of serve_core
// driving one worker context and HIP stream per slot. Query batches run
// mrc_query against the live database snapshot; insert batches are signed on
// the slot and appended under the database lock. Batches on different slots
// overlap on the device.
#include <algorithm>

#include <chrono>

#include "common.h"
#include "serve_core.h"

using namespace mrc;

namespace {

struct GpuSlot {
    mrc_ctx* ctx = nullptr;
    hipStream_t s = nullptr;
    int32_t* h_tok = nullptr;
    int64_t* h_off = nullptr;
    int64_t h_tok_cap = 0, h_off_cap = 0;
    int32_t* d_tok = nullptr;
    int64_t* d_off = nullptr;
    int64_t d_tok_cap = 0, d_off_cap = 0;
    mrc_hit* d_top = nullptr;
    int32_t* d_hits = nullptr;
    float* d_sig = nullptr;
    int64_t out_cap = 0;
    // query results come back into pinned host buffers: an asynchronous copy
    // into pageable memory goes through the runtime's staging path, which can
    // hold one slot's copies behind another slot's batch
    mrc_hit* h_top = nullptr;
    int32_t* h_hits = nullptr;
    double prep_ms = 0, work_ms = 0, fetch_ms = 0;  // phases of the last batch (structured log, level 3)
};

class GpuExecutor : public mrc_serve::Executor {
   public:
    GpuExecutor(mrc_db* db, const mrc_model* m, const mrc_serve_opts& o) : db_(db), model_(m), o_(o) {}
    ~GpuExecutor() override {
        for (auto& sl : slots_) {
            if (sl.s) (void)hipStreamSynchronize(sl.s);
            if (sl.h_tok) (void)hipHostFree(sl.h_tok);
            if (sl.h_off) (void)hipHostFree(sl.h_off);
            if (sl.h_top) (void)hipHostFree(sl.h_top);
            if (sl.h_hits) (void)hipHostFree(sl.h_hits);
            if (sl.ctx) {
                dev_free(sl.ctx, sl.d_tok, (size_t)sl.d_tok_cap * 4);
                dev_free(sl.ctx, sl.d_off, (size_t)sl.d_off_cap * 8);
                dev_free(sl.ctx, sl.d_top, (size_t)sl.out_cap * 16 * sizeof(mrc_hit));
                dev_free(sl.ctx, sl.d_hits, (size_t)sl.out_cap * 4);
                dev_free(sl.ctx, sl.d_sig, (size_t)sl.out_cap * db_->k * 4);
                mrc_ctx_destroy(sl.ctx);
            }
            if (sl.s) (void)hipStreamDestroy(sl.s);
        }
    }
    mrc_status init(mrc_ctx* main, int n) {
        slots_.resize(n);
        for (auto& sl : slots_) {
            MRC_TRY(mrc_ctx_create(&sl.ctx, main->device, main->budget));
            sl.ctx->scan_form = main->scan_form;
            MRC_HIP_TRY(main, hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking));
        }
        return MRC_OK;
    }
    int slots() const override { return (int)slots_.size(); }
    size_t batch_bytes(int kind, int64_t n, int64_t t) const override {
        const size_t per_doc = kind == mrc_serve::kQuery ? (size_t)db_->k * 40 + 16 * 2048 + 64 * 1024 : db_->k * 40;
        return (size_t)t * 4 + (size_t)(n + 1) * 8 + (size_t)n * per_doc;
    }
    int run(int slot, mrc_serve::Batch& b, std::vector<mrc_serve::Result>& out) override {
        if (log_level() < 3) return run_batch(slot, b, out);
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = run_batch(slot, b, out);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        log_line("serve_batch", "\"slot\": " + std::to_string(slot) + ", \"kind\": \"" +
                                    (b.kind == mrc_serve::kInsert ? "insert" : "query") + "\", \"docs\": " +
                                    std::to_string(b.reqs.size()) + ", \"tokens\": " + std::to_string(b.tokens) +
                                    ", \"status\": " + std::to_string(rc) + ", \"ms\": " + std::to_string(ms) +
                                    ", \"prep_ms\": " + std::to_string(slots_[slot].prep_ms) + ", \"work_ms\": " +
                                    std::to_string(slots_[slot].work_ms) + ", \"fetch_ms\": " +
                                    std::to_string(slots_[slot].fetch_ms));
        return rc;
    }

    int run_batch(int slot, mrc_serve::Batch& b, std::vector<mrc_serve::Result>& out) {
        GpuSlot& sl = slots_[slot];
        using clk = std::chrono::steady_clock;
        const auto t0 = clk::now();
        auto since = [](clk::time_point a) { return std::chrono::duration<double, std::milli>(clk::now() - a).count(); };
        const int64_t n = (int64_t)b.reqs.size(), T = std::max<int64_t>(1, b.tokens);
        mrc_status st = reserve(sl, n, T);
        if (st != MRC_OK) return st;
        sl.h_off[0] = 0;
        int64_t pos = 0;
        for (int64_t i = 0; i < n; ++i) {
            const auto& tk = b.reqs[i].tokens;
            std::copy(tk.begin(), tk.end(), sl.h_tok + pos);
            pos += (int64_t)tk.size();
            sl.h_off[i + 1] = pos;
        }
        if (hipMemcpyAsync(sl.d_tok, sl.h_tok, (size_t)std::max<int64_t>(pos, 1) * 4, hipMemcpyHostToDevice, sl.s) != hipSuccess ||
            hipMemcpyAsync(sl.d_off, sl.h_off, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, sl.s) != hipSuccess)
            return MRC_E_HIP;
        mrc_docs d{n, sl.d_off, sl.d_tok, std::max<int64_t>(pos, 1)};
        sl.prep_ms = since(t0);
        const auto t1 = clk::now();
        if (b.kind == mrc_serve::kInsert) {
            st = mrc_sign(sl.ctx, model_, &d, sl.d_sig, nullptr, sl.s);
            int64_t first = -1;
            if (st == MRC_OK) st = mrc_db_insert(db_, sl.d_sig, n, &first, sl.s);
            if (st != MRC_OK) return st;
            for (int64_t i = 0; i < n; ++i) {
                out[i].status = MRC_OK;
                out[i].id = first + i;
            }
            return MRC_OK;
        }
        const int topk = o_.topk;
        st = mrc_query(sl.ctx, db_, model_, &d, topk, o_.tau, o_.precision, sl.d_top, sl.d_hits, sl.s);
        if (st != MRC_OK) return st;
        sl.work_ms = since(t1);
        const auto t2 = clk::now();
        if (hipMemcpyAsync(sl.h_top, sl.d_top, (size_t)n * topk * sizeof(mrc_hit), hipMemcpyDeviceToHost, sl.s) != hipSuccess ||
            hipMemcpyAsync(sl.h_hits, sl.d_hits, (size_t)n * 4, hipMemcpyDeviceToHost, sl.s) != hipSuccess ||
            hipStreamSynchronize(sl.s) != hipSuccess)
            return MRC_E_HIP;
        sl.fetch_ms = since(t2);
        for (int64_t i = 0; i < n; ++i) {
            auto& r = out[i];
            r.status = MRC_OK;
            r.n_hits = sl.h_hits[i];
            r.top.clear();
            for (int p = 0; p < topk; ++p) {
                const mrc_hit& h = sl.h_top[(size_t)i * topk + p];
                if (h.id >= 0) r.top.push_back({h.id, h.s});
            }
        }
        return MRC_OK;
    }

   private:
    mrc_status reserve(GpuSlot& sl, int64_t n, int64_t T) {
        if (T > sl.h_tok_cap) {
            if (sl.h_tok) (void)hipHostFree(sl.h_tok);
            sl.h_tok = nullptr;
            const int64_t c = T + T / 2;
            MRC_HIP_TRY(sl.ctx, hipHostMalloc((void**)&sl.h_tok, (size_t)c * 4, hipHostMallocDefault));
            sl.h_tok_cap = c;
        }
        if (n + 1 > sl.h_off_cap) {
            if (sl.h_off) (void)hipHostFree(sl.h_off);
            sl.h_off = nullptr;
            const int64_t c = 2 * (n + 1);
            MRC_HIP_TRY(sl.ctx, hipHostMalloc((void**)&sl.h_off, (size_t)c * 8, hipHostMallocDefault));
            sl.h_off_cap = c;
        }
        if (T > sl.d_tok_cap) {
            dev_free(sl.ctx, sl.d_tok, (size_t)sl.d_tok_cap * 4);
            sl.d_tok = nullptr;
            const int64_t c = T + T / 2;
            MRC_TRY(dev_alloc(sl.ctx, (void**)&sl.d_tok, (size_t)c * 4));
            sl.d_tok_cap = c;
        }
        if (n + 1 > sl.d_off_cap) {
            dev_free(sl.ctx, sl.d_off, (size_t)sl.d_off_cap * 8);
            sl.d_off = nullptr;
            const int64_t c = 2 * (n + 1);
            MRC_TRY(dev_alloc(sl.ctx, (void**)&sl.d_off, (size_t)c * 8));
            sl.d_off_cap = c;
        }
        if (n > sl.out_cap) {
            dev_free(sl.ctx, sl.d_top, (size_t)sl.out_cap * 16 * sizeof(mrc_hit));
            dev_free(sl.ctx, sl.d_hits, (size_t)sl.out_cap * 4);
            dev_free(sl.ctx, sl.d_sig, (size_t)sl.out_cap * db_->k * 4);
            if (sl.h_top) (void)hipHostFree(sl.h_top);
            if (sl.h_hits) (void)hipHostFree(sl.h_hits);
            sl.d_top = nullptr;
            sl.d_hits = nullptr;
            sl.d_sig = nullptr;
            sl.h_top = nullptr;
            sl.h_hits = nullptr;
            sl.out_cap = 0;
            const int64_t c = std::max<int64_t>(2 * n, 64);
            MRC_TRY(dev_alloc(sl.ctx, (void**)&sl.d_top, (size_t)c * 16 * sizeof(mrc_hit)));
            MRC_TRY(dev_alloc(sl.ctx, (void**)&sl.d_hits, (size_t)c * 4));
            MRC_TRY(dev_alloc(sl.ctx, (void**)&sl.d_sig, (size_t)c * db_->k * 4));
            MRC_HIP_TRY(sl.ctx, hipHostMalloc((void**)&sl.h_top, (size_t)c * 16 * sizeof(mrc_hit), hipHostMallocDefault));
            MRC_HIP_TRY(sl.ctx, hipHostMalloc((void**)&sl.h_hits, (size_t)c * 4, hipHostMallocDefault));
            sl.out_cap = c;
        }
        return MRC_OK;
    }

    mrc_db* db_;
    const mrc_model* model_;
    mrc_serve_opts o_;
    std::vector<GpuSlot> slots_;
};

}  // namespace

struct mrc_server {
    GpuExecutor* ex = nullptr;
    mrc_serve::Scheduler* sched = nullptr;
    int32_t vocab = 0;
    mrc_db* db = nullptr;            // used (not owned): destroying them waits for the server
    const mrc_model* model = nullptr;
};

extern "C" {

mrc_status mrc_serve_start(mrc_ctx* ctx, mrc_db* db, const mrc_model* model, const mrc_serve_opts* opts,
                           mrc_server** out) {
    if (!ctx || !db || !model || !opts || !out) return fail(MRC_E_INVAL, "mrc_serve_start: NULL argument");
    *out = nullptr;
    if (model->k != db->k) return fail(MRC_E_INVAL, "mrc_serve_start: model and database differ in k");
    if (db->k > kQueryMaxK) return fail(MRC_E_INVAL, "mrc_serve_start: queries support k <= 512");
    if (opts->max_batch < 1 || opts->max_batch > 4096 || opts->n_streams < 1 || opts->n_streams > 4 ||
        opts->topk < 1 || opts->topk > 16 || opts->precision < MRC_PREC_FP32 || opts->precision > MRC_PREC_FP8 ||
        !(opts->hbm_frac > 0.0 && opts->hbm_frac <= 1.0) || opts->max_queue < 1 || opts->max_batch_tokens < 1 ||
        opts->max_wait_us < 0)
        return fail(MRC_E_INVAL, "mrc_serve_start: bad options");
    mrc_server* srv = new mrc_server();
    srv->vocab = model->vocab;
    srv->ex = new GpuExecutor(db, model, *opts);
    mrc_status st = srv->ex->init(ctx, opts->n_streams);
    if (st != MRC_OK) {
        delete srv->ex;
        delete srv;
        return st;
    }
    mrc_serve::Options so;
    so.max_batch = opts->max_batch;
    so.max_batch_tokens = opts->max_batch_tokens;
    so.max_queue = opts->max_queue;
    so.mem_cap = (size_t)(opts->hbm_frac * (double)ctx->budget);
    so.max_wait_us = opts->max_wait_us;
    srv->sched = new mrc_serve::Scheduler(srv->ex, so);
    srv->db = db;
    srv->model = model;
    {
        std::lock_guard<std::mutex> g(db->ctx->mu);
        ++db->users;
    }
    {
        std::lock_guard<std::mutex> g(model->ctx->mu);
        ++model->users;
    }
    *out = srv;
    return MRC_OK;
}

mrc_status mrc_serve_submit(mrc_server* srv, const int32_t* tokens, int64_t len, int32_t kind, uint64_t* ticket) {
    if (!srv || !ticket || len < 0 || (len > 0 && !tokens)) return fail(MRC_E_INVAL, "mrc_serve_submit: bad argument");
    for (int64_t i = 0; i < len; ++i)
        if (tokens[i] < 0 || tokens[i] >= srv->vocab) return fail(MRC_E_INVAL, "mrc_serve_submit: token id outside [0, vocab)");
    const int rc = srv->sched->submit(tokens, len, kind, ticket);
    if (rc == mrc_serve::kBusy) return fail(MRC_E_BUSY, "mrc_serve_submit: queue full");
    if (rc != mrc_serve::kOk) return fail(rc, "mrc_serve_submit: rejected");
    return MRC_OK;
}

mrc_status mrc_serve_submit_many(mrc_server* srv, const int64_t* offsets, const int32_t* tokens, int64_t n,
                                 int32_t kind, uint64_t* tickets, int64_t* n_accepted) {
    if (!n_accepted) return fail(MRC_E_INVAL, "mrc_serve_submit_many: NULL n_accepted");
    *n_accepted = 0;
    if (!srv || n < 0 || (n > 0 && (!offsets || !tickets)))
        return fail(MRC_E_INVAL, "mrc_serve_submit_many: bad argument");
    if (n > 0 && offsets[0] < 0) return fail(MRC_E_INVAL, "mrc_serve_submit_many: negative offset");
    for (int64_t d = 0; d < n; ++d) {
        if (offsets[d + 1] < offsets[d]) return fail(MRC_E_INVAL, "mrc_serve_submit_many: offsets decrease");
        for (int64_t i = offsets[d]; i < offsets[d + 1]; ++i)
            if (tokens[i] < 0 || tokens[i] >= srv->vocab)
                return fail(MRC_E_INVAL, "mrc_serve_submit_many: token id outside [0, vocab)");
    }
    const int rc = srv->sched->submit_many(offsets, tokens, n, kind, tickets, n_accepted);
    if (rc == mrc_serve::kBusy) return fail(MRC_E_BUSY, "mrc_serve_submit_many: queue full");
    if (rc != mrc_serve::kOk) return fail(rc, "mrc_serve_submit_many: rejected");
    return MRC_OK;
}

mrc_status mrc_serve_poll(mrc_server* srv, uint64_t ticket, mrc_result* out, int32_t wait_ms) {
    if (!srv || !out) return fail(MRC_E_INVAL, "mrc_serve_poll: NULL argument");
    mrc_serve::Result r;
    const int rc = srv->sched->poll(ticket, &r, wait_ms);
    if (rc == mrc_serve::kBusy) return MRC_E_BUSY;
    if (rc != mrc_serve::kOk) return fail(MRC_E_INVAL, "mrc_serve_poll: unknown ticket");
    memset(out, 0, sizeof(*out));
    out->status = r.status;
    out->kind = r.kind;
    out->id = r.id;
    out->n_hits = r.n_hits;
    out->n_top = (int32_t)std::min<size_t>(64, r.top.size());
    for (int i = 0; i < out->n_top; ++i) {
        out->top[i].id = r.top[i].id;
        out->top[i].s = r.top[i].s;
    }
    out->t_submit_ms = r.t_submit;
    out->t_start_ms = r.t_start;
    out->t_done_ms = r.t_done;
    return MRC_OK;
}

mrc_status mrc_serve_stop(mrc_server* srv) {
    if (!srv) return MRC_OK;
    srv->sched->stop();
    if (log_level() >= 1) {
        const mrc_serve::Stats st = srv->sched->stats();
        log_line("serve_stop", "\"submitted\": " + std::to_string(st.submitted) + ", \"rejected\": " +
                                   std::to_string(st.rejected) + ", \"completed\": " + std::to_string(st.completed) +
                                   ", \"failed\": " + std::to_string(st.failed) + ", \"batches\": " +
                                   std::to_string(st.batches) + ", \"peak_in_flight_bytes\": " +
                                   std::to_string(st.peak_in_flight_bytes) + ", \"peak_concurrent_batches\": " +
                                   std::to_string(st.peak_concurrent_batches));
    }
    delete srv->sched;
    delete srv->ex;
    // a database or model destroyed while this server ran is freed now
    mrc_db* db = srv->db;
    mrc_model* model = const_cast<mrc_model*>(srv->model);
    delete srv;
    bool free_db_now, free_model_now;
    {
        std::lock_guard<std::mutex> g(db->ctx->mu);
        free_db_now = --db->users == 0 && db->closing;
    }
    {
        std::lock_guard<std::mutex> g(model->ctx->mu);
        free_model_now = --model->users == 0 && model->closing;
    }
    if (free_db_now || free_model_now) {
        (void)hipSetDevice(db->ctx->device);
        (void)hipDeviceSynchronize();
    }
    if (free_db_now) free_db(db);
    if (free_model_now) free_model(model);
    return MRC_OK;
}

}  // extern "C"
