// Host runtime of libmrc: thread-local errors, budgeted device allocation,
// named scratch buffers, and per-kernel HIP-event timing.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace mrc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mrc_status fail(mrc_status code, const std::string& msg) {
    set_error(msg);
    return code;
}

mrc_status hip_fail(mrc_ctx* ctx, hipError_t e, const char* what, const char* file, int line) {
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e),
             what, file, line);
    set_error(buf);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MRC_E_NOMEM;
    if (ctx) ctx->sticky = MRC_E_HIP;
    return MRC_E_HIP;
}

mrc_status dev_alloc(mrc_ctx* ctx, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return MRC_OK;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (ctx->used + bytes > ctx->budget)
            return fail(MRC_E_NOMEM, "device allocation of " + std::to_string(bytes) +
                                         " bytes would exceed the context budget");
        ctx->used += bytes;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->used -= bytes;
        *p = nullptr;
        return fail(MRC_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return MRC_OK;
}

void dev_free(mrc_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->used -= bytes;
}

constexpr size_t kRetiredMax = (size_t)1 << 30;  // retired scratch kept before one synchronised sweep

mrc_status scratch(mrc_ctx* ctx, const char* name, size_t bytes, void** p) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    auto it = ctx->scratch.find(name);
    if (it != ctx->scratch.end() && it->second.second >= bytes) {
        *p = it->second.first;
        return MRC_OK;
    }
    if (it != ctx->scratch.end()) {
        // grow: the old buffer may still be in use by queued work on this
        // context's streams. Retire it instead of waiting for the whole
        // device (a device-wide wait, and hipFree, would also stall every
        // other context's work, e.g. the other serving slots)
        ctx->retired.push_back(it->second);
        ctx->retired_bytes += it->second.second;
        ctx->scratch.erase(it);
        if (ctx->retired_bytes > kRetiredMax) {
            MRC_HIP_TRY(ctx, hipDeviceSynchronize());
            for (auto& r : ctx->retired) dev_free(ctx, r.first, r.second);
            ctx->retired.clear();
            ctx->retired_bytes = 0;
        }
    }
    size_t want = bytes + bytes / 4;  // headroom against repeated growth
    void* q = nullptr;
    mrc_status st = dev_alloc(ctx, &q, want);
    if (st != MRC_OK) {
        st = dev_alloc(ctx, &q, bytes);
        if (st != MRC_OK) return st;
        want = bytes;
    }
    ctx->scratch[name] = {q, want};
    *p = q;
    return MRC_OK;
}

static hipEvent_t take_event(mrc_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timer_begin(mrc_ctx* ctx, const char* name, hipStream_t s, hipEvent_t* ev) {
    (void)name;
    if (!ctx || !ctx->timing) return;
    ev[0] = take_event(ctx);
    ev[1] = take_event(ctx);
    if (ev[0]) (void)hipEventRecord(ev[0], s);
}

void timer_end(mrc_ctx* ctx, const char* name, hipStream_t s, hipEvent_t* ev) {
    if (!ctx || !ctx->timing || !ev[0] || !ev[1]) return;
    (void)hipEventRecord(ev[1], s);
    ctx->pending.push_back({name, {ev[0], ev[1]}});
}

// ------------------------------------------------------------------ logging

namespace {
std::once_flag g_log_once;
int g_log_level = 0;
FILE* g_log_file = nullptr;
std::mutex g_log_mu;
std::chrono::steady_clock::time_point g_log_t0;

void log_init() {
    const char* lv = std::getenv("MRC_LOG");
    g_log_level = lv ? std::max(0, std::min(3, std::atoi(lv))) : 0;
    if (g_log_level == 0) return;
    const char* path = std::getenv("MRC_LOG_FILE");
    g_log_file = path && *path ? std::fopen(path, "a") : nullptr;
    if (!g_log_file) g_log_file = stderr;
    g_log_t0 = std::chrono::steady_clock::now();
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - g_log_t0).count();
}

std::string num(double v) {
    char b[64];
    std::snprintf(b, sizeof b, "%.6g", v);
    return b;
}
}  // namespace

int log_level() {
    std::call_once(g_log_once, log_init);
    return g_log_level;
}

void log_line(const std::string& event, const std::string& fields) {
    if (log_level() == 0) return;
    std::string line = "{\"t_ms\": " + num(now_ms()) + ", \"event\": \"" + event + "\"";
    if (!fields.empty()) line += ", " + fields;
    line += "}\n";
    std::lock_guard<std::mutex> g(g_log_mu);
    std::fputs(line.c_str(), g_log_file);
    std::fflush(g_log_file);
}

CallLog::CallLog(mrc_ctx* c, const char* n) : ctx(c), name(n) {
    on = log_level() >= 1;
    if (!on) return;
    t0 = now_ms();
    if (log_level() >= 2 && ctx && ctx->sticky == MRC_OK) {
        timer_collect(ctx);
        before = ctx->timers;
        timing_was = ctx->timing;
        ctx->timing = true;
        timers = true;
    }
}

void CallLog::add(const char* key, int64_t v) {
    if (!on) return;
    if (!fields.empty()) fields += ", ";
    fields += "\"" + std::string(key) + "\": " + std::to_string(v);
}

void CallLog::add(const char* key, double v) {
    if (!on) return;
    if (!fields.empty()) fields += ", ";
    fields += "\"" + std::string(key) + "\": " + num(v);
}

mrc_status CallLog::done(mrc_status st) {
    if (!on) return st;
    std::string f = "\"call\": \"" + std::string(name) + "\", \"status\": " + std::to_string(st) +
                    ", \"wall_ms\": " + num(now_ms() - t0);
    if (!fields.empty()) f += ", " + fields;
    if (timers) {
        timer_collect(ctx);
        std::string stages;
        for (const auto& kv : ctx->timers) {
            auto it = before.find(kv.first);
            const double ms = kv.second.total_ms - (it == before.end() ? 0.0 : it->second.total_ms);
            const int64_t nl = kv.second.launches - (it == before.end() ? 0 : it->second.launches);
            if (nl <= 0) continue;
            if (!stages.empty()) stages += ", ";
            stages += "\"" + kv.first + "\": {\"ms\": " + num(ms) + ", \"launches\": " + std::to_string(nl) + "}";
        }
        f += ", \"stages\": {" + stages + "}";
        ctx->timing = timing_was;
    }
    log_line("call", f);
    return st;
}

void timer_collect(mrc_ctx* ctx) {
    for (auto& p : ctx->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            auto& t = ctx->timers[p.first];
            t.total_ms += ms;
            t.launches += 1;
        }
        ctx->event_pool.push_back(p.second.first);
        ctx->event_pool.push_back(p.second.second);
    }
    ctx->pending.clear();
}

// start[b] = first tile index of band b (b = 0 .. n_bands): one thread per band
// sums the sizes of the bands before it.
__global__ void k_band_starts(int nb, int n_bands, int B, int64_t* __restrict__ start) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > n_bands) return;
    int64_t t = 0;
    for (int x = 0; x < b; ++x) {
        const int r0 = x * B, h = min(B, nb - r0);
        t += (int64_t)h * (h + 1) / 2 + (int64_t)h * (nb - r0 - h);
    }
    start[b] = t;
}

mrc_status make_tile_order(mrc_ctx* ctx, int nb, int per_block, TileOrder* ord, int64_t* grid, hipStream_t s,
                           int64_t* table, int band_h) {
    if (band_h < 1) return fail(MRC_E_INVAL, "band height must be positive");
    const int B = band_h;
    const int n_bands = (nb + B - 1) / B;
    int64_t t = 0;
    for (int b = 0; b < n_bands; ++b) {
        const int r0 = b * B, h = std::min(B, nb - r0);
        t += (int64_t)h * (h + 1) / 2 + (int64_t)h * (nb - r0 - h);
    }
    void* d = table;
    if (!table) {
        // the context keeps the table of the last tile count it was made for
        auto it = ctx->scratch.find("tile_order");
        const bool cached = ctx->tile_order_nb == nb && ctx->tile_order_bh == B && it != ctx->scratch.end();
        MRC_TRY(scratch(ctx, "tile_order", (size_t)(n_bands + 1) * sizeof(int64_t), &d));
        if (!cached) {
            hipLaunchKernelGGL(k_band_starts, dim3((unsigned)ceil_div(n_bands + 1, 256)), dim3(256), 0, s, nb,
                               n_bands, B, (int64_t*)d);
            MRC_HIP_TRY(ctx, hipGetLastError());
            ctx->tile_order_nb = nb;
            ctx->tile_order_bh = B;
        }
    } else {
        hipLaunchKernelGGL(k_band_starts, dim3((unsigned)ceil_div(n_bands + 1, 256)), dim3(256), 0, s, nb, n_bands, B,
                           table);
        MRC_HIP_TRY(ctx, hipGetLastError());
    }
    ord->nb = nb;
    ord->n_bands = n_bands;
    ord->bh = B;
    ord->per_block = per_block;
    ord->n_tiles = t;
    ord->blocks = (t + per_block - 1) / per_block;
    ord->per_xcd = (ord->blocks + 7) / 8;
    ord->band_start = (const int64_t*)d;
    *grid = ord->per_xcd * 8;
    if (*grid > 0x7FFFFFFFLL) return fail(MRC_E_INVAL, "too many tiles for one launch");
    return MRC_OK;
}

int64_t persistent_grid(mrc_ctx* ctx, const void* kernel, int block, int64_t cap) {
    // the occupancy and CU count of a (device, kernel, block size) are asked
    // of the runtime once per process
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, int>, std::pair<int, int>> known;
    int per_cu = 1, cus = 256;
    {
        std::lock_guard<std::mutex> g(mu);
        const auto key = std::make_tuple(ctx->device, kernel, block);
        auto it = known.find(key);
        if (it != known.end()) {
            per_cu = it->second.first;
            cus = it->second.second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
                cus < 1)
                cus = 256;
            (void)hipGetLastError();
            known[key] = {per_cu, cus};
        }
    }
    int64_t g = (int64_t)per_cu * cus;
    cap = (cap + 7) / 8 * 8;
    if (g > cap) g = cap;
    g = g / 8 * 8;
    return g < 8 ? 8 : g;
}

void ctx_free_now(mrc_ctx* ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    timer_collect(ctx);
    for (auto& kv : ctx->scratch) (void)hipFree(kv.second.first);
    for (auto& r : ctx->retired) (void)hipFree(r.first);
    if (ctx->model_spare) (void)hipFree(ctx->model_spare);
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    delete ctx;
}

void ctx_retain(mrc_ctx* ctx) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ++ctx->live;
}

void ctx_release(mrc_ctx* ctx) {
    bool now;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        now = --ctx->live == 0 && ctx->closing;
    }
    if (now) ctx_free_now(ctx);
}

}  // namespace mrc

using namespace mrc;

extern "C" {

const char* mrc_last_error(void) { return g_last_error.c_str(); }

mrc_status mrc_ctx_create(mrc_ctx** out, int32_t device, size_t hbm_budget_bytes) {
    if (!out) return fail(MRC_E_INVAL, "mrc_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(MRC_E_HIP, "mrc_ctx_create: no HIP device");
    if (device < 0 || device >= n) return fail(MRC_E_INVAL, "mrc_ctx_create: bad device index");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice", __FILE__, __LINE__);
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipMemGetInfo", __FILE__, __LINE__);
    mrc_ctx* ctx = new mrc_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)total_b);
    e = hipMalloc((void**)&ctx->d_flags, 64 * sizeof(int64_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_flags, 64 * sizeof(int64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(ctx->d_flags, 0, 64 * sizeof(int64_t));
    mrc_status st = e != hipSuccess ? hip_fail(nullptr, e, "context flags", __FILE__, __LINE__) : MRC_OK;
    if (st == MRC_OK) st = noalloc_setup(device);  // the no-allocation comparison's array on this device
    if (st != MRC_OK) {
        if (ctx->d_flags) (void)hipFree(ctx->d_flags);
        if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
        delete ctx;
        return st;
    }
    *out = ctx;
    return MRC_OK;
}

mrc_status mrc_ctx_destroy(mrc_ctx* ctx) {
    if (!ctx) return MRC_OK;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->closing = true;
        if (ctx->live > 0) return MRC_OK;  // the last model or database frees it
    }
    ctx_free_now(ctx);
    return MRC_OK;
}

mrc_status mrc_ctx_memory(const mrc_ctx* ctx, size_t* used, size_t* budget) {
    if (!ctx) return fail(MRC_E_INVAL, "mrc_ctx_memory: ctx is NULL");
    if (used) *used = ctx->used;
    if (budget) *budget = ctx->budget;
    return MRC_OK;
}

mrc_status mrc_ctx_set_timing(mrc_ctx* ctx, int32_t enabled) {
    if (!ctx) return fail(MRC_E_INVAL, "mrc_ctx_set_timing: ctx is NULL");
    timer_collect(ctx);
    ctx->timing = enabled != 0;
    return MRC_OK;
}

mrc_status mrc_ctx_set_scan(mrc_ctx* ctx, int32_t form) {
    if (!ctx) return fail(MRC_E_INVAL, "mrc_ctx_set_scan: ctx is NULL");
    if (form != MRC_SCAN_GRID && form != MRC_SCAN_PERSISTENT) return fail(MRC_E_INVAL, "mrc_ctx_set_scan: bad form");
    ctx->scan_form = form;
    return MRC_OK;
}

mrc_status mrc_ctx_kernel_time(mrc_ctx* ctx, const char* kernel, double* total_ms,
                               int64_t* launches, int32_t reset) {
    if (!ctx || !kernel) return fail(MRC_E_INVAL, "mrc_ctx_kernel_time: NULL argument");
    timer_collect(ctx);
    auto it = ctx->timers.find(kernel);
    if (total_ms) *total_ms = it == ctx->timers.end() ? 0.0 : it->second.total_ms;
    if (launches) *launches = it == ctx->timers.end() ? 0 : it->second.launches;
    if (reset && it != ctx->timers.end()) ctx->timers.erase(it);
    return MRC_OK;
}

}  // extern "C"
