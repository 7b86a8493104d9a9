// All-pairs FP32 comparison that allocates nothing: the same normalisation
// and FP32 matrix-core comparison kernels as mrc_compare at MRC_PREC_FP32,
// with their working memory (pair counter, the tile order's band table, the
// unit signatures in the matrix-core layout) in a fixed device array of the
// library instead of context scratch. For callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).
//
// Each GPU holds its own copy of the array until the process ends. Host code
// never uses the array's name as an address: the context's set-up resolves
// the device address once per device (hipGetSymbolAddress, that device
// current) and every launch and copy takes that pointer.
#include <mutex>

#include "common.h"

// [0, 256)                       pair counter (word 0)
// [256, 8192)                    band table of the tile order (992 words)
// [8192, 8192 + 32 MiB)          unit signatures, matrix-core layout
static __device__ __align__(256) unsigned char scratch[8192 + MRC_NOALLOC_MAX_UNIT_BYTES];

namespace {

constexpr size_t kTableOff = 256;
constexpr size_t kTableWords = (8192 - kTableOff) / sizeof(int64_t);
constexpr size_t kUnitOff = 8192;
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace mrc {

mrc_status noalloc_setup(int device) {
    // `::scratch` names the array (mrc::scratch is the context's scratch arena)
    static_assert(sizeof(::scratch) == kUnitOff + MRC_NOALLOC_MAX_UNIT_BYTES, "the fixed array");
    if (device < 0 || device >= kMaxDevices) return fail(MRC_E_INVAL, "device index above the supported 64");
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return MRC_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch));
    if (e != hipSuccess || !p) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    g_ptr[device] = p;
    return MRC_OK;
}

}  // namespace mrc

extern "C" mrc_status mrc_compare_f32_noalloc(mrc_ctx* ctx, const float* sig, int64_t n, int32_t k, float tau,
                                              mrc_pair* pairs_out, int64_t capacity, int64_t* n_found,
                                              void* hip_stream) {
    using namespace mrc;
    MRC_TRY(check_ctx(ctx, "mrc_compare_f32_noalloc"));
    if (!n_found) return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: n_found is NULL");
    *n_found = 0;
    if (n < 0 || k < 1 || k > 1024) return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: bad n or k");
    if (n > 0 && !sig) return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: sig is NULL");
    if (capacity < 0 || (capacity > 0 && !pairs_out))
        return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: bad output buffer");
    if (!(tau == tau)) return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: tau is NaN");
    // the unit signatures (128-row tiles, whole 16-column fragments) and the
    // band table (64- or 128-row tiles in bands of TileOrder::kBand) must fit
    const int64_t n_pad = ceil_div(n > 0 ? n : 1, 128) * 128;
    const int64_t kp = 16 * (int64_t)mfma_chunks(k);
    const int64_t unit_bytes = n_pad * kp * (int64_t)sizeof(float);
    const int64_t table_words = ceil_div(ceil_div(n, 64), TileOrder::kBand) + 2;
    if (unit_bytes > (int64_t)MRC_NOALLOC_MAX_UNIT_BYTES || table_words > (int64_t)kTableWords)
        return fail(MRC_E_INVAL, "mrc_compare_f32_noalloc: n x k exceeds the fixed scratch array "
                                 "(ceil(n/128)*128 rows x 16*mfma_chunks(k) columns x 4 bytes = " +
                                     std::to_string(unit_bytes) + " bytes, at most " +
                                     std::to_string(MRC_NOALLOC_MAX_UNIT_BYTES) + ")");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_ptr[ctx->device] : nullptr;
    }
    if (!base) return fail(MRC_E_STATE, "mrc_compare_f32_noalloc: the scratch array was not set up for this device");
    unsigned char* b = (unsigned char*)base;
    hipStream_t s = (hipStream_t)hip_stream;
    int64_t* counter = (int64_t*)b;
    float* umfma = (float*)(b + kUnitOff);
    MRC_TRY(clear_words(ctx, counter, 1, s));  // a fill kernel: no memset node under capture
    if (n >= 2) {
        MRC_TRY(launch_normalise(ctx, sig, n, k, nullptr, nullptr, nullptr, nullptr, nullptr, s, umfma));
        PairSink sink{pairs_out, capacity, (unsigned long long*)counter};
        MRC_TRY(launch_compare_f32(ctx, umfma, n, k, tau, sink, s, (int64_t*)(b + kTableOff)));
    }
    MRC_HIP_TRY(ctx, hipMemcpyAsync(ctx->h_flags, counter, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MRC_HIP_TRY(ctx, hipStreamSynchronize(s));
    const int64_t found = ctx->h_flags[0];
    *n_found = found;
    if (found > capacity) return fail(MRC_E_OVERFLOW, "mrc_compare_f32_noalloc: more pairs than capacity");
    return MRC_OK;
}
