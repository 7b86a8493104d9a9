// FP8-e4m3 candidate search of the all-pairs comparison (its kernels are built
// without the VGPR-accumulator option: their operand fragments need the
// registers).
#include "allpairs.h"
#include "common.h"

namespace mrc {

mrc_status launch_compare_fp8(mrc_ctx* ctx, const uint8_t* q, int ldq_bytes, const float* scale, int64_t n, int nk,
                              const float* d_lo_thr, const TileOrder& ord, int64_t grid, PairSink cand,
                              hipStream_t s) {
    return launch_lowp_kernel<MRC_PREC_FP8>(ctx, q, ldq_bytes, scale, n, nk, d_lo_thr, ord, grid, cand, s);
}

}  // namespace mrc
