// Entry points whose stages are not built yet: they fail with MRC_E_STATE.
#include "common.h"

using namespace mrc;

extern "C" {
mrc_status mrc_serve_start(mrc_ctx*, mrc_db*, const mrc_model*, const mrc_serve_opts*, mrc_server**) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_submit(mrc_server*, const int32_t*, int64_t, int32_t, uint64_t*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_poll(mrc_server*, uint64_t, mrc_result*, int32_t) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_stop(mrc_server*) { return fail(MRC_E_STATE, "not available"); }
}
