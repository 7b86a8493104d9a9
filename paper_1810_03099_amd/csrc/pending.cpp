// Entry points whose stages are not built yet: they fail with MRC_E_STATE.
#include "common.h"

using namespace mrc;

extern "C" {
mrc_status mrc_db_create(mrc_ctx*, int64_t, int32_t, uint32_t, mrc_db**) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_destroy(mrc_db*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_insert(mrc_db*, const float*, int64_t, int64_t*, void*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_insert_docs(mrc_db*, const mrc_model*, const mrc_docs*, int64_t*, void*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_size(const mrc_db*, int64_t*, int32_t*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_save(const mrc_db*, const char*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_db_load(mrc_ctx*, const char*, uint32_t, mrc_db**) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_query(mrc_ctx*, const mrc_db*, const mrc_model*, const mrc_docs*, int32_t, float, int32_t, mrc_hit*, int32_t*, void*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_start(mrc_ctx*, mrc_db*, const mrc_model*, const mrc_serve_opts*, mrc_server**) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_submit(mrc_server*, const int32_t*, int64_t, int32_t, uint64_t*) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_poll(mrc_server*, uint64_t, mrc_result*, int32_t) { return fail(MRC_E_STATE, "not available"); }
mrc_status mrc_serve_stop(mrc_server*) { return fail(MRC_E_STATE, "not available"); }
}
