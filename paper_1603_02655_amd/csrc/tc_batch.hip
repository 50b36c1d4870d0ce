// Batched census (placeholder: per-graph launches).
#include "tc_api_internal.h"

namespace tc {
struct batch_plan {};
void batch_release_all(tc_context_s* ctx) { delete ctx->batch; ctx->batch = nullptr; }
void batch_forget_graph_locked(tc_context_s* ctx, tc_graph) { delete ctx->batch; ctx->batch = nullptr; }
}  // namespace tc

extern "C" int tc_census_batch(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts) {
    return tc_census_each(ctx, graphs, count, counts);
}

extern "C" int tc_autotune(tc_context ctx, const tc_graph*, int32_t, const char*, tc_tuning* best) {
    return best ? tc_get_tuning(ctx, best) : TC_OK;
}
