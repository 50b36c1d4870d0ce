// Serving loop (placeholder: synchronous).
#include "tc_api_internal.h"

namespace tc {
struct serve_state {
    std::map<tc_ticket, std::vector<uint64_t>> done;
    tc_ticket next = 1;
};
void serve_shutdown(tc_context_s* ctx) { delete ctx->serve; ctx->serve = nullptr; }
}  // namespace tc

using namespace tc;

extern "C" int tc_submit(tc_context ctx, tc_graph g, tc_ticket* out) {
    if (!ctx || !g || !out) return TC_ERR_ARG;
    std::vector<uint64_t> c(16);
    int rc = tc_census(ctx, g, c.data());
    if (rc != TC_OK) return rc;
    if (!ctx->serve) ctx->serve = new serve_state();
    *out = ctx->serve->next++;
    ctx->serve->done[*out] = c;
    return TC_OK;
}

extern "C" int tc_poll(tc_context ctx, tc_ticket t, uint64_t counts[16], int* done) {
    if (!ctx || !counts || !done) return TC_ERR_ARG;
    if (!ctx->serve || !ctx->serve->done.count(t)) return TC_ERR_NOT_FOUND;
    for (int k = 0; k < 16; ++k) counts[k] = ctx->serve->done[t][k];
    ctx->serve->done.erase(t);
    *done = 1;
    return TC_OK;
}

extern "C" int tc_serve_get_stats(tc_context ctx, tc_serve_stats* out) {
    if (!ctx || !out) return TC_ERR_ARG;
    *out = tc_serve_stats{};
    return TC_OK;
}

extern "C" int tc_serve_reset_stats(tc_context ctx) { return ctx ? TC_OK : TC_ERR_ARG; }
