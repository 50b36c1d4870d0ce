// Autotuner for the degree-bucket thresholds and launch sizes.
//
// Coordinate descent over small candidate grids, two sweeps.  The objective is
// the wall time of the real census call on the caller's sample: tc_census for
// a single graph (the bucket kernels: thresholds, grids, LDS tiles, group
// size), the captured batched launch for several graphs (thresholds, the two
// persistent grids, the hub and batch LDS tiles).  Candidates that change how
// graphs are bucketed (thresholds, tri, hub tile) rebucket the sample graphs
// first.  Results are cached in a small JSON file keyed by device, CU count,
// mode and a coarse degree signature of the sample.  The tuning never changes
// any count; only which kernel runs each dyad and how many workgroups run.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tc_api_internal.h"

using namespace tc;

namespace {

double seconds_of(const std::chrono::steady_clock::time_point& a, const std::chrono::steady_clock::time_point& b) {
    return std::chrono::duration<double>(b - a).count();
}

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

std::string signature(tc_context ctx, const tc_graph* g, int32_t count) {
    double arcs = 0, d2 = 0, maxd = 0, n = 0;
    for (int32_t i = 0; i < count; ++i) {
        arcs += (double)g[i]->info.arcs_kept;
        d2 += (double)g[i]->info.sum_d2;
        maxd = std::max(maxd, (double)g[i]->info.max_degree);
        n += (double)g[i]->g.n;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|cu%d|%s|g%d|n%d|m%d|d2_%d|dmax%d", ctx->arch, ctx->cu_count,
                  count == 1 ? "single" : "batch", ilog2(count), ilog2(n), ilog2(arcs), ilog2(d2), ilog2(maxd));
    return buf;
}

std::string read_file(const char* path) {
    std::string s;
    FILE* f = std::fopen(path, "rb");
    if (!f) return s;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    std::fclose(f);
    return s;
}

// The tuning fields, in the order of tc_tuning, with their JSON names.
struct field_def {
    const char* name;
    uint32_t tc_tuning::*field;
};
const field_def kFields[] = {
    {"t0", &tc_tuning::t0}, {"t1", &tc_tuning::t1}, {"lane_blocks", &tc_tuning::lane_blocks},
    {"wave_blocks", &tc_tuning::wave_blocks}, {"group_blocks", &tc_tuning::group_blocks},
    {"batch_blocks", &tc_tuning::batch_blocks}, {"t_hub", &tc_tuning::t_hub}, {"hub_blocks", &tc_tuning::hub_blocks},
    {"tri", &tc_tuning::tri}, {"hub_tile", &tc_tuning::hub_tile}, {"wave_tile", &tc_tuning::wave_tile},
    {"group_tile", &tc_tuning::group_tile}, {"group_size", &tc_tuning::group_size},
    {"batch_tile", &tc_tuning::batch_tile},
};

// The cache is one JSON object: {"<key>": {"t0": .., "t1": .., ...}, ...}; an
// entry must name every field and pass the same checks as tc_set_tuning.
bool cache_lookup(const std::string& text, const std::string& key, tc_tuning* t) {
    std::string needle = "\"" + key + "\"";
    size_t p = text.find(needle);
    if (p == std::string::npos) return false;
    size_t open = text.find('{', p + needle.size());
    if (open == std::string::npos) return false;
    size_t close = text.find('}', open);
    if (close == std::string::npos) return false;
    const std::string body = text.substr(open, close - open);
    tc_tuning out{};
    for (const field_def& f : kFields) {
        const std::string name = std::string("\"") + f.name + "\":";
        size_t q = body.find(name);
        if (q == std::string::npos) return false;
        char* endp = nullptr;
        const char* start = body.c_str() + q + name.size();
        unsigned long v = std::strtoul(start, &endp, 10);
        if (endp == start || v > 0xffffffffUL) return false;
        out.*(f.field) = (uint32_t)v;
    }
    if (check_tuning(out) != TC_OK) return false;
    *t = out;
    return true;
}

void cache_store(const char* path, const std::string& key, const tc_tuning& t, double seconds) {
    std::string text = read_file(path);
    std::string entry = "\"" + key + "\": {";
    for (const field_def& f : kFields) entry += std::string("\"") + f.name + "\": " + std::to_string(t.*(f.field)) + ", ";
    char sec[64];
    std::snprintf(sec, sizeof(sec), "\"seconds\": %.6g}", seconds);
    entry += sec;
    size_t close = text.rfind('}');
    std::string out;
    if (text.empty() || close == std::string::npos || text.find('{') == std::string::npos) {
        out = std::string("{\n  ") + entry + "\n}\n";
    } else {
        std::string head = text.substr(0, close);
        while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
        bool empty_obj = !head.empty() && head.back() == '{';
        out = head + (empty_obj ? "\n  " : ",\n  ") + entry + "\n}\n";
    }
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fwrite(out.data(), 1, out.size(), f);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

int apply(tc_context ctx, const tc_graph* g, int32_t count, const tc_tuning& t) {
    int rc = tc_set_tuning(ctx, &t);
    for (int32_t i = 0; i < count && rc == TC_OK; ++i) rc = tc_graph_rebucket(ctx, g[i]);
    return rc;
}

// Best of `reps` timed calls after one warm-up call.
int measure(tc_context ctx, const tc_graph* g, int32_t count, int reps, double* best) {
    std::vector<uint64_t> out((size_t)count * 16);
    *best = 1e30;
    for (int r = 0; r <= reps; ++r) {
        auto a = std::chrono::steady_clock::now();
        int rc = count == 1 ? tc_census(ctx, g[0], out.data()) : tc_census_batch(ctx, g, count, out.data());
        auto b = std::chrono::steady_clock::now();
        if (rc != TC_OK) return rc;
        if (r > 0) *best = std::min(*best, seconds_of(a, b));
    }
    return TC_OK;
}

}  // namespace

extern "C" int tc_autotune(tc_context ctx, const tc_graph* sample, int32_t count, const char* cache_path,
                           tc_tuning* best_out) {
    if (!ctx || count <= 0 || !sample) return TC_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (int32_t i = 0; i < count; ++i)
            if (!sample[i] || !ctx->graphs.count(sample[i])) return TC_ERR_ARG;
    }
    const std::string key = signature(ctx, sample, count);
    tc_tuning best;
    int rc = tc_get_tuning(ctx, &best);
    if (rc != TC_OK) return rc;
    if (cache_path) {
        tc_tuning cached;
        if (cache_lookup(read_file(cache_path), key, &cached)) {
            rc = apply(ctx, sample, count, cached);
            if (rc == TC_OK && best_out) *best_out = cached;
            return rc;
        }
    }
    const uint32_t cu = (uint32_t)(ctx->cu_count > 0 ? ctx->cu_count : 256);
    const uint32_t kInf = 0xffffffffu;
    const bool single = count == 1;
    // The search space: every field the objective depends on, with the values
    // tried.  Thresholds, tri and the hub tile change how graphs are bucketed
    // (apply() rebuckets the sample); the rest only change launches.  A single
    // graph runs the per-bucket kernels (lane / wave / group / hub grids and
    // tiles); a batch runs the two persistent kernels (batch and hub grids,
    // batch and hub tiles).
    struct param {
        uint32_t tc_tuning::*field;
        std::vector<uint32_t> values;
        bool for_single, for_batch;
    };
    const param params[] = {
        {&tc_tuning::tri, {0, 1}, true, true},
        {&tc_tuning::t1, {256, 512, 1024, 2048, 4096, 8192, 16384, kInf}, true, true},
        {&tc_tuning::t0, {8, 16, 32, 64, 128, 256}, true, true},
        {&tc_tuning::t_hub, {32, 64, 128, 256, 512, 1024, 4096, kInf}, true, true},
        {&tc_tuning::lane_blocks, {cu * 4, cu * 8, cu * 16}, true, false},
        {&tc_tuning::wave_blocks, {cu * 5, cu * 10, cu * 20}, true, false},
        {&tc_tuning::group_blocks, {cu * 1, cu * 2, cu * 4}, true, false},
        {&tc_tuning::batch_blocks, {cu * 2, cu * 4, cu * 7, cu * 8}, false, true},
        {&tc_tuning::hub_blocks, {cu * 2, cu * 3, cu * 5, cu * 8}, true, true},
        {&tc_tuning::hub_tile, {512, 1024, 2048}, true, true},
        {&tc_tuning::wave_tile, {512, 1024, 2048}, true, false},
        {&tc_tuning::group_tile, {2048, 4096, 8192}, true, false},
        {&tc_tuning::group_size, {256, 512}, true, false},
        {&tc_tuning::batch_tile, {512, 1024, 2048}, false, true},
    };
    const int reps = 3;

    rc = apply(ctx, sample, count, best);
    double best_s = 0;
    if (rc == TC_OK) rc = measure(ctx, sample, count, reps, &best_s);
    for (int sweep = 0; sweep < 2 && rc == TC_OK; ++sweep) {
        for (const param& pr : params) {
            if (rc != TC_OK) break;
            if (single ? !pr.for_single : !pr.for_batch) continue;
            for (uint32_t v : pr.values) {
                tc_tuning c = best;
                if (c.*(pr.field) == v) continue;
                c.*(pr.field) = v;
                if (check_tuning(c) != TC_OK) continue;
                rc = apply(ctx, sample, count, c);
                double s = 0;
                if (rc == TC_OK) rc = measure(ctx, sample, count, reps, &s);
                if (rc != TC_OK) break;
                if (s < best_s * 0.98) {
                    best = c;
                    best_s = s;
                }
            }
        }
    }
    int rc2 = apply(ctx, sample, count, best);
    if (rc == TC_OK) rc = rc2;
    if (rc != TC_OK) return rc;
    if (cache_path) cache_store(cache_path, key, best, best_s);
    if (best_out) *best_out = best;
    return TC_OK;
}
