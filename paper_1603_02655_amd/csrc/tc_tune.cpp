// Autotuner for the degree-bucket thresholds and launch sizes.
//
// Coordinate descent over small candidate grids, two sweeps.  The objective is
// the wall time of the real census call on the caller's sample: tc_census for
// a single graph (all three bucket kernels and their grids matter), the
// captured batched launch for several graphs (thresholds and the persistent
// grid matter).  Candidates that change thresholds rebucket the sample graphs
// first.  Results are cached in a small JSON file keyed by device, CU count,
// mode and a coarse degree signature of the sample.  The tuning never changes
// any count; only which kernel runs each dyad and how many workgroups run.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

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

// The cache is one JSON object: {"<key>": {"t0": .., "t1": .., ...}, ...}
bool cache_lookup(const std::string& text, const std::string& key, tc_tuning* t) {
    std::string needle = "\"" + key + "\"";
    size_t p = text.find(needle);
    if (p == std::string::npos) return false;
    p = text.find('{', p + needle.size());
    if (p == std::string::npos) return false;
    unsigned a[6];
    unsigned b[3];
    int got = std::sscanf(text.c_str() + p,
                          "{\"t0\": %u, \"t1\": %u, \"lane_blocks\": %u, \"wave_blocks\": %u, \"group_blocks\": %u, "
                          "\"batch_blocks\": %u, \"t_hub\": %u, \"hub_blocks\": %u, \"tri\": %u",
                          &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &b[0], &b[1], &b[2]);
    if (got != 9) return false;
    *t = tc_tuning{a[0], a[1], a[2], a[3], a[4], a[5], b[0], b[1], b[2]};
    return t->t0 <= t->t1 && a[2] && a[3] && a[4] && a[5] && b[1] && b[2] <= 1;
}

void cache_store(const char* path, const std::string& key, const tc_tuning& t, double seconds) {
    std::string text = read_file(path);
    char entry[512];
    std::snprintf(entry, sizeof(entry),
                  "\"%s\": {\"t0\": %u, \"t1\": %u, \"lane_blocks\": %u, \"wave_blocks\": %u, \"group_blocks\": %u, "
                  "\"batch_blocks\": %u, \"t_hub\": %u, \"hub_blocks\": %u, \"tri\": %u, \"seconds\": %.6g}",
                  key.c_str(), t.t0, t.t1, t.lane_blocks, t.wave_blocks, t.group_blocks, t.batch_blocks, t.t_hub,
                  t.hub_blocks, t.tri, seconds);
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
    const std::vector<uint32_t> t0s = {8, 16, 32, 64, 128, 256};
    const std::vector<uint32_t> t1s = {256, 512, 1024, 2048, 4096, 8192, 16384, kInf};
    const std::vector<uint32_t> lane = {cu * 4, cu * 8, cu * 16};
    const std::vector<uint32_t> wave = {cu * 5, cu * 10, cu * 20};
    const std::vector<uint32_t> group = {cu * 1, cu * 2, cu * 4};
    const std::vector<uint32_t> batch = {cu * 2, cu * 3, cu * 4, cu * 6};
    const std::vector<uint32_t> hubt = {32, 64, 128, 256, 512, 1024, 4096, kInf};
    const std::vector<uint32_t> hubb = {cu * 2, cu * 3, cu * 5, cu * 8};
    const std::vector<uint32_t> tris = {0, 1};
    const int reps = 3;

    rc = apply(ctx, sample, count, best);
    double best_s = 0;
    if (rc == TC_OK) rc = measure(ctx, sample, count, reps, &best_s);
    for (int sweep = 0; sweep < 2 && rc == TC_OK; ++sweep) {
        for (int param = -1; param < 8 && rc == TC_OK; ++param) {
            const std::vector<uint32_t>* cands = nullptr;
            if (param == -1 && count == 1) cands = &tris;   // the batched kernel has no forward-list path
            if (param == 0) cands = &t1s;
            if (param == 1) cands = &t0s;
            if (param == 6) cands = &hubt;
            if (param == 7 && count == 1) cands = &hubb;
            if (count == 1) {
                if (param == 2) cands = &lane;
                if (param == 3) cands = &wave;
                if (param == 4) cands = &group;
            } else if (param == 5) {
                cands = &batch;
            }
            if (!cands) continue;
            for (uint32_t v : *cands) {
                tc_tuning c = best;
                uint32_t* field = param == -1 ? &c.tri : param == 0 ? &c.t1 : param == 1 ? &c.t0 : param == 2 ? &c.lane_blocks
                                : param == 3 ? &c.wave_blocks : param == 4 ? &c.group_blocks
                                : param == 5 ? &c.batch_blocks : param == 6 ? &c.t_hub : &c.hub_blocks;
                if (*field == v) continue;
                *field = v;
                if (c.t0 > c.t1) continue;
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
