// Host-side state behind the C ABI handles.
#pragma once
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../../include/tc.h"
#include "tc_census.h"

struct tc_graph_s {
    tc::device_graph g;
    tc_graph_info info{};
    std::atomic<int> pending{0};     // tickets in flight that use this graph
};

namespace tc {
struct batch_plan;     // tc_batch.hip
struct serve_state;    // tc_serve.cpp
}

struct tc_context_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    int cu_count = 0;
    char arch[64] = {0};
    std::mutex mu;                      // serialises work on `stream` and the buffers below
    std::mutex tuning_mu;               // held (inside mu) while `tuning` is written; lets the
                                        // serving thread copy it without waiting for mu
    unsigned long long* acc = nullptr;  // 16 accumulators (device)
    unsigned int* counters = nullptr;   // work counters (device)
    unsigned long long* host_raw = nullptr;  // pinned copy of acc
    uint8_t* tables = nullptr;          // 4 x 64 bin indices (device): the 16-class table,
                                        // then the labelled census's pass tables for f_uv = 1, 2, 3
    hipEvent_t ev[2 * tc::kBuckets + 2] = {};
    hipStream_t side = nullptr;         // runs the totals pass beside the bucket kernels
    hipEvent_t fork[2] = {};            // side stream start / end
    bool timing = false;
    tc_kernel_stats kstats{};
    tc_tuning tuning{};
    std::set<tc_graph> graphs;
    void* scratch = nullptr;            // this device's copy of the no-allocation scratch array
    unsigned long long* host_many = nullptr;  // pinned read-back area of tc_census_each_noalloc
    tc::batch_plan* batch = nullptr;    // cached batched launch (captured hipGraph), owned
    tc::serve_state* serve = nullptr;   // serving loop, started on first submit, owned
    double watchdog_ms = 0;             // serving watchdog (0: the default)
};

namespace tc {

int status_from_hip(hipError_t e);
void finalize_counts(int64_t n, const unsigned long long* raw, uint64_t out[16]);
census_slices full_slices(const device_graph& g, bool tri = false);
census_config config_of(const tc_tuning& t);
void fill_info(const tc_graph_s* g, tc_graph_info* info);
// Runs the bucket kernels over `sl` with table `table` (0: 16 classes; 1..3:
// labelled census pass for f_uv = table) and copies the 16 raw sums to host.
// With `tri` the slices index the forward-list edge records.
int run_census_locked(tc_context_s* ctx, const device_graph& g, const census_slices& sl, unsigned long long raw[16],
                      int table = 0, bool tri = false);
// The whole census of g: through the forward lists when the tuning asks for
// them and g has them, else through the dyad records.
int run_full_locked(tc_context_s* ctx, const device_graph& g, unsigned long long raw[16], int table = 0);
// Builds a device graph from host (or, with TC_BUILD_DEVICE_PTRS, device) arcs
// on `stream`; returns a TC_* status and fills the build part of *info.
int build_into(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, uint32_t flags, const bucket_params& bp,
               hipStream_t stream, device_graph* out, tc_graph_info* info);
bucket_params params_of(const tc_tuning& t);
// A copy of ctx->tuning taken under tuning_mu (for threads that do not hold mu).
tc_tuning tuning_snapshot(tc_context_s* ctx);
// TC_OK when every field of t is in range (thresholds ordered, grids non-zero,
// tiles and group size among the built kernel variants).
int check_tuning(const tc_tuning& t);

inline tc_tuning default_tuning(int cu_count) {
    tc_tuning t;
    int cu = cu_count > 0 ? cu_count : 256;
    t.t0 = 64;      // lane mode for k < 64
    t.t1 = 4096;    // wave mode for 64 <= k < 4096, group mode above
    t.t_hub = 32;   // records with a row of length >= 32: hub mode
    t.lane_blocks = (uint32_t)cu * 8;
    t.wave_blocks = (uint32_t)cu * 10;
    t.group_blocks = (uint32_t)cu * 2;
    t.batch_blocks = (uint32_t)cu * 7;   // seven waves per SIMD: the batched kernel waits on memory
    t.hub_blocks = (uint32_t)cu * 8;
    t.tri = 1;      // whole-graph census through the triangles of the forward lists
    t.hub_tile = 1024;
    t.wave_tile = 1024;
    t.group_tile = 4096;
    t.group_size = 256;
    t.batch_tile = 512;
    return t;
}

// batched mode (tc_batch.hip)
graph_desc describe(const device_graph& g);
void append_items(const device_graph& g, uint32_t gi, bool tri, std::vector<work_item>& hub,
                  std::vector<work_item>& out);
void batch_release_all(tc_context_s* ctx);
void batch_forget_graph_locked(tc_context_s* ctx, tc_graph g);

// serving loop (tc_serve.cpp)
void serve_stop(tc_context_s* ctx);
void serve_shutdown(tc_context_s* ctx);

}  // namespace tc
