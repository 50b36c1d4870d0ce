// Device graph storage and the build entry points (definitions in tc_build.hip).
#pragma once
#include "tc_internal.h"

namespace tc {

constexpr int kCounters = 16;

struct device_graph {
    int32_t n = 0;
    uint64_t U = 0;            // neighbour entries (2 x canonical dyads)
    uint64_t p = 0;            // canonical dyads
    uint64_t mutual = 0;       // mutual canonical dyads
    int64_t* row_ptr = nullptr;
    uint32_t* nbr = nullptr;
    uint32_t* owner = nullptr; // row of each entry (used to rebuild the buckets)
    uint64_t* tpre = nullptr;
    dyad_rec* dyads = nullptr;
    uint64_t bucket_off[kBuckets + 1] = {0, 0, 0, 0};
    uint64_t bucket_cost[kBuckets] = {0, 0, 0};   // sum of |N(u)|+|N(v)| per bucket
    uint32_t t0 = 0, t1 = 0;
};

struct build_status {
    bool ok = false;
    bool too_large = false;
    hipError_t hip = hipSuccess;
    int64_t bad_ids = 0, self_loops = 0, duplicates = 0, arcs_kept = 0, max_degree = 0;
    uint64_t sum_d2 = 0;
};

build_status build_graph_device(int32_t n, int64_t m, const int32_t* src_dev, const int32_t* dst_dev,
                                uint32_t t0, uint32_t t1, hipStream_t s, device_graph* g);
hipError_t bucket_dyads(device_graph* g, uint32_t t0, uint32_t t1, hipStream_t s);
void free_device_graph(device_graph* g);
uint64_t device_graph_bytes(const device_graph& g);
hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);

}  // namespace tc
