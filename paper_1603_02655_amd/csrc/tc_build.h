// Device graph storage and the build entry points (definitions in tc_build.hip).
#pragma once
#include "tc_internal.h"

namespace tc {

constexpr int kCounters = 16;

// Bucketed task records over one adjacency view: the canonical dyads of the
// neighbour CSR, or the oriented edges of the forward lists.
struct rec_set {
    dyad_rec* recs = nullptr;
    hub_task* tasks = nullptr;
    uint32_t n_tasks = 0;
    uint32_t n_groups = 0;                    // groups of consecutive tasks (hub_task::group)
    uint32_t chunk = kHubChunk;               // records per task and per group
    // A second set of tasks and groups of kHubChunk / 2 records over the same
    // records (forward-list hub buckets of kHubSplitRecords records or more):
    // the set a single-graph census runs, on the hub kernel with the smaller LDS.
    hub_task* fine_tasks = nullptr;
    uint32_t fine_n_tasks = 0;
    uint32_t fine_n_groups = 0;
    uint64_t off[kBuckets + 1] = {0, 0, 0, 0, 0};
    uint64_t cost[kBuckets] = {0, 0, 0, 0};   // sum of the two row lengths per bucket
    uint64_t stream = 0;                      // hub: sum of the non-anchor row lengths
    uint64_t staged = 0;                      // hub: sum over tasks of the anchor row length
    uint64_t fine_staged = 0;                 // ... over the tasks of the second set
};

// Degree order: x precedes y when (|N(x)|, x) < (|N(y)|, y).  The forward list
// N+(x) holds the neighbours that follow x, sorted by id with the direction
// bits relative to x; every joined pair appears in exactly one forward list.
// A triangle {x, y, z} in degree order is found exactly once, as the shared
// vertex z of the forward lists of x and y.  The edge records (recs of `edges`)
// use the dyad_rec layout with forward-list bounds: bu..ev bound N+(u), N+(v)
// for u < v by id, vf = (v << 2) | f_uv, iv = iu = 0; edges whose two forward
// lists cannot share a vertex (one is empty) are left out.
struct forward_lists {
    uint32_t* fwd = nullptr;
    uint32_t* fwd_owner = nullptr;
    int64_t* fwd_ptr = nullptr;   // n + 1
    uint64_t entries = 0;         // = canonical dyads
    rec_set edges;
};

struct device_graph {
    int32_t n = 0;
    uint64_t U = 0;            // neighbour entries (2 x canonical dyads)
    uint64_t p = 0;            // canonical dyads
    uint64_t mutual = 0;       // mutual canonical dyads
    int64_t* row_ptr = nullptr;
    uint32_t* nbr = nullptr;
    uint32_t* owner = nullptr; // row of each entry (used to rebuild the buckets)
    uint64_t* tpre = nullptr;
    uint4* rinfo = nullptr;    // per row x: row_ptr[x], row_ptr[x+1] and the prefix counts tpre[row_ptr[x+1]]
    dyad_rec* dyads = nullptr;
    hub_task* hub_tasks = nullptr;
    uint32_t n_hub_tasks = 0;
    uint32_t n_hub_groups = 0;
    uint32_t hub_chunk = kHubChunk;  // records per hub task and per group
    uint64_t bucket_off[kBuckets + 1] = {0, 0, 0, 0, 0};
    uint64_t bucket_cost[kBuckets] = {0, 0, 0, 0};   // sum of |N(u)|+|N(v)| per bucket
    uint64_t hub_stream = 0;   // sum over hub dyads of the non-anchor degree (entries probed)
    uint64_t hub_staged = 0;   // sum over hub tasks of the anchor degree (entries staged)
    bucket_params bp{0, 0, 0, 0, kHubTileEntries};
    forward_lists tri;         // built when bp.tri
};

struct build_status {
    bool ok = false;
    bool too_large = false;
    hipError_t hip = hipSuccess;
    int64_t bad_ids = 0, self_loops = 0, duplicates = 0, arcs_kept = 0, max_degree = 0;
    uint64_t sum_d2 = 0;
};

build_status build_graph_device(int32_t n, int64_t m, const int32_t* src_dev, const int32_t* dst_dev,
                                const bucket_params& bp, hipStream_t s, device_graph* g);
hipError_t bucket_dyads(device_graph* g, const bucket_params& bp, hipStream_t s);
void free_device_graph(device_graph* g);
uint64_t device_graph_bytes(const device_graph& g);
hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);

}  // namespace tc
