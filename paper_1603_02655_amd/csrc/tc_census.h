// Census kernel launch interface (definitions in tc_census.hip).
#pragma once
#include "tc_build.h"

namespace tc {

struct census_config {
    uint32_t lane_blocks = 2048;    // grid cap of the lane-per-dyad kernel
    uint32_t wave_blocks = 8192;    // resident one-wave workgroups of the wave kernel
    uint32_t group_blocks = 1024;   // resident workgroups of the group kernel
    uint32_t hub_blocks = 1024;     // resident workgroups of the hub kernel
    uint32_t side_blocks = 256;     // workgroups of the totals pass when it runs on the side stream
    uint32_t hub_tile = 1024;       // anchor entries per LDS tile, hub mode (512, 1024, 2048)
    uint32_t wave_tile = 1024;      // row entries staged per round, wave mode (512, 1024, 2048)
    uint32_t group_tile = 4096;     // row entries staged per round, group mode (2048, 4096, 8192)
    uint32_t group_size = 256;      // threads per workgroup, group mode (256, 512)
};

// Whether the kernels are built for these LDS tiles and group size.
bool tile_supported(uint32_t hub_tile, uint32_t wave_tile, uint32_t group_tile, uint32_t group_size,
                    uint32_t batch_tile);

// Per-bucket record slices [begin, end) into g.dyads or the edge records
// (merge buckets); the hub bucket runs its task groups [hub_g0, hub_g1),
// restricted to dyads with u in [u_lo, u_hi); the totals pass of the
// forward-list path covers the neighbour entries [totals_begin, totals_end).
struct census_slices {
    uint64_t begin[kBuckets];
    uint64_t end[kBuckets];
    uint32_t u_lo = 0, u_hi = 0xffffffffu;
    uint32_t hub_g0 = 0, hub_g1 = 0xffffffffu;
    uint64_t totals_begin = 0, totals_end = ~0ull;
};

// ---- batched launch over many graphs ----
struct graph_desc {
    const dyad_rec* dyads;       // dyad records
    const uint32_t* nbr;
    const uint64_t* tpre;
    uint64_t n;
    const hub_task* hub_tasks;
    const uint32_t* owner;
    const int64_t* row_ptr;
    uint64_t U;                  // neighbour entries
    const dyad_rec* edges;       // forward-list edge records (null without forward lists)
    const uint32_t* fwd;
    const hub_task* edge_tasks;
    const uint4* rinfo;          // per row: bounds and prefix counts at its end
    uint32_t hub_ntasks, hub_groups;   // tasks and task groups over the dyad records
    uint32_t tri_tasks, tri_groups;    // tasks and task groups over the edge records
    uint32_t hub_chunk, tri_chunk;     // records per hub task and per group, each view
};
// Item kinds: the mode (lane / wave / group / hub), with kItemTri when the item
// indexes the forward-list edge records; kItemTotals covers neighbour entries
// [begin, end) of the totals pass.
enum : uint32_t { kItemLane = 0, kItemWave = 1, kItemGroup = 2, kItemHub = 3, kItemTri = 4, kItemTotals = 8 };
struct work_item {
    uint32_t graph, kind, begin, end;   // records [begin, end) of graph `graph`'s record array;
                                        // hub items: task groups [begin, end) of the graph
};
constexpr uint32_t kBatchTotalsPerItem = 4096;   // neighbour entries per totals item
constexpr uint32_t kBatchLanePerItem = 256;   // one dyad per thread of a 256-thread workgroup
constexpr uint32_t kBatchWavePerItem = 16;    // four wavefronts, four dyads each

// Zeroes accs[0..acc_words) and 16 work counters, then runs two persistent
// kernels: the hub kernel (LDS tile of hub_tile anchor entries) over the hub
// items items[0..nums[0]) with hub_grid workgroups, and the batch kernel
// (wave-mode tile batch_tile, group-mode tile 4 x batch_tile) over the other
// items items[nums[0]..nums[1]) with `grid` workgroups (nums: 2 words of
// device memory).  hub_chunk: the largest records per hub task of the graphs
// (a launch of graphs with half-size tasks only runs the hub kernel instance
// with the smaller LDS).  hipErrorInvalidValue for a tile the kernels are not
// built for.
hipError_t batch_launch(const graph_desc* descs, const work_item* items, const uint32_t* nums,
                        unsigned long long* accs, uint64_t acc_words, unsigned int* counters, uint32_t grid,
                        uint32_t hub_grid, uint32_t hub_tile, uint32_t batch_tile, uint32_t hub_chunk, hipStream_t s);

// Copies the 16-class table into the constant table the batch kernel reads.
hipError_t census_upload_table();
// Zeroes acc (16 x u64) and counters (kBuckets x u32), then runs the bucket
// kernels over the given slices with `table` (64 bytes of device memory: the
// bin of every code, kNumClasses for codes that are not counted).  With `tri`
// the slices index the forward-list edge records (g.tri.edges) and a totals
// pass over every dyad record runs too: first on s, or, when `side` is given
// (with two events in `fork`) and the hub bucket streams more entries than the
// graph has, on `side` with side_blocks workgroups, followed there by the lane
// bucket, beside the other bucket kernels; s waits for it at the end.  ev, when not null, holds
// 2*kBuckets + 2 events: around each bucket's launch, then around the totals.
hipError_t census_launch(const device_graph& g, const census_slices& sl, bool tri, const uint8_t* table,
                         unsigned long long* acc, unsigned int* counters, const census_config& cfg, hipStream_t s,
                         hipEvent_t* ev, hipStream_t side = nullptr, hipEvent_t* fork = nullptr);

}  // namespace tc
