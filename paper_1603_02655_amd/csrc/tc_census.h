// Census kernel launch interface (definitions in tc_census.hip).
#pragma once
#include "tc_build.h"

namespace tc {

struct census_config {
    uint32_t lane_blocks = 2048;    // grid cap of the lane-per-dyad kernel
    uint32_t wave_blocks = 8192;    // resident one-wave workgroups of the wave kernel
    uint32_t group_blocks = 1024;   // resident workgroups of the group kernel
};

// Per-bucket dyad slices [begin, end) into g.dyads.
struct census_slices {
    uint64_t begin[kBuckets];
    uint64_t end[kBuckets];
};

hipError_t census_upload_table();
// Zeroes acc (16 x u64) and counters (kBuckets x u32), then runs the three
// bucket kernels over the given slices.  ev, when not null, holds 2*kBuckets
// events recorded around each bucket's launch.
hipError_t census_launch(const device_graph& g, const census_slices& sl, unsigned long long* acc,
                         unsigned int* counters, const census_config& cfg, hipStream_t s, hipEvent_t* ev);

}  // namespace tc
