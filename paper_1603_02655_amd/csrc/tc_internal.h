// Internal declarations shared by the HIP translation units of libtc.
//
// Device graph layout (one graph):
//   row_ptr[n+1]  int64   offsets into nbr (undirected neighbour rows)
//   nbr[U]        uint32  entry (w << 2) | f, rows sorted by w; f bit0 = owner->w
//                         is an arc, bit1 = w->owner is an arc (U = 2 * dyads)
//   tpre[U+1]     uint64  exclusive prefix over all entries of (f & 1) in the low
//                         32 bits and (f >> 1) in the high 32 bits; a range
//                         [a, b) of a row holds lo(tpre[b]-tpre[a]) arcs leaving
//                         the owner and hi(...) arcs entering it
//   dyads[p]      dyad_rec one task per canonical dyad (u < v joined either way),
//                         partitioned into degree buckets; u-major inside the
//                         merge buckets, anchor-major inside the hub bucket
//   hub_tasks[]   hub_task runs of at most kHubChunk hub-bucket records that
//                         share their anchor (the endpoint of larger degree),
//                         and the first task of each group of tasks
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

constexpr int kNumClasses = 16;
constexpr int kBuckets = 4;            // lane, wave, group (canonical-order merges), hub (anchor-major)
constexpr int kBucketHub = 3;
constexpr int kMaxN = 4801280;         // largest n with C(n,3) < 2^64

// One canonical dyad (u, v), u < v.  All indices are global positions in nbr.
struct __attribute__((aligned(16))) dyad_rec {
    uint32_t bu, eu;   // row of u: [bu, eu)
    uint32_t bv, ev;   // row of v: [bv, ev)
    uint32_t iv;       // position of v inside row u
    uint32_t iu;       // position of u inside row v
    uint32_t u;        // vertex u
    uint32_t vf;       // (v << 2) | f_uv, f_uv = IsEdge(u,v) + 2 IsEdge(v,u)
};
static_assert(sizeof(dyad_rec) == 32, "dyad record is two 16-byte loads");

// A run of hub-bucket records [begin, end) whose dyads all contain `anchor`.
// Consecutive tasks form groups that a workgroup runs with one LDS tile;
// `group` of task g holds the first task of group g (g below the group count).
struct hub_task {
    uint32_t begin, end, anchor, group;
};
constexpr uint32_t kHubChunk = 512;           // records per hub task and per group of tasks (hub kernels' LDS)
// A forward-list hub bucket of at least this many records also gets tasks and
// groups of kHubChunk / 2 records, which a single-graph census runs on the hub
// kernel instance with the smaller LDS (R-MAT 2^20: the hub kernel takes 7 %
// less time); batched launches keep the kHubChunk tasks (fewer, larger items).
constexpr uint64_t kHubSplitRecords = 1ull << 20;
constexpr uint32_t kHubTileEntries = 1024;    // anchor-row entries staged per LDS tile (default)
constexpr uint32_t kHubGroupTasks = 8;        // consecutive hub tasks a workgroup takes at a time
constexpr uint64_t kRowPad = 8;               // entries allocated past the end of a row array (block reads)

// Bucket thresholds.  Dyads with max(|N(u)|, |N(v)|) >= t_hub go to the hub
// bucket (anchored at the larger-degree endpoint, ties to the larger id); the
// others by k = |N(u)| + |N(v)| - 2: lane if k < t0, wave if k < t1, else group.
struct bucket_params {
    uint32_t t0, t1, t_hub;
    uint32_t tri;        // also build the degree-ordered forward lists and their edge records
    uint32_t hub_tile;   // anchor entries per LDS tile of the hub mode: hub tasks are grouped for it
};

// ---------------------------------------------------------------------------
// 64 -> 16 class table, derived here from the naming rules of the 16 classes
// (MAN digits: mutual / asymmetric / null dyads; D out-star, U in-star,
// C cyclic or chain, T transitive).  The code bits follow TriadCode:
// 1 u->v, 2 v->u, 4 u->w, 8 w->u, 16 v->w, 32 w->v.
// ---------------------------------------------------------------------------
constexpr int arc_bit(int x, int y) {
    return (x == 0 && y == 1) ? 1 : (x == 1 && y == 0) ? 2 : (x == 0 && y == 2) ? 4
         : (x == 2 && y == 0) ? 8 : (x == 1 && y == 2) ? 16 : (x == 2 && y == 1) ? 32 : 0;
}
constexpr bool has_arc(int code, int x, int y) { return (code & arc_bit(x, y)) != 0; }

constexpr int classify_code(int code) {
    int mutual = 0, asym = 0;
    const int px[3] = {0, 0, 1}, py[3] = {1, 2, 2};
    int mx = -1, my = -1;       // the mutual pair (when exactly one)
    for (int k = 0; k < 3; ++k) {
        bool a = has_arc(code, px[k], py[k]), b = has_arc(code, py[k], px[k]);
        if (a && b) { ++mutual; mx = px[k]; my = py[k]; }
        else if (a || b) ++asym;
    }
    int outd[3] = {0, 0, 0}, ind[3] = {0, 0, 0};
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y)
            if (x != y && has_arc(code, x, y)) { ++outd[x]; ++ind[y]; }
    // indices: 0 003, 1 012, 2 102, 3 021D, 4 021U, 5 021C, 6 111D, 7 111U,
    //          8 030T, 9 030C, 10 201, 11 120D, 12 120U, 13 120C, 14 210, 15 300
    if (mutual == 0 && asym == 0) return 0;
    if (mutual == 0 && asym == 1) return 1;
    if (mutual == 1 && asym == 0) return 2;
    if (mutual == 0 && asym == 2) {
        for (int x = 0; x < 3; ++x) if (outd[x] == 2) return 3;   // out-star
        for (int x = 0; x < 3; ++x) if (ind[x] == 2) return 4;    // in-star
        return 5;                                                  // chain
    }
    if (mutual == 1 && asym == 1) {
        // the asymmetric arc enters the mutual dyad (D) or leaves it (U)
        for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y)
                if (x != y && has_arc(code, x, y) && !has_arc(code, y, x))
                    return (y == mx || y == my) ? 6 : 7;
        return -1;
    }
    if (mutual == 0 && asym == 3)
        return (outd[0] == 1 && outd[1] == 1 && outd[2] == 1) ? 9 : 8;
    if (mutual == 2 && asym == 0) return 10;
    if (mutual == 1 && asym == 2) {
        int r = 3 - mx - my;                   // the vertex outside the mutual dyad
        int r_out = (has_arc(code, r, mx) ? 1 : 0) + (has_arc(code, r, my) ? 1 : 0);
        return r_out == 2 ? 11 : r_out == 0 ? 12 : 13;
    }
    if (mutual == 2 && asym == 1) return 14;
    if (mutual == 3) return 15;
    return -1;
}

struct class_table { uint8_t t[64]; };
constexpr class_table make_table() {
    class_table ct{};
    for (int c = 0; c < 64; ++c) ct.t[c] = (uint8_t)classify_code(c);
    return ct;
}
constexpr class_table kTable = make_table();
static_assert(kTable.t[0] == 0 && kTable.t[63] == 15, "table endpoints");

// ---------------------------------------------------------------------------
// kernels launched from the host side (definitions in tc_build.hip / tc_census.hip)
// ---------------------------------------------------------------------------
struct census_args {
    const dyad_rec* dyads;    // bucket slice (the whole record array for the hub kernel)
    uint32_t count;           // dyads in the slice
    const uint32_t* nbr;
    const uint64_t* tpre;
    uint64_t n;               // vertices of the graph
    unsigned long long* acc;  // 16 accumulators of the graph
    uint32_t u_lo, u_hi;      // hub kernel: only dyads with u in [u_lo, u_hi)
    const uint8_t* table;     // 64 bin indices (device memory), one per code
    uint32_t hub_chunk;       // hub kernel: records per task and per group of tasks
};

// device scan / sort helpers (tc_build.hip)
hipError_t scan_exclusive_u64(const uint64_t* in, uint64_t* out, uint64_t count, uint64_t* total_dev,
                              hipStream_t s);
}  // namespace tc
