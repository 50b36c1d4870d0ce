/*
 * tc.h -- exact 16-class directed triad census on AMD MI355X (gfx950).
 *
 * The problem (Nagpal 2013, section "Triad Census Algorithm"): a strict digraph
 * G = [V, E], V = {0 .. n-1}, E a set of ordered pairs, goes in; the census
 * array with the frequency of each of the 16 isomorphic triad types comes out.
 * Classes are indexed 0..15 in the thesis's numbering (types 1..16):
 *   0 003, 1 012, 2 102, 3 021D, 4 021U, 5 021C, 6 111D, 7 111U,
 *   8 030T, 9 030C, 10 201, 11 120D, 12 120U, 13 120C, 14 210, 15 300.
 * The counts sum to C(n,3).  The census is computed by the subquadratic
 * dyad-based method (figure "Subquadratic Triad Census Algorithm"), one task per
 * canonical dyad (connected pair u < v), on the GPU; every count is exact.
 *
 * Conventions for every function:
 *   - returns TC_OK (0) or a negative TC_ERR_* code; no exception crosses the ABI;
 *   - on error, caller-visible outputs are left untouched;
 *   - pointers documented as host pointers must be host memory; device
 *     pointers (TC_BUILD_DEVICE_PTRS) must be allocated on the context's device;
 *   - a tc_context owns one HIP stream (its own or the caller's) on one device;
 *     calls on one context are serialised internally and may come from any thread.
 */
#ifndef TC_H
#define TC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_context_s* tc_context;
typedef struct tc_graph_s* tc_graph;
typedef uint64_t tc_ticket;

enum {
    TC_OK = 0,
    TC_ERR_ARG = -1,       /* bad argument: null pointer, id outside [0, n), strict-mode violation */
    TC_ERR_RANGE = -2,     /* n > 4,801,280 (C(n,3) would not fit uint64) or > 2^32 neighbour entries */
    TC_ERR_NOMEM = -3,     /* device or host allocation failed, or the job exceeds the HBM budget */
    TC_ERR_DEVICE = -4,    /* a HIP call failed */
    TC_ERR_BUSY = -5,      /* graph still referenced by pending tickets */
    TC_ERR_NOT_FOUND = -6, /* unknown ticket */
    TC_ERR_SHUTDOWN = -7   /* context is shutting down; ticket cancelled */
};

enum {
    TC_BUILD_DEFAULT = 0,     /* drop loops (u,u) and merge repeated arcs */
    TC_BUILD_STRICT = 1,      /* reject loops and repeated arcs with TC_ERR_ARG */
    TC_BUILD_DEVICE_PTRS = 2  /* src/dst are device pointers (e.g. torch tensors) */
};

enum { TC_NUM_CLASSES = 16, TC_NUM_BUCKETS = 4 };

/* Most graphs one tc_census_each_noalloc call takes. */
enum { TC_NOALLOC_MAX_GRAPHS = 256 };

/* What the build kept and how the canonical dyads were bucketed. */
typedef struct {
    int64_t arcs_in;              /* m as passed */
    int64_t arcs_kept;            /* distinct arcs after dropping loops and repeats */
    int64_t self_loops_dropped;
    int64_t duplicates_dropped;
    int64_t asym_dyads;           /* canonical dyads joined one way */
    int64_t mutual_dyads;         /* canonical dyads joined both ways */
    int64_t max_degree;           /* max |N(u)| (undirected) */
    uint64_t device_bytes;        /* HBM held by the resident graph */
    uint64_t sum_d2;              /* sum over u of |N(u)|^2 = sum over dyads of |N(u)|+|N(v)| */
    uint64_t bucket_dyads[TC_NUM_BUCKETS];  /* dyads in the lane / wave / group / hub buckets */
    uint64_t bucket_cost[TC_NUM_BUCKETS];   /* sum of |N(u)|+|N(v)| per bucket */
    uint64_t hub_tasks;           /* runs of hub dyads sharing their anchor */
    uint64_t hub_stream;          /* sum over hub dyads of the non-anchor degree (entries probed) */
    uint64_t hub_staged;          /* sum over hub tasks of the anchor degree (entries staged in LDS) */
    /* forward lists (built when the tuning has tri = 1; zero otherwise) */
    uint64_t fwd_entries;                      /* = canonical dyads */
    uint64_t tri_bucket_edges[TC_NUM_BUCKETS]; /* edge records per bucket (edges with an empty forward list omitted) */
    uint64_t tri_bucket_cost[TC_NUM_BUCKETS];  /* sum of |N+(x)|+|N+(y)| per bucket */
    uint64_t tri_tasks;           /* hub tasks over the forward lists */
    uint64_t tri_stream;          /* sum over hub edges of the non-anchor forward-list length */
    uint64_t tri_staged;          /* sum over those tasks of the anchor forward-list length */
    /* groups of consecutive hub tasks that one workgroup stages into a single LDS tile */
    uint64_t hub_groups;          /* over the hub dyads */
    uint64_t tri_groups;          /* over the hub edges of the forward lists */
    uint64_t hub_chunk;           /* records per hub task and per group, hub dyads (512) */
    uint64_t tri_chunk;           /* the same over the hub edges of the forward lists as tc_census runs
                                     them: 256 for hub buckets of 2^20 edges or more, else 512; such a
                                     bucket also holds a set of 512-record tasks over the same edges,
                                     which batched and served launches run.  tri_tasks, tri_staged and
                                     tri_groups describe the set tc_census runs */
} tc_graph_info;

/* Degree-bucket thresholds and launch sizes.  A dyad one of whose endpoints
 * has degree >= t_hub is a hub dyad: it is grouped with the other dyads of that
 * endpoint (its anchor, the endpoint of larger degree), whose row a workgroup
 * stages once in LDS while the other rows stream against it.  Any other dyad,
 * with key k = |N(u)| + |N(v)| - 2 (the thesis's uniform-distribution
 * workload estimate, figure "Canonical Dyad (uniform distr.)"), runs one lane
 * per dyad when k < t0, one wavefront per dyad when t0 <= k < t1, one
 * workgroup per dyad when k >= t1.  t_hub = 0xffffffff disables the hub mode.
 *
 * tri = 1 (graphs built or rebucketed while it is set) also builds forward
 * lists: N+(x), the neighbours that follow x in degree order ((|N|, id)
 * ascending).  tc_census, tc_census_each and tc_census64 then add the
 * intersection-free per-dyad terms in one pass over the dyads and find every
 * shared vertex of every dyad through the triangles of the graph, each
 * triangle once, as a shared vertex of the forward lists of its two first
 * vertices; the same thresholds bucket those edge records by
 * |N+(x)| + |N+(y)| (and t_hub by the longer forward list).  The counts are
 * identical either way.  The batched and the served modes take the same path
 * per graph (forward-list items for graphs that have forward lists while tri
 * is set, dyad-record items otherwise; requests that carry their arcs are built
 * without forward lists).  tc_census_range always uses the dyad records. */
typedef struct {
    uint32_t t0, t1;
    uint32_t lane_blocks;    /* grid cap, lane kernel (256-thread blocks) */
    uint32_t wave_blocks;    /* resident one-wave blocks, wave kernel */
    uint32_t group_blocks;   /* resident 256-thread blocks, group kernel */
    uint32_t batch_blocks;   /* resident 256-thread blocks, batched (persistent) kernel */
    uint32_t t_hub;
    uint32_t hub_blocks;     /* resident 256-thread blocks, hub kernel */
    uint32_t tri;            /* 1: whole-graph census through triangles of the forward lists */
    /* LDS tiles and group size (each among the kernel variants the library is built with) */
    uint32_t hub_tile;       /* anchor entries staged per LDS tile, hub mode: 512, 1024, 2048; graphs built
                                or rebucketed while it is set group their hub tasks for it */
    uint32_t wave_tile;      /* entries of each row staged per round, wave mode: 512, 1024, 2048 */
    uint32_t group_tile;     /* entries of each row staged per round, group mode: 2048, 4096, 8192 */
    uint32_t group_size;     /* threads per workgroup, group mode: 256, 512 */
    uint32_t batch_tile;     /* wave-mode tile of the batched kernel (its group-mode tile is 4x): 512, 1024, 2048 */
} tc_tuning;

/* Accumulated device time of the census kernels, per bucket (lane, wave,
 * group, hub), measured with HIP events recorded on the context's stream. */
typedef struct {
    double ms[TC_NUM_BUCKETS];
    uint64_t launches[TC_NUM_BUCKETS];
    uint64_t census_calls;
    double batch_ms;             /* replays of the captured batched launch */
    uint64_t batch_launches;
    double totals_ms;            /* per-dyad totals pass (tri = 1 only) */
    uint64_t totals_launches;
} tc_kernel_stats;

/* Serving statistics (tc_submit / tc_poll). */
typedef struct {
    uint64_t submitted, completed, rounds;
    uint64_t resident_graphs;
    uint64_t bytes_in_flight;
    double p50_ms, p99_ms;         /* submit -> completion latency of the admitted requests
                                      (histogram with 64 buckets per decade: within 3.7 %) */
    double mean_admission_ms;      /* submit -> admission wait */
    uint64_t failed_rounds;        /* rounds whose launch failed (their tickets carry the error) */
    uint64_t abandoned_rounds;     /* rounds that ran past the watchdog (tickets: TC_ERR_DEVICE) */
} tc_serve_stats;

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory of jobs admitted by tc_submit (0 = 90% of free memory).  hip_stream,
 * when not null, is a hipStream_t the context uses instead of its own (the
 * caller keeps it alive until tc_context_destroy).  *out receives the handle. */
int tc_context_create(int device, uint64_t hbm_budget_bytes, void* hip_stream, tc_context* out);

/* Stops the serving loop (pending tickets finish with TC_ERR_SHUTDOWN), frees
 * every graph still owned by the context and the context itself. */
int tc_context_destroy(tc_context ctx);

/* Builds a resident device graph from m arcs src[i] -> dst[i] (0-based int32
 * ids in [0, n)): the input G = [V, E] of section "Triad Census Algorithm",
 * read as a strict digraph with E a set.  On the device: the neighbour rows
 * N(u) with the direction of every joined pair (what the loop's IsEdge and
 * IsNeighbour ask), the canonical dyads u < v bucketed by |N(u)| + |N(v)| - 2
 * (figure "Canonical Dyad (uniform distr.)"), and, when the tuning has tri = 1,
 * the degree-ordered forward lists.  src/dst are read during the call only; host pointers unless
 * TC_BUILD_DEVICE_PTRS.  Loops and repeated arcs are dropped (counted in info)
 * unless TC_BUILD_STRICT, which rejects them.  Errors: TC_ERR_ARG (null pointer,
 * n < 0, m < 0, id out of range, strict violation), TC_ERR_RANGE (n too large),
 * TC_ERR_NOMEM, TC_ERR_DEVICE.  info may be null. */
int tc_build_graph(tc_context ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   uint32_t flags, tc_graph* out, tc_graph_info* info);

/* Copies the build information of g into *info. */
int tc_graph_get_info(tc_context ctx, tc_graph g, tc_graph_info* info);

/* Frees g.  TC_ERR_BUSY while tickets that use g are pending. */
int tc_graph_release(tc_context ctx, tc_graph g);

/* Synchronous census: counts[16] (host) receives the 16 class counts of g,
 * the census array of section "Triad Census Algorithm" (figure "Subquadratic
 * Triad Census Algorithm": per canonical dyad the n - |S| - 2 dyadic triads and
 * the triads of the third vertices it counts; the null class as C(n,3) minus
 * the rest).  Errors: TC_ERR_ARG (null or unknown handle), TC_ERR_DEVICE. */
int tc_census(tc_context ctx, tc_graph g, uint64_t counts[16]);

/* Labelled 64-class census: counts[64] (host) receives the histogram of the
 * raw 6-bit TriadCode (bit 1 u->v, 2 v->u, 4 u->w, 8 w->u, 16 v->w, 32 w->v)
 * that the census loop computes before the table folds codes into classes
 * (section "Triad Census Algorithm", TriadCode and TriadTable): each counted
 * triple is read in the roles the loop gives it (u < v the canonical dyad that
 * counts it, w the third vertex); the term n - |S| - 2 of a dyad goes to the
 * code of the (u, v) pair alone; counts[0] is C(n, 3) minus the rest.  The
 * histogram depends on the vertex ids (it is not an isomorphism invariant);
 * folding it through the 64 -> 16 table gives tc_census.  Runs the census
 * kernels three times (one pass per (u, v) dyad type).  Errors as tc_census. */
int tc_census64(tc_context ctx, tc_graph g, uint64_t counts[64]);

/* Partial census over the canonical dyads (u, v) with u in [u_begin, u_end):
 * the local census of one task queue (figure "Subquadratic Triad Census
 * Algorithm based on distributed task queues").  partial[0] (class 003) is 0;
 * summing the partials of a partition of [0, n) gives counts[1..15]. */
int tc_census_range(tc_context ctx, tc_graph g, int32_t u_begin, int32_t u_end, uint64_t partial[16]);

/* Shard `shard` of `nshards` of the census of g, on the path tc_census takes:
 * each bucket's records (dyads, or forward-list edge records), the hub task
 * groups and the neighbour entries of the per-dyad totals pass are cut into
 * nshards contiguous ranges of equal length and this call runs range `shard`
 * of each; every record, task group and entry falls in exactly one shard.
 * This is the unit of work a multi-GPU census would give one GPU (section
 * "Future work": distribute the canonical dyads).  partial[0] is 0; the other
 * counts are exact modulo 2^64 (a shard may hold only one side of a dyad's
 * terms, so a single partial can wrap), and their sum over the nshards shards,
 * modulo 2^64, is counts[1..15] of tc_census; 003 follows as C(n,3) minus the
 * rest.  Errors: TC_ERR_ARG (null or unknown handle, nshards < 1, shard
 * outside [0, nshards)), TC_ERR_DEVICE. */
int tc_census_shard(tc_context ctx, tc_graph g, int32_t shard, int32_t nshards, uint64_t partial[16]);

/* Census of `count` resident graphs in one persistent launch, replayed from a
 * captured HIP graph when the same set of graphs is passed again.
 * counts (host) receives count*16 values, graph i at counts[16*i]. */
int tc_census_batch(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts);

/* Same result as tc_census_batch, but one tc_census-style launch sequence per
 * graph (the per-graph baseline of the batched mode). */
int tc_census_each(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same counts as tc_census_each, without any allocation.  The kernels'
 * scratch (work counters and one block of 16 accumulators per graph) lives in
 * a fixed device array of the library, 33,024 bytes per GPU, held until the
 * process ends; the read-back goes through pinned host memory the context
 * allocated when it was created.  The launches of all graphs are queued back
 * to back and the counts read once at the end.
 *   graphs: count resident graphs of ctx (the same graph may repeat);
 *   counts (host): receives count*16 values, graph i at counts[16*i].
 * Errors: TC_ERR_ARG (null or unknown handle, count < 0), TC_ERR_RANGE
 * (count > TC_NOALLOC_MAX_GRAPHS), TC_ERR_DEVICE.  Every context on one GPU
 * shares that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (from two contexts, or from two threads) race and may
 * return wrong counts.  Calls on one context are serialised.  Kernel timing
 * (tc_set_timing) is not recorded by this call. */
int tc_census_each_noalloc(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts);

/* Queues a census of g for the serving loop and returns at once.  The loop
 * admits jobs while their device footprint fits the budget, runs all admitted
 * jobs of a round in one batched launch on a free stream, and overlaps rounds.
 * g must stay alive until the ticket is polled done (release returns BUSY). */
int tc_submit(tc_context ctx, tc_graph g, tc_ticket* out);

/* A request that carries its graph: n and m host arcs src[i] -> dst[i], copied
 * during the call.  The serving loop admits it when the build footprint fits
 * the budget, builds the graph on a serving stream, censuses it in a round and
 * frees it; a round with graphs to build holds no resident graph's request and
 * is prepared on a thread of the loop's own, so rounds of resident graphs keep
 * starting meanwhile, and at most two of the loop's four rounds in flight
 * build at once (a request to build waits at the front of the queue while the
 * resident requests behind it run).  flags may hold
 * TC_BUILD_STRICT.  Argument errors are returned at once; build errors (bad
 * ids, strict violations) by tc_poll. */
int tc_submit_arcs(tc_context ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst, uint32_t flags,
                   tc_ticket* out);

/* Non-blocking.  When the ticket has finished, *done = 1 and the ticket is
 * retired: the return value is its status (counts[16] filled when TC_OK;
 * TC_ERR_NOMEM if its footprint exceeds the whole budget, TC_ERR_SHUTDOWN if
 * the loop stopped before running it).  Otherwise *done = 0 and TC_OK is
 * returned (TC_ERR_SHUTDOWN once the loop is stopping).  TC_ERR_NOT_FOUND for
 * an unknown or already retired ticket. */
int tc_poll(tc_context ctx, tc_ticket ticket, uint64_t counts[16], int* done);

/* Stops the serving loop: running rounds finish, queued tickets end with
 * TC_ERR_SHUTDOWN, later submissions fail with TC_ERR_SHUTDOWN.  The context
 * stays usable for synchronous calls. */
int tc_serve_stop(tc_context ctx);

/* Watchdog of the serving loop: a round still running ms milliseconds after
 * its device work was issued (for a round with graphs to build: after the
 * builds) fails its tickets with TC_ERR_DEVICE, and its stream slot is not
 * used again (when every slot is lost, queued and new tickets fail with
 * TC_ERR_DEVICE).  Default 60000.  TC_ERR_ARG unless ms > 0. */
int tc_serve_set_watchdog_ms(tc_context ctx, double ms);

/* Serving statistics since the context was created (or last reset). */
int tc_serve_get_stats(tc_context ctx, tc_serve_stats* out);
int tc_serve_reset_stats(tc_context ctx);

/* Tuning: thresholds apply to graphs built afterwards and to graphs passed to
 * tc_graph_rebucket; launch sizes apply to the next census call. */
int tc_set_tuning(tc_context ctx, const tc_tuning* t);
int tc_get_tuning(tc_context ctx, tc_tuning* t);
int tc_graph_rebucket(tc_context ctx, tc_graph g);

/* Searches thresholds and launch sizes on the given sample graphs by
 * coordinate descent (objective: wall time of tc_census for one sample graph,
 * of tc_census_batch for several), applies the best to the context, rebuckets
 * the sample graphs and writes it to *best (may be null).  cache_path, when not
 * null, is a JSON file keyed by device name, CU count and the sample's degree
 * signature: a hit skips the search; a search adds its result.  Counts never
 * depend on the tuning. */
int tc_autotune(tc_context ctx, const tc_graph* sample, int32_t count, const char* cache_path, tc_tuning* best);

/* Kernel timing: when enabled, every census records HIP events around each
 * bucket kernel on the context stream and accumulates their durations. */
int tc_set_timing(tc_context ctx, int enable);
int tc_get_kernel_stats(tc_context ctx, tc_kernel_stats* out);
int tc_reset_kernel_stats(tc_context ctx);

/* The library's 64 -> 16 class table (host only, needs no device). */
int tc_class_table(uint8_t out[64]);

/* Static string for a status code. */
const char* tc_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
