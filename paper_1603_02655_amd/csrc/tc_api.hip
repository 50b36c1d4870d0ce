// C ABI of libtc: contexts, resident graphs, single-graph and range census.
// Batched, served and autotuned modes live in tc_batch.hip / tc_serve.cpp.
#include "tc_api_internal.h"

#include <cstring>
#include <new>

using namespace tc;

namespace tc {

int status_from_hip(hipError_t e) {
    if (e == hipSuccess) return TC_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return TC_ERR_NOMEM;
    return TC_ERR_DEVICE;
}

void finalize_counts(int64_t n, const unsigned long long* raw, uint64_t out[16]) {
    typedef unsigned __int128 u128;
    u128 total = n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
    u128 sum = 0;
    for (int k = 1; k < kNumClasses; ++k) {
        out[k] = raw[k];
        sum += raw[k];
    }
    out[0] = (uint64_t)(total - sum);
}

census_slices full_slices(const device_graph& g, bool tri) {
    census_slices sl;
    for (int b = 0; b < kBuckets; ++b) {
        sl.begin[b] = tri ? g.tri.edges.off[b] : g.bucket_off[b];
        sl.end[b] = tri ? g.tri.edges.off[b + 1] : g.bucket_off[b + 1];
    }
    return sl;
}

census_config config_of(const tc_tuning& t) {
    census_config c;
    c.lane_blocks = t.lane_blocks;
    c.wave_blocks = t.wave_blocks;
    c.group_blocks = t.group_blocks;
    c.hub_blocks = t.hub_blocks;
    c.hub_tile = t.hub_tile;
    c.wave_tile = t.wave_tile;
    c.group_tile = t.group_tile;
    c.group_size = t.group_size;
    return c;
}

bucket_params params_of(const tc_tuning& t) { return bucket_params{t.t0, t.t1, t.t_hub, t.tri, t.hub_tile}; }

tc_tuning tuning_snapshot(tc_context_s* ctx) {
    std::lock_guard<std::mutex> lk(ctx->tuning_mu);
    return ctx->tuning;
}

int check_tuning(const tc_tuning& t) {
    if (t.t0 > t.t1 || t.lane_blocks == 0 || t.wave_blocks == 0 || t.group_blocks == 0 || t.batch_blocks == 0 ||
        t.hub_blocks == 0 || t.tri > 1)
        return TC_ERR_ARG;
    if (!tile_supported(t.hub_tile, t.wave_tile, t.group_tile, t.group_size, t.batch_tile)) return TC_ERR_ARG;
    return TC_OK;
}

void fill_info(const tc_graph_s* g, tc_graph_info* info) {
    *info = g->info;
    info->device_bytes = device_graph_bytes(g->g);
    info->asym_dyads = (int64_t)(g->g.p - g->g.mutual);
    info->mutual_dyads = (int64_t)g->g.mutual;
    for (int b = 0; b < kBuckets; ++b) {
        info->bucket_dyads[b] = g->g.bucket_off[b + 1] - g->g.bucket_off[b];
        info->bucket_cost[b] = g->g.bucket_cost[b];
    }
    info->hub_tasks = g->g.n_hub_tasks;
    info->hub_stream = g->g.hub_stream;
    info->hub_staged = g->g.hub_staged;
    const forward_lists& t = g->g.tri;
    info->fwd_entries = t.fwd_ptr ? t.entries : 0;
    for (int b = 0; b < kBuckets; ++b) {
        info->tri_bucket_edges[b] = t.edges.off[b + 1] - t.edges.off[b];
        info->tri_bucket_cost[b] = t.edges.cost[b];
    }
    // the forward lists' hub tasks a census runs: the half-size set when there is one
    const bool fine = t.edges.fine_tasks != nullptr;
    info->tri_tasks = fine ? t.edges.fine_n_tasks : t.edges.n_tasks;
    info->tri_stream = t.edges.stream;
    info->tri_staged = fine ? t.edges.fine_staged : t.edges.staged;
    info->hub_groups = g->g.n_hub_groups;
    info->tri_groups = fine ? t.edges.fine_n_groups : t.edges.n_groups;
    info->hub_chunk = g->g.hub_chunk;
    info->tri_chunk = !t.fwd_ptr ? 0 : fine ? kHubChunk / 2 : t.edges.chunk;
}

int run_census_locked(tc_context_s* ctx, const device_graph& g, const census_slices& sl,
                      unsigned long long raw[16], int table, bool tri) {
    hipEvent_t* ev = ctx->timing ? ctx->ev : nullptr;
    census_config cfg = config_of(ctx->tuning);
    cfg.side_blocks = (uint32_t)ctx->cu_count;
    hipError_t e = census_launch(g, sl, tri, ctx->tables + 64 * table, ctx->acc, ctx->counters, cfg, ctx->stream,
                                 ev, ctx->side, ctx->fork);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->host_raw, ctx->acc, sizeof(unsigned long long) * kNumClasses,
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return status_from_hip(e);
    std::memcpy(raw, ctx->host_raw, sizeof(unsigned long long) * kNumClasses);
    if (ev) {
        for (int b = 0; b < kBuckets; ++b) {
            if (sl.end[b] <= sl.begin[b]) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * b], ev[2 * b + 1]) == hipSuccess) {
                ctx->kstats.ms[b] += ms;
                ctx->kstats.launches[b] += 1;
            }
        }
        float ms = 0.f;
        if (tri && g.p > 0 && hipEventElapsedTime(&ms, ev[2 * kBuckets], ev[2 * kBuckets + 1]) == hipSuccess) {
            ctx->kstats.totals_ms += ms;
            ctx->kstats.totals_launches += 1;
        }
    }
    ctx->kstats.census_calls += 1;
    return TC_OK;
}

int run_full_locked(tc_context_s* ctx, const device_graph& g, unsigned long long raw[16], int table) {
    const bool tri = ctx->tuning.tri && g.tri.fwd_ptr;
    return run_census_locked(ctx, g, full_slices(g, tri), raw, table, tri);
}

int build_into(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, uint32_t flags, const bucket_params& bp,
               hipStream_t stream, device_graph* out, tc_graph_info* info) {
    const int32_t *s_dev = src, *d_dev = dst;
    int32_t* tmp = nullptr;
    hipError_t e = hipSuccess;
    if (!(flags & TC_BUILD_DEVICE_PTRS) && m > 0) {
        e = hipMalloc((void**)&tmp, sizeof(int32_t) * 2 * (size_t)m);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp, src, sizeof(int32_t) * m, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp + m, dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, stream);
        s_dev = tmp;
        d_dev = tmp + m;
    }
    build_status st;
    if (e == hipSuccess) st = build_graph_device(n, m, s_dev, d_dev, bp, stream, out);
    if (tmp) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(tmp);
    }
    int rc = TC_OK;
    if (e != hipSuccess) rc = status_from_hip(e);
    else if (st.bad_ids) rc = TC_ERR_ARG;
    else if (st.too_large) rc = TC_ERR_RANGE;
    else if (!st.ok) rc = status_from_hip(st.hip);
    else if ((flags & TC_BUILD_STRICT) && (st.self_loops > 0 || st.duplicates > 0)) rc = TC_ERR_ARG;
    if (rc != TC_OK) {
        free_device_graph(out);
        return rc;
    }
    if (info) {
        *info = tc_graph_info{};
        info->arcs_in = m;
        info->arcs_kept = st.arcs_kept;
        info->self_loops_dropped = st.self_loops;
        info->duplicates_dropped = m - st.self_loops - st.arcs_kept;
        info->max_degree = st.max_degree;
        info->sum_d2 = st.sum_d2;
    }
    return TC_OK;
}

// ---------------------------------------------------------------------------
// Scratch of tc_census_each_noalloc: kNoAllocCounterBytes of work counters,
// then one block of 16 accumulators per graph.  Each GPU holds its own copy of
// this array; host code never passes its name to a kernel (on the host it is a
// stand-in, not a device address) but the address hipGetSymbolAddress returns
// for the current device, looked up once per device by scratch_for_device.
constexpr size_t kNoAllocCounterBytes = 256;   // 64 work counters (the kernels use kBuckets x 8)
constexpr size_t kNoAllocBytes =
    kNoAllocCounterBytes + sizeof(unsigned long long) * kNumClasses * (size_t)TC_NOALLOC_MAX_GRAPHS;
static_assert(kNoAllocBytes == 33024, "size stated in tc.h");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`; `device` must be current.
hipError_t scratch_for_device(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// u-range bounds inside the u-major merge buckets (the hub bucket is filtered
// by the kernel instead).
__global__ void k_bounds(const dyad_rec* dyads, const uint64_t* off, uint32_t u0, uint32_t u1, uint64_t* out) {
    int b = threadIdx.x >> 1;
    if (b >= kBucketHub) return;
    uint32_t key = (threadIdx.x & 1) ? u1 : u0;
    uint64_t lo = off[b], hi = off[b + 1];
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (dyads[mid].u < key) lo = mid + 1; else hi = mid;
    }
    out[threadIdx.x] = lo;
}

}  // namespace

}  // namespace tc

// ---------------------------------------------------------------------------

extern "C" {

const char* tc_status_string(int s) {
    switch (s) {
        case TC_OK: return "ok";
        case TC_ERR_ARG: return "invalid argument";
        case TC_ERR_RANGE: return "size out of range";
        case TC_ERR_NOMEM: return "out of memory";
        case TC_ERR_DEVICE: return "device error";
        case TC_ERR_BUSY: return "graph busy";
        case TC_ERR_NOT_FOUND: return "ticket not found";
        case TC_ERR_SHUTDOWN: return "context shutting down";
        default: return "unknown status";
    }
}

int tc_class_table(uint8_t out[64]) {
    if (!out) return TC_ERR_ARG;
    std::memcpy(out, kTable.t, 64);
    return TC_OK;
}

int tc_context_create(int device, uint64_t hbm_budget_bytes, void* hip_stream, tc_context* out) {
    if (!out) return TC_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TC_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return TC_ERR_DEVICE;
    tc_context_s* ctx = new (std::nothrow) tc_context_s();
    if (!ctx) return TC_ERR_NOMEM;
    ctx->device = device;
    hipError_t e = hipSuccess;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
        ctx->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        ctx->own_stream = true;
    }
    if (e == hipSuccess) e = census_upload_table();
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->acc, sizeof(unsigned long long) * kNumClasses);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->counters, sizeof(unsigned int) * 64);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->host_raw, sizeof(unsigned long long) * kNumClasses);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&ctx->host_many,
                          sizeof(unsigned long long) * kNumClasses * (size_t)TC_NOALLOC_MAX_GRAPHS);
    if (e == hipSuccess) e = scratch_for_device(device, &ctx->scratch);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->tables, 4 * 64);
    if (e == hipSuccess) {
        // table 0: the 64 -> 16 class map; table f (1..3): code -> code >> 2 for
        // the codes whose (u, v) part is f, every other code to the discard bin
        uint8_t host[4 * 64];
        for (int c = 0; c < 64; ++c) {
            host[c] = kTable.t[c];
            for (int f = 1; f < 4; ++f) host[64 * f + c] = (c & 3) == f ? (uint8_t)(c >> 2) : (uint8_t)kNumClasses;
        }
        e = hipMemcpy(ctx->tables, host, sizeof(host), hipMemcpyHostToDevice);
    }
    for (int i = 0; i < 2 * kBuckets + 2 && e == hipSuccess; ++i) e = hipEventCreate(&ctx->ev[i]);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ctx->fork[i], hipEventDisableTiming);
    if (e == hipSuccess) {
        size_t free_b = 0, total_b = 0;
        e = hipMemGetInfo(&free_b, &total_b);
        ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
        hipDeviceProp_t prop;
        if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
        if (e == hipSuccess) {
            ctx->cu_count = prop.multiProcessorCount;
            std::strncpy(ctx->arch, prop.gcnArchName, sizeof(ctx->arch) - 1);
        }
    }
    if (e != hipSuccess) {
        tc_context_destroy(ctx);
        return status_from_hip(e);
    }
    ctx->tuning = default_tuning(ctx->cu_count);
    *out = ctx;
    return TC_OK;
}

int tc_context_destroy(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    serve_shutdown(ctx);
    batch_release_all(ctx);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (tc_graph g : ctx->graphs) {
            free_device_graph(&g->g);
            delete g;
        }
        ctx->graphs.clear();
    }
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (int i = 0; i < 2 * kBuckets + 2; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    for (int i = 0; i < 2; ++i)
        if (ctx->fork[i]) (void)hipEventDestroy(ctx->fork[i]);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->acc) (void)hipFree(ctx->acc);
    if (ctx->tables) (void)hipFree(ctx->tables);
    if (ctx->counters) (void)hipFree(ctx->counters);
    if (ctx->host_raw) (void)hipHostFree(ctx->host_raw);
    if (ctx->host_many) (void)hipHostFree(ctx->host_many);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return TC_OK;
}

int tc_build_graph(tc_context ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst, uint32_t flags,
                   tc_graph* out, tc_graph_info* info) {
    if (!ctx || !out || n < 0 || m < 0) return TC_ERR_ARG;
    if (m > 0 && (!src || !dst)) return TC_ERR_ARG;
    if (flags & ~(uint32_t)(TC_BUILD_STRICT | TC_BUILD_DEVICE_PTRS)) return TC_ERR_ARG;
    if (n > kMaxN) return TC_ERR_RANGE;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    tc_graph_s* g = new (std::nothrow) tc_graph_s();
    if (!g) return TC_ERR_NOMEM;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int rc = build_into(n, m, src, dst, flags, params_of(ctx->tuning), ctx->stream, &g->g, &g->info);
    if (rc != TC_OK) {
        delete g;
        return rc;
    }
    ctx->graphs.insert(g);
    *out = g;
    if (info) fill_info(g, info);
    return TC_OK;
}

int tc_graph_get_info(tc_context ctx, tc_graph g, tc_graph_info* info) {
    if (!ctx || !g || !info) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    fill_info(g, info);
    return TC_OK;
}

int tc_graph_release(tc_context ctx, tc_graph g) {
    if (!ctx || !g) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    if (g->pending.load() > 0) return TC_ERR_BUSY;
    batch_forget_graph_locked(ctx, g);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->graphs.erase(g);
    free_device_graph(&g->g);
    delete g;
    return TC_OK;
}

int tc_census(tc_context ctx, tc_graph g, uint64_t counts[16]) {
    if (!ctx || !g || !counts) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    unsigned long long raw[16];
    int rc = run_full_locked(ctx, g->g, raw);
    if (rc != TC_OK) return rc;
    finalize_counts(g->g.n, raw, counts);
    return TC_OK;
}

int tc_census64(tc_context ctx, tc_graph g, uint64_t counts[64]) {
    if (!ctx || !g || !counts) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    uint64_t out[64] = {0};
    typedef unsigned __int128 u128;
    u128 sum = 0;
    for (int f = 1; f < 4; ++f) {
        unsigned long long raw[16];
        int rc = run_full_locked(ctx, g->g, raw, f);
        if (rc != TC_OK) return rc;
        for (int b = 0; b < kNumClasses; ++b) {
            out[f | (b << 2)] = raw[b];
            sum += raw[b];
        }
    }
    const int64_t n = g->g.n;
    const u128 total = n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
    out[0] = (uint64_t)(total - sum);
    std::memcpy(counts, out, sizeof(out));
    return TC_OK;
}

int tc_census_range(tc_context ctx, tc_graph g, int32_t u_begin, int32_t u_end, uint64_t partial[16]) {
    if (!ctx || !g || !partial) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    int32_t n = g->g.n;
    if (u_begin < 0) u_begin = 0;
    if (u_end > n) u_end = n;
    unsigned long long raw[16] = {0};
    if (u_begin < u_end && g->g.p > 0) {
        uint64_t *off_dev = nullptr, *bnd_dev = nullptr;
        uint64_t bnd[2 * kBuckets];
        hipError_t e = hipMalloc((void**)&off_dev, sizeof(uint64_t) * (kBuckets + 1 + 2 * kBuckets));
        if (e != hipSuccess) return status_from_hip(e);
        bnd_dev = off_dev + kBuckets + 1;
        e = hipMemcpyAsync(off_dev, g->g.bucket_off, sizeof(uint64_t) * (kBuckets + 1), hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_bounds, dim3(1), dim3(64), 0, ctx->stream, g->g.dyads, off_dev, (uint32_t)u_begin,
                               (uint32_t)u_end, bnd_dev);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(bnd, bnd_dev, sizeof(bnd), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        (void)hipFree(off_dev);
        if (e != hipSuccess) return status_from_hip(e);
        census_slices sl;
        for (int b = 0; b < kBucketHub; ++b) {
            sl.begin[b] = bnd[2 * b];
            sl.end[b] = bnd[2 * b + 1];
        }
        sl.begin[kBucketHub] = g->g.bucket_off[kBucketHub];
        sl.end[kBucketHub] = g->g.bucket_off[kBucketHub + 1];
        sl.u_lo = (uint32_t)u_begin;
        sl.u_hi = (uint32_t)u_end;
        int rc = run_census_locked(ctx, g->g, sl, raw);
        if (rc != TC_OK) return rc;
    }
    partial[0] = 0;
    for (int k = 1; k < kNumClasses; ++k) partial[k] = raw[k];
    return TC_OK;
}

int tc_census_shard(tc_context ctx, tc_graph g, int32_t shard, int32_t nshards, uint64_t partial[16]) {
    if (!ctx || !g || !partial || nshards < 1 || shard < 0 || shard >= nshards) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    const device_graph& dg = g->g;
    unsigned long long raw[16] = {0};
    if (dg.p > 0) {
        const bool tri = ctx->tuning.tri && dg.tri.fwd_ptr;
        census_slices sl = full_slices(dg, tri);
        const uint64_t k = (uint64_t)shard, G = (uint64_t)nshards;
        for (int b = 0; b < kBucketHub; ++b) {
            const uint64_t lo = sl.begin[b], len = sl.end[b] - sl.begin[b];
            sl.begin[b] = lo + len * k / G;
            sl.end[b] = lo + len * (k + 1) / G;
        }
        const uint64_t ng = !tri ? dg.n_hub_groups
                            : dg.tri.edges.fine_tasks ? dg.tri.edges.fine_n_groups : dg.tri.edges.n_groups;
        sl.hub_g0 = (uint32_t)(ng * k / G);
        sl.hub_g1 = (uint32_t)(ng * (k + 1) / G);
        sl.totals_begin = dg.U * k / G;
        sl.totals_end = dg.U * (k + 1) / G;
        int rc = run_census_locked(ctx, dg, sl, raw, 0, tri);
        if (rc != TC_OK) return rc;
    }
    partial[0] = 0;
    for (int c = 1; c < kNumClasses; ++c) partial[c] = raw[c];
    return TC_OK;
}

int tc_census_each(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts) {
    if (!ctx || count < 0 || (count > 0 && (!graphs || !counts))) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int32_t i = 0; i < count; ++i)
        if (!graphs[i] || !ctx->graphs.count(graphs[i])) return TC_ERR_ARG;
    for (int32_t i = 0; i < count; ++i) {
        unsigned long long raw[16];
        int rc = run_full_locked(ctx, graphs[i]->g, raw);
        if (rc != TC_OK) return rc;
        finalize_counts(graphs[i]->g.n, raw, counts + 16 * (size_t)i);
    }
    return TC_OK;
}

int tc_census_each_noalloc(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts) {
    if (!ctx || count < 0 || (count > 0 && (!graphs || !counts))) return TC_ERR_ARG;
    if (count > TC_NOALLOC_MAX_GRAPHS) return TC_ERR_RANGE;
    if (!ctx->scratch || !ctx->host_many) return TC_ERR_DEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int32_t i = 0; i < count; ++i)
        if (!graphs[i] || !ctx->graphs.count(graphs[i])) return TC_ERR_ARG;
    if (count == 0) return TC_OK;
    unsigned int* ctr = reinterpret_cast<unsigned int*>(ctx->scratch);
    unsigned long long* accs =
        reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(ctx->scratch) + kNoAllocCounterBytes);
    census_config cfg = config_of(ctx->tuning);
    cfg.side_blocks = (uint32_t)ctx->cu_count;
    // every graph's launch sequence zeroes its own accumulator block and the
    // counters before its kernels; the stream orders the graphs
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
        const device_graph& g = graphs[i]->g;
        const bool tri = ctx->tuning.tri && g.tri.fwd_ptr;
        e = census_launch(g, full_slices(g, tri), tri, ctx->tables, accs + (size_t)kNumClasses * i, ctr, cfg,
                          ctx->stream, nullptr, ctx->side, ctx->fork);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->host_many, accs, sizeof(unsigned long long) * kNumClasses * (size_t)count,
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return status_from_hip(e);
    for (int32_t i = 0; i < count; ++i)
        finalize_counts(graphs[i]->g.n, ctx->host_many + (size_t)kNumClasses * i, counts + 16 * (size_t)i);
    ctx->kstats.census_calls += (uint64_t)count;
    return TC_OK;
}

int tc_set_tuning(tc_context ctx, const tc_tuning* t) {
    if (!ctx || !t) return TC_ERR_ARG;
    if (check_tuning(*t) != TC_OK) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> lt(ctx->tuning_mu);
    ctx->tuning = *t;
    return TC_OK;
}

int tc_get_tuning(tc_context ctx, tc_tuning* t) {
    if (!ctx || !t) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    *t = ctx->tuning;
    return TC_OK;
}

int tc_graph_rebucket(tc_context ctx, tc_graph g) {
    if (!ctx || !g) return TC_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->graphs.count(g)) return TC_ERR_ARG;
    if (g->pending.load() > 0) return TC_ERR_BUSY;
    const bucket_params bp = params_of(ctx->tuning);
    if (g->g.bp.t0 == bp.t0 && g->g.bp.t1 == bp.t1 && g->g.bp.t_hub == bp.t_hub && g->g.bp.tri == bp.tri &&
        g->g.bp.hub_tile == bp.hub_tile)
        return TC_OK;
    batch_forget_graph_locked(ctx, g);
    return status_from_hip(bucket_dyads(&g->g, bp, ctx->stream));
}

int tc_set_timing(tc_context ctx, int enable) {
    if (!ctx) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->timing = enable != 0;
    return TC_OK;
}

int tc_get_kernel_stats(tc_context ctx, tc_kernel_stats* out) {
    if (!ctx || !out) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    *out = ctx->kstats;
    return TC_OK;
}

int tc_reset_kernel_stats(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->kstats = tc_kernel_stats{};
    return TC_OK;
}

}  // extern "C"
