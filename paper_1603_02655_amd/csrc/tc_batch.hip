// Batched census over many resident graphs: one persistent kernel launch over
// a work-item list (graph, execution mode, dyad range), captured once into a
// HIP graph (zero accumulators -> persistent kernel -> 16 counts per graph back
// to pinned host memory) and replayed.  Descriptors and items live in device
// buffers read by the kernel, so another set of graphs that fits the captured
// capacities is served by rewriting those buffers and replaying; the capture is
// redone only when a capacity grows.
#include <algorithm>
#include <cstring>

#include "tc_api_internal.h"

namespace tc {

struct batch_plan {
    std::vector<tc_graph> graphs;       // graphs the device buffers currently describe
    uint32_t cap_graphs = 0, cap_items = 0;
    graph_desc* d_desc = nullptr;
    work_item* d_items = nullptr;
    uint32_t* d_num = nullptr;
    unsigned long long* d_accs = nullptr;
    unsigned int* d_ctr = nullptr;
    unsigned long long* h_accs = nullptr;   // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t grid = 0, hub_grid = 0;
    uint32_t hub_tile = 0, batch_tile = 0;  // LDS tiles the captured kernels use
    uint32_t hub_chunk = 0;                 // largest records per hub task of the graphs (hub kernel instance)
    bool valid = false;                     // buffers describe `graphs`
    bool tri = false;                       // ... through their forward lists

    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_desc) (void)hipFree(d_desc);
        if (d_items) (void)hipFree(d_items);
        if (d_num) (void)hipFree(d_num);
        if (d_accs) (void)hipFree(d_accs);
        if (d_ctr) (void)hipFree(d_ctr);
        if (h_accs) (void)hipHostFree(h_accs);
        *this = batch_plan{};
    }
};

void batch_release_all(tc_context_s* ctx) {
    if (ctx->batch) {
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        ctx->batch->release();
        delete ctx->batch;
        ctx->batch = nullptr;
    }
}

void batch_forget_graph_locked(tc_context_s* ctx, tc_graph g) {
    batch_plan* p = ctx->batch;
    if (p && std::find(p->graphs.begin(), p->graphs.end(), g) != p->graphs.end()) {
        p->graphs.clear();
        p->valid = false;
    }
}

graph_desc describe(const device_graph& g) {
    graph_desc d{};
    d.dyads = g.dyads;
    d.nbr = g.nbr;
    d.tpre = g.tpre;
    d.rinfo = g.rinfo;
    d.n = (uint64_t)g.n;
    d.hub_tasks = g.hub_tasks;
    d.owner = g.owner;
    d.row_ptr = g.row_ptr;
    d.U = g.U;
    d.edges = g.tri.edges.recs;
    d.fwd = g.tri.fwd;
    d.edge_tasks = g.tri.edges.tasks;
    d.hub_ntasks = g.n_hub_tasks;
    d.hub_groups = g.n_hub_groups;
    d.tri_tasks = g.tri.edges.n_tasks;
    d.tri_groups = g.tri.edges.n_groups;
    d.hub_chunk = g.hub_chunk;
    d.tri_chunk = g.tri.edges.chunk;
    return d;
}

// Work items of one graph: hub tasks into `hub`; into `out` the totals chunks
// (when `tri`), then group-mode records (largest), wave-mode chunks and
// lane-mode chunks, over the forward-list edge records when `tri`.
void append_items(const device_graph& g, uint32_t gi, bool tri, std::vector<work_item>& hub,
                  std::vector<work_item>& out) {
    const uint64_t* off = g.bucket_off;
    uint32_t ngroups = g.n_hub_groups, flag = 0;
    if (tri) {
        for (uint64_t e = 0; e < g.U; e += kBatchTotalsPerItem)
            out.push_back(work_item{gi, kItemTotals, (uint32_t)e,
                                    (uint32_t)std::min<uint64_t>(e + kBatchTotalsPerItem, g.U)});
        off = g.tri.edges.off;
        ngroups = g.tri.edges.n_groups;
        flag = kItemTri;
    }
    for (uint32_t t = 0; t < ngroups; ++t) hub.push_back(work_item{gi, kItemHub | flag, t, t + 1});
    for (uint64_t d = off[2]; d < off[3]; ++d)
        out.push_back(work_item{gi, kItemGroup | flag, (uint32_t)d, (uint32_t)d + 1});
    for (uint64_t d = off[1]; d < off[2]; d += kBatchWavePerItem)
        out.push_back(work_item{gi, kItemWave | flag, (uint32_t)d,
                                (uint32_t)std::min<uint64_t>(d + kBatchWavePerItem, off[2])});
    for (uint64_t d = off[0]; d < off[1]; d += kBatchLanePerItem)
        out.push_back(work_item{gi, kItemLane | flag, (uint32_t)d,
                                (uint32_t)std::min<uint64_t>(d + kBatchLanePerItem, off[1])});
}

namespace {

hipError_t ensure_capacity(batch_plan* p, uint32_t graphs, uint32_t items, hipStream_t s, uint32_t grid,
                           uint32_t hub_grid, uint32_t hub_tile, uint32_t batch_tile, uint32_t hub_chunk) {
    if (p->exec && graphs <= p->cap_graphs && items <= p->cap_items && grid == p->grid && hub_grid == p->hub_grid &&
        hub_tile == p->hub_tile && batch_tile == p->batch_tile && hub_chunk == p->hub_chunk)
        return hipSuccess;
    (void)hipStreamSynchronize(s);
    p->release();
    p->cap_graphs = std::max<uint32_t>(graphs + graphs / 4, 16);
    p->cap_items = std::max<uint32_t>(items + items / 4, 1024);
    p->grid = grid;
    p->hub_grid = hub_grid;
    p->hub_tile = hub_tile;
    p->batch_tile = batch_tile;
    p->hub_chunk = hub_chunk;
    hipError_t e = hipMalloc((void**)&p->d_desc, sizeof(graph_desc) * p->cap_graphs);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_items, sizeof(work_item) * p->cap_items);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_num, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_accs, sizeof(unsigned long long) * kNumClasses * p->cap_graphs);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ctr, sizeof(unsigned int) * 64);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&p->h_accs, sizeof(unsigned long long) * kNumClasses * p->cap_graphs);
    if (e != hipSuccess) {
        p->release();
        return e;
    }
    // capture: zero accumulators and counters, persistent kernel, read-back
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = batch_launch(p->d_desc, p->d_items, p->d_num, p->d_accs, (uint64_t)kNumClasses * p->cap_graphs,
                                 p->d_ctr, p->grid, p->hub_grid, p->hub_tile, p->batch_tile, p->hub_chunk, s);
    hipError_t ec = hipMemcpyAsync(p->h_accs, p->d_accs, sizeof(unsigned long long) * kNumClasses * p->cap_graphs,
                                   hipMemcpyDeviceToHost, s);
    e = hipStreamEndCapture(s, &p->graph);
    if (el != hipSuccess) e = el;
    if (ec != hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) p->release();
    return e;
}

}  // namespace

}  // namespace tc

using namespace tc;

extern "C" int tc_census_batch(tc_context ctx, const tc_graph* graphs, int32_t count, uint64_t* counts) {
    if (!ctx || count < 0 || (count > 0 && (!graphs || !counts))) return TC_ERR_ARG;
    if (count == 0) return TC_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int32_t i = 0; i < count; ++i)
        if (!graphs[i] || !ctx->graphs.count(graphs[i])) return TC_ERR_ARG;
    if (!ctx->batch) ctx->batch = new (std::nothrow) batch_plan();
    if (!ctx->batch) return TC_ERR_NOMEM;
    batch_plan* p = ctx->batch;
    std::vector<tc_graph> want(graphs, graphs + count);
    hipError_t e = hipSuccess;
    const bool tri = ctx->tuning.tri != 0;
    if (!(p->valid && p->graphs == want && p->grid == ctx->tuning.batch_blocks &&
          p->hub_grid == ctx->tuning.hub_blocks && p->hub_tile == ctx->tuning.hub_tile &&
          p->batch_tile == ctx->tuning.batch_tile && p->tri == tri)) {
        std::vector<work_item> items, rest;
        std::vector<graph_desc> descs(count);
        uint32_t hub_chunk = 0;
        for (int32_t i = 0; i < count; ++i) {
            const device_graph& g = graphs[i]->g;
            descs[i] = describe(g);
            append_items(g, (uint32_t)i, tri && g.tri.fwd_ptr, items, rest);
            hub_chunk = std::max(hub_chunk, tri && g.tri.fwd_ptr ? g.tri.edges.chunk : g.hub_chunk);
        }
        const uint32_t nums[2] = {(uint32_t)items.size(), (uint32_t)(items.size() + rest.size())};
        items.insert(items.end(), rest.begin(), rest.end());     // hub items first
        e = ensure_capacity(p, (uint32_t)count, (uint32_t)items.size(), ctx->stream, ctx->tuning.batch_blocks,
                            ctx->tuning.hub_blocks, ctx->tuning.hub_tile, ctx->tuning.batch_tile, hub_chunk);
        if (e != hipSuccess) return status_from_hip(e);
        uint32_t nitems = (uint32_t)items.size();
        e = hipMemcpyAsync(p->d_desc, descs.data(), sizeof(graph_desc) * count, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess && nitems)
            e = hipMemcpyAsync(p->d_items, items.data(), sizeof(work_item) * nitems, hipMemcpyHostToDevice,
                               ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_num, nums, sizeof(nums), hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);   // host vectors go out of scope
        if (e != hipSuccess) {
            p->valid = false;
            return status_from_hip(e);
        }
        p->graphs = want;
        p->valid = true;
        p->tri = tri;
    }
    if (ctx->timing) (void)hipEventRecord(ctx->ev[0], ctx->stream);
    e = hipGraphLaunch(p->exec, ctx->stream);
    if (ctx->timing) (void)hipEventRecord(ctx->ev[1], ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return status_from_hip(e);
    if (ctx->timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) {
            ctx->kstats.batch_ms += ms;
            ctx->kstats.batch_launches += 1;
        }
    }
    for (int32_t i = 0; i < count; ++i)
        finalize_counts(graphs[i]->g.n, p->h_accs + (size_t)kNumClasses * i, counts + (size_t)kNumClasses * i);
    return TC_OK;
}
