// Serving loop: continuous batching of census requests on one device.
//
// tc_submit / tc_submit_arcs put a job on a host queue and return.  A worker
// thread admits queued jobs in arrival order while their device footprint fits
// the context's budget (a resident graph costs only its work-item and
// accumulator space; a request that carries arcs also costs its build), packs
// the admitted jobs of the moment into one round, and runs the round as one
// batched persistent launch on a free stream of a small pool.  Rounds on
// different streams overlap on the device; jobs that arrive while rounds run
// form the next round.  A host callback enqueued after each round's read-back
// marks its completion; tc_poll never blocks.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "tc_api_internal.h"

namespace tc {

namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kSlots = 3;                 // rounds in flight
constexpr size_t kMaxJobsPerRound = 512;
// A round closes once its jobs hold this many neighbour entries (about 5 ms of
// census at the batched rate): rounds stay short, so a request admitted behind
// a full queue waits for a few short rounds instead of one long one.
constexpr uint64_t kMaxRoundEntries = 64ull << 20;

enum job_state { kQueued, kRunning, kDone };

struct job {
    tc_ticket ticket = 0;
    tc_graph g = nullptr;                 // resident graph (not owned)
    bool cold = false;                    // arcs carried by the request, built on admission
    int32_t n = 0;
    uint32_t flags = 0;
    std::vector<int32_t> src, dst;
    device_graph built;                   // a cold job's graph, freed when the round ends
    uint64_t footprint = 0;
    uint64_t entries = 0;                 // neighbour entries (2 x dyads; 2 x arcs for a cold job)
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = TC_OK;
    job_state state = kQueued;
    uint64_t counts[16] = {0};
};

struct slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    std::atomic<bool> finished{false};    // set by the host callback (which takes no lock)
    std::vector<job*> jobs;
    uint32_t cap_graphs = 0, cap_items = 0;
    graph_desc* d_desc = nullptr;
    work_item* d_items = nullptr;
    uint32_t* d_num = nullptr;
    unsigned long long* d_accs = nullptr;
    unsigned int* d_ctr = nullptr;
    graph_desc* h_desc = nullptr;         // pinned staging
    work_item* h_items = nullptr;
    uint32_t* h_num = nullptr;
    unsigned long long* h_accs = nullptr;
};

void slot_free(slot& s) {
    if (s.d_desc) (void)hipFree(s.d_desc);
    if (s.d_items) (void)hipFree(s.d_items);
    if (s.d_num) (void)hipFree(s.d_num);
    if (s.d_accs) (void)hipFree(s.d_accs);
    if (s.d_ctr) (void)hipFree(s.d_ctr);
    if (s.h_desc) (void)hipHostFree(s.h_desc);
    if (s.h_items) (void)hipHostFree(s.h_items);
    if (s.h_num) (void)hipHostFree(s.h_num);
    if (s.h_accs) (void)hipHostFree(s.h_accs);
    s.d_desc = nullptr; s.d_items = nullptr; s.d_num = nullptr; s.d_accs = nullptr; s.d_ctr = nullptr;
    s.h_desc = nullptr; s.h_items = nullptr; s.h_num = nullptr; s.h_accs = nullptr;
    s.cap_graphs = s.cap_items = 0;
}

hipError_t slot_reserve(slot& s, uint32_t graphs, uint32_t items) {
    if (s.d_desc && graphs <= s.cap_graphs && items <= s.cap_items) return hipSuccess;
    (void)hipStreamSynchronize(s.stream);
    slot_free(s);
    s.cap_graphs = std::max<uint32_t>(graphs * 2, 64);
    s.cap_items = std::max<uint32_t>(items + items / 2, 4096);
    hipError_t e = hipMalloc((void**)&s.d_desc, sizeof(graph_desc) * s.cap_graphs);
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_items, sizeof(work_item) * s.cap_items);
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_num, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_accs, sizeof(unsigned long long) * kNumClasses * s.cap_graphs);
    if (e == hipSuccess) e = hipMalloc((void**)&s.d_ctr, sizeof(unsigned int) * 64);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_desc, sizeof(graph_desc) * s.cap_graphs);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_items, sizeof(work_item) * s.cap_items);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_num, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_accs, sizeof(unsigned long long) * kNumClasses * s.cap_graphs);
    if (e != hipSuccess) slot_free(s);
    return e;
}

// Bytes a job holds on the device while it is in flight.
uint64_t job_footprint(const job& j) {
    uint64_t ws = sizeof(unsigned long long) * kNumClasses + sizeof(graph_desc);
    if (!j.cold) {
        // the items append_items makes for the graph (forward-list items when it has forward lists)
        const device_graph& g = j.g->g;
        const bool tri = g.tri.fwd_ptr != nullptr;
        const uint64_t* off = tri ? g.tri.edges.off : g.bucket_off;
        uint64_t items = (tri ? g.tri.edges.n_groups : g.n_hub_groups) + (off[3] - off[2]) +
                         (off[2] - off[1] + kBatchWavePerItem - 1) / kBatchWavePerItem +
                         (off[1] - off[0] + kBatchLanePerItem - 1) / kBatchLanePerItem;
        if (tri) items += (g.U + kBatchTotalsPerItem - 1) / kBatchTotalsPerItem;
        return ws + sizeof(work_item) * items;
    }
    uint64_t m = j.src.size();
    // arcs on the device, two sort buffers, run heads and unique index, the
    // graph (entries, owners, prefix counts, dyad records) and its work items
    return ws + 8 * m + 2 * m * 8 * 2 + 2 * m * 16 + 2 * m * 16 + m * sizeof(dyad_rec) + 16 * ((uint64_t)j.n + 1) +
           sizeof(work_item) * (m + 1);
}

}  // namespace

struct serve_state {
    tc_context_s* ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<job*> queue;
    std::map<tc_ticket, job*> jobs;
    slot slots[kSlots];
    std::thread worker;
    bool stop = false;
    tc_ticket next_ticket = 1;
    uint64_t bytes_in_flight = 0;
    uint64_t submitted = 0, completed = 0, rounds = 0;
    std::vector<double> latency_ms;
    double admission_ms_sum = 0;
    uint64_t admitted = 0;
    int rotate = 0;
};

namespace {

struct cb_arg {
    serve_state* S;
    int slot;
};

// Host callback after a round's read-back.  It must not block: the stream
// (and anything that synchronises the device, e.g. hipFree) waits for it, so
// it takes no lock; it sets the slot's flag and wakes the worker, whose waits
// are also bounded in time in case the wake-up races with its check.
void on_round_done(void* arg) {
    cb_arg* a = static_cast<cb_arg*>(arg);
    serve_state* S = a->S;
    S->slots[a->slot].finished.store(true);
    S->cv.notify_all();
    delete a;
}

// Retires a finished round.  Called with the lock held, so it makes no HIP
// call: graphs built for cold requests are handed back in `to_free` and freed
// by the caller after it has released the lock.
void complete_slot_locked(serve_state* S, slot& s, std::vector<device_graph>& to_free) {
    const double t = now_ms();
    for (size_t i = 0; i < s.jobs.size(); ++i) {
        job* j = s.jobs[i];
        if (j->status == TC_OK) {
            int32_t n = j->cold ? j->built.n : j->g->g.n;
            finalize_counts(n, s.h_accs + kNumClasses * i, j->counts);
        }
        if (j->cold) {
            to_free.push_back(j->built);
            j->built = device_graph{};
        } else {
            j->g->pending.fetch_sub(1);
        }
        j->t_done = t;
        j->state = kDone;
        S->bytes_in_flight -= j->footprint;
        S->completed += 1;
        S->latency_ms.push_back(j->t_done - j->t_submit);
    }
    s.jobs.clear();
    s.busy = false;
    s.finished.store(false);
}

void free_graphs_unlocked(std::unique_lock<std::mutex>& lk, std::vector<device_graph>& to_free) {
    if (to_free.empty()) return;
    lk.unlock();
    for (device_graph& g : to_free) free_device_graph(&g);
    to_free.clear();
    lk.lock();
}

// Builds cold graphs, stages descriptors and items, and enqueues the round on
// the slot's stream.  Runs on the worker thread without the lock.  Returns
// false if nothing was enqueued (every job failed), in which case the caller
// completes the slot itself.
bool launch_round(serve_state* S, int si) {
    slot& s = S->slots[si];
    tc_context_s* ctx = S->ctx;
    const tc_tuning tun = tuning_snapshot(ctx);
    for (job* j : s.jobs) {
        if (!j->cold) continue;
        bucket_params bp = params_of(tun);
        bp.tri = 0;   // cold graphs live for one round: no forward lists (not in their footprint)
        j->status = build_into(j->n, (int64_t)j->src.size(), j->src.data(), j->dst.data(), j->flags, bp, s.stream,
                               &j->built, nullptr);
        std::vector<int32_t>().swap(j->src);
        std::vector<int32_t>().swap(j->dst);
    }
    std::vector<work_item> items, rest;
    std::vector<graph_desc> descs(s.jobs.size());
    for (size_t i = 0; i < s.jobs.size(); ++i) {
        job* j = s.jobs[i];
        if (j->status != TC_OK) {
            descs[i] = graph_desc{};
            continue;
        }
        const device_graph& g = j->cold ? j->built : j->g->g;
        descs[i] = describe(g);
        append_items(g, (uint32_t)i, tun.tri && g.tri.fwd_ptr, items, rest);
    }
    const uint32_t n_hub = (uint32_t)items.size();
    items.insert(items.end(), rest.begin(), rest.end());     // hub items first
    hipError_t e = slot_reserve(s, (uint32_t)s.jobs.size(), (uint32_t)items.size());
    if (e == hipSuccess) {
        std::memcpy(s.h_desc, descs.data(), sizeof(graph_desc) * descs.size());
        if (!items.empty()) std::memcpy(s.h_items, items.data(), sizeof(work_item) * items.size());
        s.h_num[0] = n_hub;
        s.h_num[1] = (uint32_t)items.size();
        e = hipMemcpyAsync(s.d_desc, s.h_desc, sizeof(graph_desc) * descs.size(), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && !items.empty())
            e = hipMemcpyAsync(s.d_items, s.h_items, sizeof(work_item) * items.size(), hipMemcpyHostToDevice,
                               s.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.d_num, s.h_num, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess)
            e = batch_launch(s.d_desc, s.d_items, s.d_num, s.d_accs, (uint64_t)kNumClasses * s.jobs.size(), s.d_ctr,
                             tun.batch_blocks, tun.hub_blocks, tun.hub_tile, tun.batch_tile, s.stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.h_accs, s.d_accs, sizeof(unsigned long long) * kNumClasses * s.jobs.size(),
                               hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipLaunchHostFunc(s.stream, on_round_done, new cb_arg{S, si});
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s.stream);
        for (job* j : s.jobs)
            if (j->status == TC_OK) j->status = status_from_hip(e);
        return false;
    }
    return true;
}

void worker_main(serve_state* S) {
    (void)hipSetDevice(S->ctx->device);
    std::vector<device_graph> to_free;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // 1. retire finished rounds
        for (slot& s : S->slots)
            if (s.busy && s.finished.load()) complete_slot_locked(S, s, to_free);
        free_graphs_unlocked(lk, to_free);
        if (S->stop) break;
        // 2. admit queued jobs into a free slot
        int free_slot = -1;
        for (int k = 0; k < kSlots; ++k) {
            int si = (S->rotate + k) % kSlots;
            if (!S->slots[si].busy) { free_slot = si; break; }
        }
        if (free_slot >= 0 && !S->queue.empty()) {
            slot& s = S->slots[free_slot];
            const double t = now_ms();
            uint64_t round_entries = 0;
            while (!S->queue.empty() && s.jobs.size() < kMaxJobsPerRound &&
                   (s.jobs.empty() || round_entries + S->queue.front()->entries <= kMaxRoundEntries)) {
                job* j = S->queue.front();
                if (j->footprint > S->ctx->budget) {          // can never fit
                    S->queue.pop_front();
                    j->status = TC_ERR_NOMEM;
                    j->state = kDone;
                    j->t_done = t;
                    if (!j->cold) j->g->pending.fetch_sub(1);
                    S->completed += 1;
                    continue;
                }
                if (S->bytes_in_flight + j->footprint > S->ctx->budget) break;   // wait for memory
                S->queue.pop_front();
                S->bytes_in_flight += j->footprint;
                round_entries += j->entries;
                j->state = kRunning;
                j->t_admit = t;
                S->admission_ms_sum += t - j->t_submit;
                S->admitted += 1;
                s.jobs.push_back(j);
            }
            if (!s.jobs.empty()) {
                s.busy = true;
                s.finished = false;
                S->rounds += 1;
                S->rotate = (free_slot + 1) % kSlots;
                lk.unlock();
                bool ok = launch_round(S, free_slot);
                lk.lock();
                if (!ok) complete_slot_locked(S, s, to_free);
                continue;
            }
        }
        bool any_busy = false;
        for (slot& s : S->slots) any_busy |= s.busy;
        if (any_busy) S->cv.wait_for(lk, std::chrono::milliseconds(1));
        else S->cv.wait(lk);
    }
    // shutdown: drain the device, cancel what is left
    lk.unlock();
    for (slot& s : S->slots) (void)hipStreamSynchronize(s.stream);
    lk.lock();
    for (slot& s : S->slots)
        if (s.busy) complete_slot_locked(S, s, to_free);
    free_graphs_unlocked(lk, to_free);
    for (job* j : S->queue) {
        j->status = TC_ERR_SHUTDOWN;
        j->state = kDone;
        if (!j->cold) j->g->pending.fetch_sub(1);
    }
    S->queue.clear();
}

serve_state* ensure_serving(tc_context_s* ctx, int* rc) {
    *rc = TC_OK;
    if (ctx->serve) return ctx->serve;
    serve_state* S = new (std::nothrow) serve_state();
    if (!S) { *rc = TC_ERR_NOMEM; return nullptr; }
    S->ctx = ctx;
    for (slot& s : S->slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            for (slot& t : S->slots)
                if (t.stream) (void)hipStreamDestroy(t.stream);
            delete S;
            *rc = TC_ERR_DEVICE;
            return nullptr;
        }
    }
    S->worker = std::thread(worker_main, S);
    ctx->serve = S;
    return S;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::min<double>((double)v.size() - 1, q * (double)(v.size() - 1) + 0.5);
    return v[k];
}

}  // namespace

// Stops the worker; queued tickets end with TC_ERR_SHUTDOWN (still pollable).
void serve_stop(tc_context_s* ctx) {
    serve_state* S = ctx->serve;
    if (!S || !S->worker.joinable()) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    S->worker.join();
}

void serve_shutdown(tc_context_s* ctx) {
    serve_state* S = ctx->serve;
    if (!S) return;
    serve_stop(ctx);
    for (auto& kv : S->jobs) {
        if (kv.second->cold) free_device_graph(&kv.second->built);
        delete kv.second;
    }
    for (slot& s : S->slots) {
        slot_free(s);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    delete S;
    ctx->serve = nullptr;
}

}  // namespace tc

using namespace tc;

namespace {

int submit_job(tc_context ctx, job* j, tc_ticket* out) {
    int rc;
    serve_state* S;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S = ensure_serving(ctx, &rc);
    }
    if (!S) {
        delete j;
        return rc;
    }
    j->footprint = job_footprint(*j);
    j->entries = j->cold ? 2 * (uint64_t)j->src.size() : j->g->g.U;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            if (!j->cold) j->g->pending.fetch_sub(1);
            delete j;
            return TC_ERR_SHUTDOWN;
        }
        j->ticket = S->next_ticket++;
        j->t_submit = now_ms();
        S->jobs[j->ticket] = j;
        S->queue.push_back(j);
        S->submitted += 1;
        *out = j->ticket;
    }
    S->cv.notify_all();
    return TC_OK;
}

}  // namespace

extern "C" int tc_submit(tc_context ctx, tc_graph g, tc_ticket* out) {
    if (!ctx || !g || !out) return TC_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->graphs.count(g)) return TC_ERR_ARG;
        g->pending.fetch_add(1);
    }
    job* j = new (std::nothrow) job();
    if (!j) {
        g->pending.fetch_sub(1);
        return TC_ERR_NOMEM;
    }
    j->g = g;
    int rc = submit_job(ctx, j, out);
    if (rc != TC_OK && rc != TC_ERR_SHUTDOWN) g->pending.fetch_sub(1);
    return rc;
}

extern "C" int tc_submit_arcs(tc_context ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              uint32_t flags, tc_ticket* out) {
    if (!ctx || !out || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return TC_ERR_ARG;
    if (flags & ~(uint32_t)TC_BUILD_STRICT) return TC_ERR_ARG;
    if (n > kMaxN) return TC_ERR_RANGE;
    job* j = new (std::nothrow) job();
    if (!j) return TC_ERR_NOMEM;
    j->cold = true;
    j->n = n;
    j->flags = flags;
    try {
        j->src.assign(src, src + m);
        j->dst.assign(dst, dst + m);
    } catch (...) {
        delete j;
        return TC_ERR_NOMEM;
    }
    return submit_job(ctx, j, out);
}

extern "C" int tc_poll(tc_context ctx, tc_ticket ticket, uint64_t counts[16], int* done) {
    if (!ctx || !counts || !done) return TC_ERR_ARG;
    serve_state* S = ctx->serve;
    if (!S) return TC_ERR_NOT_FOUND;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return TC_ERR_NOT_FOUND;
    job* j = it->second;
    if (j->state != kDone) {
        *done = 0;
        return S->stop ? TC_ERR_SHUTDOWN : TC_OK;
    }
    int st = j->status;
    if (st == TC_OK) std::memcpy(counts, j->counts, sizeof(j->counts));
    *done = 1;
    S->jobs.erase(it);
    delete j;
    return st;
}

extern "C" int tc_serve_stop(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    serve_stop(ctx);
    return TC_OK;
}

extern "C" int tc_serve_get_stats(tc_context ctx, tc_serve_stats* out) {
    if (!ctx || !out) return TC_ERR_ARG;
    *out = tc_serve_stats{};
    serve_state* S = ctx->serve;
    if (!S) return TC_OK;
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rounds = S->rounds;
    out->bytes_in_flight = S->bytes_in_flight;
    out->p50_ms = percentile(S->latency_ms, 0.50);
    out->p99_ms = percentile(S->latency_ms, 0.99);
    out->mean_admission_ms = S->admitted ? S->admission_ms_sum / (double)S->admitted : 0.0;
    {
        std::lock_guard<std::mutex> lk2(ctx->mu);
        out->resident_graphs = ctx->graphs.size();
    }
    return TC_OK;
}

extern "C" int tc_serve_reset_stats(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    serve_state* S = ctx->serve;
    if (!S) return TC_OK;
    std::lock_guard<std::mutex> lk(S->mu);
    S->submitted = S->completed = S->rounds = S->admitted = 0;
    S->latency_ms.clear();
    S->admission_ms_sum = 0;
    return TC_OK;
}
