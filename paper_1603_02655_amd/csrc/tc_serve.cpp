// Serving loop: continuous batching of census requests on one device.
//
// tc_submit / tc_submit_arcs hand a job to the scheduler (tc_sched.h), which
// admits queued jobs in arrival order while their device footprint fits the
// context's budget (a resident graph costs only its work-item and
// accumulator space; a request that carries arcs also costs its build), packs
// the admitted jobs of the moment into one round, and runs the round on a
// free slot of the HIP executor below: one batched persistent launch on the
// slot's stream.  Rounds on different slots overlap on the device; jobs that
// arrive while rounds run form the next round.  A host callback enqueued after
// each round's read-back tells the scheduler that the round finished; tc_poll
// never blocks.  A round that runs past the watchdog fails its tickets with
// TC_ERR_DEVICE and its slot is not used again.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <thread>

#include "tc_api_internal.h"
#include "tc_sched.h"

namespace tc {

namespace {

constexpr int kSlots = 4;                 // rounds in flight (HIP maps streams onto four hardware queues by default)
constexpr size_t kMaxJobsPerRound = 512;
// A round closes once its jobs hold this many neighbour entries (about 5 ms of
// census at the batched rate): rounds stay short, so a request admitted behind
// a full queue waits for a few short rounds instead of one long one.
constexpr uint64_t kMaxRoundEntries = 64ull << 20;
constexpr double kDefaultWatchdogMs = 60000.0;

struct serve_job : sched::job {
    tc_graph g = nullptr;                 // resident graph (not owned)
    bool cold = false;                    // arcs carried by the request, built on admission
    int32_t n = 0;
    uint32_t flags = 0;
    std::vector<int32_t> src, dst;
    device_graph built;                   // a cold job's graph, handed to the executor when the job ends
};

struct slot_buf {
    hipStream_t stream = nullptr;
    bool dead = false;                    // abandoned by the watchdog: never reused
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

void slot_free(slot_buf& s) {
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

// Grows the slot's buffers (geometrically, so this is rare).
hipError_t slot_reserve(slot_buf& s, uint32_t graphs, uint32_t items) {
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
uint64_t job_footprint(const serve_job& j) {
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

// The device side of the rounds: one stream and one set of staging buffers
// per slot, the batched persistent kernels, a host callback per round.  A
// round with requests to build goes to its slot's builder thread: a build
// waits on the device several times, and the scheduler's thread keeps
// launching rounds on the other slots meanwhile (the builds of different
// slots overlap as well).
class hip_executor : public sched::round_executor {
public:
    explicit hip_executor(tc_context_s* ctx) : ctx_(ctx) {
        for (int k = 0; k < kSlots; ++k) {
            launched_[k].store(0);
            issued_[k].store(0);
        }
    }
    ~hip_executor() override { stop_builder(); }
    sched::scheduler* sched = nullptr;    // set before the first launch
    slot_buf slots[kSlots];

    int slot_count() const override { return kSlots; }

    int launch(int si, std::vector<sched::job*>& jobs) override {
        bool cold = false;
        for (sched::job* jb : jobs) cold = cold || static_cast<serve_job*>(jb)->cold;
        if (!cold) return start_round(si, jobs, launched_[si].load());
        std::lock_guard<std::mutex> lk(bmu_);
        if (bstop_) return TC_ERR_SHUTDOWN;
        if (!builder_[si].joinable()) builder_[si] = std::thread([this, si] { builder_main(si); });
        const uint64_t gen = launched_[si].load() + 1;
        launched_[si].store(gen);   // not issued until the builder issues it
        pend_[si] = pending_round{gen, jobs};
        has_[si] = true;            // (a slot holds one round at a time)
        bcv_.notify_all();
        return TC_OK;
    }

    // Rounds are numbered per slot; the builder marks a round issued once its
    // work is on the stream (a late mark of an earlier round does not count).
    bool issued(int si) const override { return issued_[si].load() == launched_[si].load(); }

    // Ends the builder threads once their rounds are started.
    void stop_builder() {
        {
            std::lock_guard<std::mutex> lk(bmu_);
            bstop_ = true;
        }
        bcv_.notify_all();
        for (std::thread& t : builder_)
            if (t.joinable()) t.join();
    }

private:
    // Builds the round's cold requests, uploads its items and starts the
    // batched launch, the read-back and the completion callback on the
    // slot's stream.  TC_OK: round_done(si) follows from the callback.
    int start_round(int si, std::vector<sched::job*>& jobs, uint64_t gen) {
        slot_buf& s = slots[si];
        const tc_tuning tun = tuning_snapshot(ctx_);
        for (sched::job* jb : jobs) {
            serve_job* j = static_cast<serve_job*>(jb);
            if (!j->cold) continue;
            bucket_params bp = params_of(tun);
            bp.tri = 0;   // cold graphs live for one round: no forward lists (not in their footprint)
            j->status = build_into(j->n, (int64_t)j->src.size(), j->src.data(), j->dst.data(), j->flags, bp, s.stream,
                                   &j->built, nullptr);
            std::vector<int32_t>().swap(j->src);
            std::vector<int32_t>().swap(j->dst);
        }
        std::vector<work_item> items, rest;
        std::vector<graph_desc> descs(jobs.size());
        uint32_t hub_chunk = 0;
        for (size_t i = 0; i < jobs.size(); ++i) {
            serve_job* j = static_cast<serve_job*>(jobs[i]);
            if (j->status != TC_OK) {
                descs[i] = graph_desc{};
                continue;
            }
            const device_graph& g = j->cold ? j->built : j->g->g;
            descs[i] = describe(g);
            const bool tri = tun.tri && g.tri.fwd_ptr;
            append_items(g, (uint32_t)i, tri, items, rest);
            hub_chunk = std::max(hub_chunk, tri ? g.tri.edges.chunk : g.hub_chunk);
        }
        const uint32_t n_hub = (uint32_t)items.size();
        items.insert(items.end(), rest.begin(), rest.end());     // hub items first
        hipError_t e = slot_reserve(s, (uint32_t)jobs.size(), (uint32_t)items.size());
        if (e == hipSuccess) {
            std::memcpy(s.h_desc, descs.data(), sizeof(graph_desc) * descs.size());
            if (!items.empty()) std::memcpy(s.h_items, items.data(), sizeof(work_item) * items.size());
            s.h_num[0] = n_hub;
            s.h_num[1] = (uint32_t)items.size();
            e = hipMemcpyAsync(s.d_desc, s.h_desc, sizeof(graph_desc) * descs.size(), hipMemcpyHostToDevice,
                               s.stream);
            if (e == hipSuccess && !items.empty())
                e = hipMemcpyAsync(s.d_items, s.h_items, sizeof(work_item) * items.size(), hipMemcpyHostToDevice,
                                   s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.d_num, s.h_num, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, s.stream);
            // grids no larger than the round's items, so that small rounds
            // leave the rest of the GPU to the rounds beside them
            const uint32_t n_rest = (uint32_t)items.size() - n_hub;
            const uint32_t grid = std::max<uint32_t>(1u, std::min<uint32_t>(tun.batch_blocks, n_rest));
            const uint32_t hub_grid = std::max<uint32_t>(1u, std::min<uint32_t>(tun.hub_blocks, n_hub));
            if (e == hipSuccess)
                e = batch_launch(s.d_desc, s.d_items, s.d_num, s.d_accs, (uint64_t)kNumClasses * jobs.size(),
                                 s.d_ctr, grid, hub_grid, tun.hub_tile, tun.batch_tile, hub_chunk, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.h_accs, s.d_accs, sizeof(unsigned long long) * kNumClasses * jobs.size(),
                                   hipMemcpyDeviceToHost, s.stream);
            if (e == hipSuccess) e = hipLaunchHostFunc(s.stream, on_round_done, new cb_arg{this, si});
        }
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s.stream);
            return status_from_hip(e);
        }
        issued_[si].store(gen);
        return TC_OK;
    }

    struct pending_round {
        uint64_t gen = 0;
        std::vector<sched::job*> jobs;
    };

    void builder_main(int si) {
        std::unique_lock<std::mutex> lk(bmu_);
        for (;;) {
            bcv_.wait(lk, [&] { return bstop_ || has_[si]; });
            if (!has_[si]) return;   // stopping, nothing left
            pending_round p = std::move(pend_[si]);
            busy_[si] = true;
            has_[si] = false;
            lk.unlock();
            const int rc = start_round(si, p.jobs, p.gen);
            if (rc != TC_OK) {
                // nothing runs (and the watchdog never timed the round, so its
                // jobs are still the scheduler's): it completes now with rc
                for (sched::job* j : p.jobs)
                    if (j->status == TC_OK) j->status = rc;
                issued_[si].store(p.gen);
                sched->round_done(si);
            }
            lk.lock();
            busy_[si] = false;
            bcv_.notify_all();
        }
    }

public:

    void collect(int si, std::vector<sched::job*>& jobs) override {
        for (size_t i = 0; i < jobs.size(); ++i) {
            serve_job* j = static_cast<serve_job*>(jobs[i]);
            if (j->status != TC_OK) continue;
            const int32_t n = j->cold ? j->built.n : j->g->g.n;
            finalize_counts(n, slots[si].h_accs + kNumClasses * i, j->counts);
        }
    }

    void job_done(sched::job* jb) override {
        serve_job* j = static_cast<serve_job*>(jb);
        if (!j->cold) {
            j->g->pending.fetch_sub(1);
            return;
        }
        if (j->built.nbr || j->built.row_ptr) {
            std::lock_guard<std::mutex> lk(held_mu_);
            held_bytes_ += device_graph_bytes(j->built);
            held_.push_back(j->built);
            j->built = device_graph{};
        }
    }

    // Graphs built for cold requests are freed when no round is in flight (a
    // free synchronises the device and would stall the rounds), or once they
    // hold a quarter of the budget.
    void release(bool idle) override {
        std::vector<device_graph> out;
        {
            std::lock_guard<std::mutex> lk(held_mu_);
            if (held_.empty() || (!idle && held_bytes_ < ctx_->budget / 4)) return;
            out.swap(held_);
        }
        uint64_t freed = 0;
        for (device_graph& g : out) {
            freed += device_graph_bytes(g);
            free_device_graph(&g);
        }
        std::lock_guard<std::mutex> lk(held_mu_);
        held_bytes_ -= freed;
    }

    uint64_t held_bytes() const override {
        std::lock_guard<std::mutex> lk(held_mu_);
        return held_bytes_;
    }

    void abandon(int si) override { slots[si].dead = true; }

    void drain() override {
        {
            std::unique_lock<std::mutex> lk(bmu_);
            bcv_.wait(lk, [&] {
                for (int k = 0; k < kSlots; ++k)
                    if (has_[k] || busy_[k]) return false;
                return true;
            });
        }
        for (slot_buf& s : slots)
            if (!s.dead) (void)hipStreamSynchronize(s.stream);
    }

private:
    struct cb_arg {
        hip_executor* ex;
        int slot;
    };
    // Host callback after a round's read-back.  It must not block: the stream
    // (and anything that synchronises the device) waits for it.
    static void on_round_done(void* arg) {
        cb_arg* a = static_cast<cb_arg*>(arg);
        a->ex->sched->round_done(a->slot);
        delete a;
    }

    tc_context_s* ctx_;
    mutable std::mutex held_mu_;
    std::vector<device_graph> held_;
    uint64_t held_bytes_ = 0;
    // builder threads, one per slot: the round with requests to build that
    // the slot holds, if any
    std::atomic<uint64_t> launched_[kSlots], issued_[kSlots];
    std::mutex bmu_;
    std::condition_variable bcv_;
    pending_round pend_[kSlots];
    bool has_[kSlots] = {}, busy_[kSlots] = {}, bstop_ = false;
    std::thread builder_[kSlots];
};

}  // namespace

struct serve_state {
    explicit serve_state(tc_context_s* ctx) : ex(ctx) {}
    hip_executor ex;
    std::unique_ptr<sched::scheduler> S;
};

namespace {

serve_state* ensure_serving(tc_context_s* ctx, int* rc) {
    *rc = TC_OK;
    if (ctx->serve) return ctx->serve;
    serve_state* st = new (std::nothrow) serve_state(ctx);
    if (!st) {
        *rc = TC_ERR_NOMEM;
        return nullptr;
    }
    for (slot_buf& s : st->ex.slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            for (slot_buf& t : st->ex.slots)
                if (t.stream) (void)hipStreamDestroy(t.stream);
            delete st;
            *rc = TC_ERR_DEVICE;
            return nullptr;
        }
    }
    sched::sched_limits lim;
    lim.budget = ctx->budget;
    lim.max_jobs_per_round = kMaxJobsPerRound;
    lim.max_round_entries = kMaxRoundEntries;
    lim.watchdog_ms = ctx->watchdog_ms > 0 ? ctx->watchdog_ms : kDefaultWatchdogMs;
    lim.max_build_rounds = kSlots / 2;   // the other slots stay free for resident graphs
    st->ex.sched = nullptr;
    try {
        st->S.reset(new sched::scheduler(&st->ex, lim));
    } catch (...) {
        for (slot_buf& t : st->ex.slots) (void)hipStreamDestroy(t.stream);
        delete st;
        *rc = TC_ERR_NOMEM;
        return nullptr;
    }
    st->ex.sched = st->S.get();           // before any job is submitted, so before any launch
    ctx->serve = st;
    return st;
}

}  // namespace

// Stops the scheduler; queued tickets end with TC_ERR_SHUTDOWN (still pollable).
void serve_stop(tc_context_s* ctx) {
    if (ctx->serve) ctx->serve->S->stop();
}

void serve_shutdown(tc_context_s* ctx) {
    serve_state* st = ctx->serve;
    if (!st) return;
    st->S->stop();
    st->ex.stop_builder();
    // rounds the watchdog gave up on may still call back into the scheduler
    for (slot_buf& s : st->ex.slots)
        if (s.stream) (void)hipStreamSynchronize(s.stream);
    st->S.reset();                        // frees the jobs left unpolled
    for (slot_buf& s : st->ex.slots) {
        slot_free(s);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    st->ex.release(true);
    delete st;
    ctx->serve = nullptr;
}

}  // namespace tc

using namespace tc;

namespace {

int submit_job(tc_context ctx, serve_job* j, tc_ticket* out) {
    int rc;
    serve_state* st;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = ensure_serving(ctx, &rc);
    }
    if (!st) {
        if (!j->cold) j->g->pending.fetch_sub(1);
        delete j;
        return rc;
    }
    j->footprint = job_footprint(*j);
    j->entries = j->cold ? 2 * (uint64_t)j->src.size() : j->g->g.U;
    uint64_t ticket = 0;
    rc = st->S->submit(j, &ticket);       // owns j from here, also on error
    if (rc == TC_OK) *out = ticket;
    return rc;
}

}  // namespace

extern "C" int tc_submit(tc_context ctx, tc_graph g, tc_ticket* out) {
    if (!ctx || !g || !out) return TC_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->graphs.count(g)) return TC_ERR_ARG;
        g->pending.fetch_add(1);
    }
    serve_job* j = new (std::nothrow) serve_job();
    if (!j) {
        g->pending.fetch_sub(1);
        return TC_ERR_NOMEM;
    }
    j->g = g;
    return submit_job(ctx, j, out);
}

extern "C" int tc_submit_arcs(tc_context ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              uint32_t flags, tc_ticket* out) {
    if (!ctx || !out || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return TC_ERR_ARG;
    if (flags & ~(uint32_t)TC_BUILD_STRICT) return TC_ERR_ARG;
    if (n > kMaxN) return TC_ERR_RANGE;
    serve_job* j = new (std::nothrow) serve_job();
    if (!j) return TC_ERR_NOMEM;
    j->cold = true;
    j->builds = true;   // its round runs no resident request
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
    serve_state* st = ctx->serve;
    if (!st) return TC_ERR_NOT_FOUND;
    return st->S->poll(ticket, counts, done);
}

extern "C" int tc_serve_stop(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    serve_stop(ctx);
    return TC_OK;
}

extern "C" int tc_serve_set_watchdog_ms(tc_context ctx, double ms) {
    if (!ctx || !(ms > 0)) return TC_ERR_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->watchdog_ms = ms;
    if (ctx->serve) ctx->serve->S->set_watchdog_ms(ms);
    return TC_OK;
}

extern "C" int tc_serve_get_stats(tc_context ctx, tc_serve_stats* out) {
    if (!ctx || !out) return TC_ERR_ARG;
    *out = tc_serve_stats{};
    serve_state* st = ctx->serve;
    if (!st) return TC_OK;
    const sched::sched_stats s = st->S->stats();
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->rounds = s.rounds;
    out->bytes_in_flight = s.bytes_in_flight;
    out->p50_ms = s.p50_ms;
    out->p99_ms = s.p99_ms;
    out->mean_admission_ms = s.mean_admission_ms;
    out->failed_rounds = s.failed_rounds;
    out->abandoned_rounds = s.abandoned_rounds;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        out->resident_graphs = ctx->graphs.size();
    }
    return TC_OK;
}

extern "C" int tc_serve_reset_stats(tc_context ctx) {
    if (!ctx) return TC_ERR_ARG;
    serve_state* st = ctx->serve;
    if (st) st->S->reset_stats();
    return TC_OK;
}
