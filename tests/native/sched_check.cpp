// Host-only checks of the serving scheduler (paper_1603_02655_amd/csrc/tc_sched.cpp)
// driven by a fake round executor: rounds "run" on threads that sleep, and
// faults are injected on demand (a launch that fails, a build error, a round
// that never finishes, a round held until the test lets it go).  No GPU, no
// census arithmetic: a job's counts are a function of its graph id, so the
// checks are about routing, admission, ordering, failure handling and
// shutdown.  Built and run by tests/test_native_sanitizers.py, also under ASan/UBSan and
// TSan.  Exit status 0 when every scenario passes.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "tc_sched.h"

using namespace tc::sched;

static int g_failures = 0;
#define CHECK(cond)                                                                      \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_failures;                                                                \
        }                                                                                \
    } while (0)

static void sleep_ms(double ms) { std::this_thread::sleep_for(std::chrono::microseconds((long)(ms * 1000))); }

struct fake_job : job {
    int graph = 0;
    double delay_ms = 0;       // how long the round of this job takes (the round takes its longest)
    bool build_fails = false;  // the executor reports a build error for it
    bool cold = false;         // holds `footprint` bytes after it ends, until release()
    bool hold = false;         // its round finishes only when the test lets it go
    bool hang = false;         // its round never finishes
    double prepare_ms = 0;     // its round issues its work only after this long (a build first)
};

class fake_exec : public round_executor {
public:
    fake_exec(int slots, uint64_t budget) : slots_(slots), budget_(budget), in_flight_(slots, 0) {}
    ~fake_exec() override { join_all(); }
    scheduler* S = nullptr;
    int fail_launch_at = -1;   // 1-based launch index that fails with kErrNoMem

    int slot_count() const override { return slots_; }

    // a round being prepared has not issued its work yet
    bool issued(int slot) const override { return now_ms() >= issue_at_[slot].load(); }

    int launch(int slot, std::vector<job*>& jobs) override {
        std::lock_guard<std::mutex> lk(mu_);
        ++launches_;
        CHECK(slot >= 0 && slot < slots_);
        CHECK(!in_flight_[(size_t)slot]);   // never two rounds on one slot
        // admission invariant: what is admitted plus what is held fits the budget
        uint64_t fp = 0;
        double delay = 0, prep = 0;
        bool hold = false, hang = false;
        for (job* jb : jobs) {
            fake_job* j = static_cast<fake_job*>(jb);
            CHECK(j->state == kRunning);
            CHECK(j->builds == jobs[0]->builds);   // a round holds one kind of job
            fp += j->footprint;
            delay = std::max(delay, j->delay_ms);
            prep = std::max(prep, j->prepare_ms);
            hold = hold || j->hold;
            hang = hang || j->hang;
            if (j->build_fails) j->status = -1;
        }
        admitted_bytes_ += fp;
        CHECK(admitted_bytes_ + held_ <= budget_);
        if (launches_ == fail_launch_at) {
            for (job* jb : jobs) jb->status = kOk;   // the scheduler gives them the launch's error
            return kErrNoMem;
        }
        max_round_ = std::max<size_t>(max_round_, jobs.size());
        in_flight_[(size_t)slot] = fp + 1;
        issue_at_[slot].store(now_ms() + prep);
        if (hang) return kOk;                 // round_done is never called
        threads_.emplace_back([this, slot, delay, hold, prep] {
            sleep_ms(prep);
            if (hold) {
                std::unique_lock<std::mutex> l2(hold_mu_);
                hold_cv_.wait(l2, [this] { return released_; });
            }
            sleep_ms(delay);
            {
                std::lock_guard<std::mutex> l3(mu_);
                in_flight_[(size_t)slot] = 0;
            }
            S->round_done(slot);
        });
        return kOk;
    }

    void collect(int slot, std::vector<job*>& jobs) override {
        (void)slot;
        for (job* jb : jobs) {
            fake_job* j = static_cast<fake_job*>(jb);
            if (j->status != kOk) continue;
            for (int k = 0; k < 16; ++k) j->counts[k] = (uint64_t)j->graph * 100 + (uint64_t)k;
        }
    }

    void job_done(job* jb) override {
        fake_job* j = static_cast<fake_job*>(jb);
        std::lock_guard<std::mutex> lk(mu_);
        done_tickets_.insert(j->ticket);
        pending_[j->graph] -= 1;
        if (j->state == kDone && j->t_admit > 0) admitted_bytes_ -= j->footprint;
        if (j->cold && j->t_admit > 0) held_ += j->footprint;
    }

    void release(bool idle) override {
        std::lock_guard<std::mutex> lk(mu_);
        if (idle || held_ >= budget_ / 4) held_ = 0;
    }

    uint64_t held_bytes() const override {
        std::lock_guard<std::mutex> lk(mu_);
        return held_;
    }

    void abandon(int slot) override {
        std::lock_guard<std::mutex> lk(mu_);
        dead_.insert(slot);
        in_flight_[(size_t)slot] = 0;   // the slot is never launched on again
        ++abandoned_;
    }

    // The rounds that can finish (held ones once the test lets them go; hung
    // ones never do and have no thread).
    void drain() override {
        std::vector<std::thread> ts;
        {
            std::lock_guard<std::mutex> lk(mu_);
            ts.swap(threads_);
        }
        for (auto& t : ts) t.join();
    }

    // test side
    void let_go() {
        {
            std::lock_guard<std::mutex> lk(hold_mu_);
            released_ = true;
        }
        hold_cv_.notify_all();
    }
    void join_all() {
        let_go();
        std::vector<std::thread> ts;
        {
            std::lock_guard<std::mutex> lk(mu_);
            ts.swap(threads_);
        }
        for (auto& t : ts) t.join();
    }
    void add_pending(int graph) {
        std::lock_guard<std::mutex> lk(mu_);
        pending_[graph] += 1;
    }
    int pending(int graph) {
        std::lock_guard<std::mutex> lk(mu_);
        return pending_[graph];
    }
    bool was_done(uint64_t t) {
        std::lock_guard<std::mutex> lk(mu_);
        return done_tickets_.count(t) != 0;
    }
    int launches() {
        std::lock_guard<std::mutex> lk(mu_);
        return launches_;
    }
    size_t max_round() {
        std::lock_guard<std::mutex> lk(mu_);
        return max_round_;
    }
    int abandoned() {
        std::lock_guard<std::mutex> lk(mu_);
        return abandoned_;
    }

private:
    int slots_;
    uint64_t budget_;
    mutable std::mutex mu_;
    std::vector<uint64_t> in_flight_;
    std::vector<std::thread> threads_;
    std::map<int, int> pending_;
    std::set<uint64_t> done_tickets_;
    std::set<int> dead_;
    uint64_t admitted_bytes_ = 0, held_ = 0;
    size_t max_round_ = 0;
    int launches_ = 0, abandoned_ = 0;
    std::mutex hold_mu_;
    std::condition_variable hold_cv_;
    bool released_ = false;
    std::atomic<double> issue_at_[16] = {};
};

struct harness {
    harness(int slots, uint64_t budget, double watchdog_ms = 60000.0, size_t max_jobs = 512, size_t max_build = 0)
        : ex(slots, budget) {
        sched_limits lim;
        lim.budget = budget;
        lim.watchdog_ms = watchdog_ms;
        lim.max_jobs_per_round = max_jobs;
        lim.max_build_rounds = max_build;
        S = new scheduler(&ex, lim);
        ex.S = S;
    }
    ~harness() {
        ex.let_go();
        delete S;          // stops the worker (and waits for the rounds it can)
        ex.join_all();
    }
    uint64_t submit(fake_job* j) {
        ex.add_pending(j->graph);
        uint64_t t = 0;
        const int rc = S->submit(j, &t);
        CHECK(rc == kOk);
        return t;
    }
    // waits until the executor has started k rounds
    void wait_launches(int k) {
        const double t0 = now_ms();
        while (ex.launches() < k) {
            if (now_ms() - t0 > 20000.0) {
                CHECK(!"round did not start in time");
                return;
            }
            sleep_ms(0.05);
        }
    }
    // polls until done or timeout; returns the status, fills counts
    int wait(uint64_t ticket, uint64_t counts[16], double timeout_ms = 20000.0) {
        const double t0 = now_ms();
        for (;;) {
            int done = 0;
            const int rc = S->poll(ticket, counts, &done);
            if (done || rc == kErrNotFound) return rc;
            if (now_ms() - t0 > timeout_ms) {
                CHECK(!"ticket did not finish in time");
                return -100;
            }
            sleep_ms(0.05);
        }
    }
    fake_exec ex;
    scheduler* S;
};

static fake_job* mk(int graph, uint64_t fp, double delay = 0.0) {
    fake_job* j = new fake_job();
    j->graph = graph;
    j->footprint = fp;
    j->entries = 1000;
    j->delay_ms = delay;
    return j;
}

// Many jobs from several threads: every result belongs to its own graph, every
// pending count returns to zero, the counters add up.
static void scenario_basic() {
    harness h(3, 1ull << 30);
    std::mutex mu;
    std::vector<std::pair<uint64_t, int>> tickets;
    std::vector<std::thread> subs;
    for (int s = 0; s < 4; ++s) {
        subs.emplace_back([&, s] {
            std::mt19937 rng(s + 1);
            for (int k = 0; k < 100; ++k) {
                const int graph = (int)(rng() % 10);
                const uint64_t t = h.submit(mk(graph, 100 + rng() % 1000, (rng() % 20) / 10.0));
                std::lock_guard<std::mutex> lk(mu);
                tickets.emplace_back(t, graph);
                if (k % 10 == 0) sleep_ms(0.2);
            }
        });
    }
    for (auto& t : subs) t.join();
    for (auto& tg : tickets) {
        uint64_t c[16];
        CHECK(h.wait(tg.first, c) == kOk);
        for (int k = 0; k < 16; ++k) CHECK(c[k] == (uint64_t)tg.second * 100 + (uint64_t)k);
        int done = 0;
        CHECK(h.S->poll(tg.first, c, &done) == kErrNotFound);   // retired
    }
    for (int g = 0; g < 10; ++g) CHECK(h.ex.pending(g) == 0);
    const sched_stats st = h.S->stats();
    CHECK(st.submitted == 400 && st.completed == 400);
    CHECK(st.rounds >= 1 && st.rounds <= 400 && st.failed_rounds == 0 && st.abandoned_rounds == 0);
    CHECK(st.bytes_in_flight == 0);
    CHECK(st.p50_ms > 0 && st.p50_ms <= st.p99_ms);
    std::printf("ok basic: 400 jobs in %llu rounds, p50 %.3f ms, p99 %.3f ms\n", (unsigned long long)st.rounds,
                st.p50_ms, st.p99_ms);
}

// Admission by footprint: a job larger than the budget fails with kErrNoMem
// at once; the others run with what is in flight never above the budget (the
// executor checks at every launch).
static void scenario_budget() {
    harness h(3, 1000);
    std::vector<std::pair<uint64_t, int>> t;
    std::mt19937 rng(7);
    for (int k = 0; k < 200; ++k) t.emplace_back(h.submit(mk(k % 5, 1 + rng() % 400, 0.3)), 0);
    const uint64_t big = h.submit(mk(9, 5000));
    for (int k = 0; k < 50; ++k) t.emplace_back(h.submit(mk(k % 5, 1 + rng() % 400, 0.1)), 0);
    uint64_t c[16];
    CHECK(h.wait(big, c) == kErrNoMem);
    for (auto& x : t) CHECK(h.wait(x.first, c) == kOk);
    CHECK(h.ex.pending(9) == 0);
    std::printf("ok budget: largest round %zu jobs\n", h.ex.max_round());
}

// A launch that fails: its jobs get the error, the following rounds run.
static void scenario_launch_failure() {
    harness h(1, 1ull << 30, 60000.0, 4);
    h.ex.fail_launch_at = 2;
    std::vector<uint64_t> t;
    for (int k = 0; k < 16; ++k) t.push_back(h.submit(mk(1, 10, 0.5)));
    int ok = 0, nomem = 0;
    for (uint64_t x : t) {
        uint64_t c[16];
        const int rc = h.wait(x, c);
        ok += rc == kOk;
        nomem += rc == kErrNoMem;
    }
    CHECK(nomem >= 1 && nomem <= 4 && ok + nomem == 16);
    CHECK(h.S->stats().failed_rounds == 1);
    CHECK(h.ex.pending(1) == 0);
    std::printf("ok launch failure: %d failed, %d ran\n", nomem, ok);
}

// A build error fails that job only; the rest of its round runs.
static void scenario_build_error() {
    harness h(2, 1ull << 30);
    std::vector<std::pair<uint64_t, bool>> t;
    for (int k = 0; k < 40; ++k) {
        fake_job* j = mk(k % 3, 10, 0.2);
        j->build_fails = k % 7 == 3;
        t.emplace_back(h.submit(j), j->build_fails);
    }
    for (auto& x : t) {
        uint64_t c[16];
        CHECK(h.wait(x.first, c) == (x.second ? -1 : kOk));
    }
    std::printf("ok build error\n");
}

// A round that never finishes: after the watchdog its jobs fail with
// kErrDevice and its slot is dropped; the other slots keep serving.  When
// every slot is lost, queued and new jobs fail with kErrDevice.
static void scenario_watchdog() {
    harness h(3, 1ull << 30, 50.0);
    fake_job* stuck = mk(4, 10);
    stuck->hang = true;
    const uint64_t ts = h.submit(stuck);
    sleep_ms(5);
    std::vector<uint64_t> t;
    for (int k = 0; k < 30; ++k) t.push_back(h.submit(mk(5, 10, 0.2)));
    uint64_t c[16];
    for (uint64_t x : t) CHECK(h.wait(x, c) == kOk);
    const double t0 = now_ms();
    CHECK(h.wait(ts, c) == kErrDevice);
    CHECK(now_ms() - t0 < 5000);
    CHECK(h.S->stats().abandoned_rounds == 1 && h.ex.abandoned() == 1);
    CHECK(h.ex.pending(4) == 0);
    // lose the two remaining slots
    for (int k = 0; k < 2; ++k) {
        fake_job* j = mk(6, 10);
        j->hang = true;
        const uint64_t x = h.submit(j);
        sleep_ms(20);      // in a round of its own
        (void)x;
    }
    sleep_ms(200);
    CHECK(h.S->stats().abandoned_rounds == 3);
    const uint64_t late = h.submit(mk(7, 10));
    CHECK(h.wait(late, c) == kErrDevice);
    std::printf("ok watchdog\n");
}

// A round still being prepared (its work not yet issued) is not timed by the
// watchdog: a preparation far longer than the watchdog completes normally;
// once a round has issued its work and then hangs, the watchdog drops it.
static void scenario_watchdog_after_issue() {
    harness h(2, 1ull << 30, 40.0);
    fake_job* slow = mk(8, 10, 2.0);
    slow->prepare_ms = 150.0;
    const uint64_t ts = h.submit(slow);
    uint64_t c[16];
    CHECK(h.wait(ts, c) == kOk);
    CHECK(h.S->stats().abandoned_rounds == 0);
    fake_job* stuck = mk(9, 10);
    stuck->prepare_ms = 100.0;
    stuck->hang = true;
    const double t0 = now_ms();
    const uint64_t tk = h.submit(stuck);
    CHECK(h.wait(tk, c) == kErrDevice);
    CHECK(now_ms() - t0 >= 100.0 + 40.0 - 5.0);   // not before it issued its work plus the watchdog
    CHECK(h.S->stats().abandoned_rounds == 1);
    std::printf("ok watchdog after issue\n");
}

// While a graph has a job in flight its pending count is positive (the C API
// returns TC_ERR_BUSY on release then); it drops to zero exactly when the
// ticket is done.
static void scenario_busy_contract() {
    harness h(1, 1ull << 30);
    fake_job* j = mk(8, 10);
    j->hold = true;
    const uint64_t t = h.submit(j);
    sleep_ms(20);
    CHECK(h.ex.pending(8) == 1);          // release would return TC_ERR_BUSY
    uint64_t c[16];
    int done = 1;
    CHECK(h.S->poll(t, c, &done) == kOk && done == 0);
    h.ex.let_go();
    CHECK(h.wait(t, c) == kOk);
    CHECK(h.ex.pending(8) == 0);          // now release succeeds
    std::printf("ok busy contract\n");
}

// Stop: the round in flight finishes, queued jobs end with kErrShutdown,
// later submissions are refused, unknown tickets are not found.
static void scenario_stop() {
    harness h(1, 1ull << 30, 60000.0, 1);
    fake_job* first = mk(1, 10);
    first->hold = true;
    const uint64_t t1 = h.submit(first);
    sleep_ms(10);
    const uint64_t t2 = h.submit(mk(2, 10));
    const uint64_t t3 = h.submit(mk(3, 10));
    std::thread stopper([&] { h.S->stop(); });
    sleep_ms(20);
    h.ex.let_go();
    stopper.join();
    uint64_t c[16];
    CHECK(h.wait(t1, c) == kOk);
    CHECK(h.wait(t2, c) == kErrShutdown);
    CHECK(h.wait(t3, c) == kErrShutdown);
    fake_job* late = mk(4, 10);
    h.ex.add_pending(4);
    uint64_t t4 = 0;
    CHECK(h.S->submit(late, &t4) == kErrShutdown);
    int done = 0;
    CHECK(h.S->poll(987654321ull, c, &done) == kErrNotFound);
    for (int g = 1; g <= 4; ++g) CHECK(h.ex.pending(g) == 0);
    std::printf("ok stop\n");
}

// Arrival order: a job that does not fit yet holds back the ones behind it
// (no overtaking), so admission follows the tickets and a large job is not
// starved by a stream of small ones.
static void scenario_fifo() {
    harness h(3, 100);
    std::vector<fake_job*> js;
    std::vector<uint64_t> t;
    for (int k = 0; k < 60; ++k) {
        fake_job* j = mk(k % 4, k % 10 == 5 ? 90 : 5 + (uint64_t)(k % 7), 0.3);
        js.push_back(j);
        t.push_back(h.submit(j));
    }
    // admission times are read from the fake jobs before they are polled away
    std::vector<double> admit(t.size());
    uint64_t c[16];
    for (size_t k = 0; k < t.size(); ++k) {
        for (;;) {
            // wait until done, remember t_admit, then poll
            if (h.ex.was_done(t[k])) break;
            sleep_ms(0.05);
        }
        admit[k] = js[k]->t_admit;
        CHECK(h.wait(t[k], c) == kOk);
    }
    for (size_t k = 1; k < admit.size(); ++k) CHECK(admit[k] >= admit[k - 1]);
    std::printf("ok fifo\n");
}

// Rounds hold one kind of job: a resident job never shares the round of a job
// whose graph is built first, jobs of the other kind keep their place, and the
// first queued job opens each round.
static void scenario_kinds() {
    harness h(1, 1ull << 30);
    fake_job* first = mk(0, 10);
    first->hold = true;
    const uint64_t t0 = h.submit(first);
    h.wait_launches(1);                    // its round holds the one slot: the rest queue up
    std::vector<fake_job*> js;
    std::vector<uint64_t> t;
    for (int k = 0; k < 6; ++k) {
        fake_job* j = mk(k + 1, 10);
        j->builds = k % 3 == 1;            // resident, builds, resident, resident, builds, resident
        js.push_back(j);
        t.push_back(h.submit(j));
    }
    h.ex.let_go();
    uint64_t c[16];
    CHECK(h.wait(t0, c) == kOk);
    std::vector<double> admit(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
        while (!h.ex.was_done(t[k])) sleep_ms(0.05);
        admit[k] = js[k]->t_admit;         // read before the poll retires the job
        CHECK(h.wait(t[k], c) == kOk);
        for (int q = 0; q < 16; ++q) CHECK(c[q] == (uint64_t)(k + 1) * 100 + (uint64_t)q);
    }
    // the four resident jobs in one round, then the two that build in the next
    CHECK(admit[0] == admit[2] && admit[0] == admit[3] && admit[0] == admit[5]);
    CHECK(admit[1] == admit[4] && admit[1] > admit[0]);
    CHECK(h.ex.launches() == 3);
    std::printf("ok kinds\n");
}

// The same with a job that builds at the front of the queue: it opens the
// round (with the other job that builds), the resident jobs follow.
static void scenario_kinds_build_first() {
    harness h(1, 1ull << 30);
    fake_job* first = mk(0, 10);
    first->hold = true;
    const uint64_t t0 = h.submit(first);
    h.wait_launches(1);
    std::vector<fake_job*> js;
    std::vector<uint64_t> t;
    for (int k = 0; k < 4; ++k) {
        fake_job* j = mk(k + 1, 10);
        j->builds = k == 0 || k == 3;      // builds, resident, resident, builds
        js.push_back(j);
        t.push_back(h.submit(j));
    }
    h.ex.let_go();
    uint64_t c[16];
    CHECK(h.wait(t0, c) == kOk);
    std::vector<double> admit(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
        while (!h.ex.was_done(t[k])) sleep_ms(0.05);
        admit[k] = js[k]->t_admit;
        CHECK(h.wait(t[k], c) == kOk);
    }
    CHECK(admit[0] == admit[3] && admit[1] == admit[2] && admit[1] > admit[0]);
    CHECK(h.ex.launches() == 3);
    std::printf("ok kinds, build first\n");
}

// At most max_build_rounds rounds build at once: a job that builds waits at
// the front while the resident jobs behind it run, and it opens the round
// after the building one ends.
static void scenario_build_rounds_capped() {
    harness h(3, 1ull << 30, 60000.0, 512, 1);
    fake_job* b1 = mk(1, 10);
    b1->builds = true;
    b1->hold = true;
    const uint64_t t1 = h.submit(b1);
    h.wait_launches(1);                    // b1's round builds on one slot
    fake_job* b2 = mk(2, 10);
    b2->builds = true;
    const uint64_t t2 = h.submit(b2);
    const uint64_t t3 = h.submit(mk(3, 10));
    const uint64_t t4 = h.submit(mk(4, 10));
    uint64_t c[16];
    CHECK(h.wait(t3, c) == kOk);           // resident jobs run while b1 still builds
    CHECK(h.wait(t4, c) == kOk);
    CHECK(!h.ex.was_done(t1) && !h.ex.was_done(t2));
    sleep_ms(10);
    CHECK(!h.ex.was_done(t2));             // the one build slot is still taken
    h.ex.let_go();
    CHECK(h.wait(t1, c) == kOk);
    CHECK(h.wait(t2, c) == kOk);
    for (int q = 0; q < 16; ++q) CHECK(c[q] == 200u + (uint64_t)q);
    CHECK(h.ex.launches() >= 3);           // (the resident jobs may have run in two rounds)
    std::printf("ok build rounds capped\n");
}

// Cold jobs hold their bytes after they end until the executor releases them
// (when idle, or past a quarter of the budget); admission counts them.
static void scenario_held_bytes() {
    harness h(2, 1000);
    std::vector<uint64_t> t;
    for (int k = 0; k < 50; ++k) {
        fake_job* j = mk(k % 2, 150, 0.2);
        j->cold = true;
        t.push_back(h.submit(j));
    }
    uint64_t c[16];
    for (uint64_t x : t) CHECK(h.wait(x, c) == kOk);
    sleep_ms(20);
    CHECK(h.ex.held_bytes() == 0);        // released once idle
    std::printf("ok held bytes\n");
}

static void scenario_histogram() {
    latency_hist hist;
    CHECK(hist.percentile(0.5) == 0.0);
    for (int k = 1; k <= 1000; ++k) hist.add((double)k);      // 1 .. 1000 ms
    const double p50 = hist.percentile(0.50), p99 = hist.percentile(0.99);
    CHECK(p50 >= 500.0 && p50 <= 500.0 * 1.037);
    CHECK(p99 >= 990.0 && p99 <= 990.0 * 1.037);
    hist.add(0.0);
    hist.add(1e9);
    CHECK(hist.count() == 1002);
    hist.clear();
    CHECK(hist.count() == 0);
    std::printf("ok histogram: p50 %.2f p99 %.2f\n", p50, p99);
}

int main() {
    scenario_histogram();
    scenario_basic();
    scenario_budget();
    scenario_launch_failure();
    scenario_build_error();
    scenario_watchdog();
    scenario_watchdog_after_issue();
    scenario_busy_contract();
    scenario_stop();
    scenario_fifo();
    scenario_kinds();
    scenario_kinds_build_first();
    scenario_build_rounds_capped();
    scenario_held_bytes();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("all scheduler scenarios passed\n");
    return 0;
}
