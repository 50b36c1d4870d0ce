// Scheduler of the serving loop (see tc_sched.h).
#include "tc_sched.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace tc {
namespace sched {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// latency histogram

void latency_hist::add(double ms) {
    int k = 0;
    if (ms >= 1e-3) {
        const double x = std::floor((std::log10(ms) + 3.0) * kPerDecade);
        k = 1 + (int)std::min<double>(x, kBuckets - 2);
    }
    n_[k] += 1;
    total_ += 1;
}

double latency_hist::percentile(double q) const {
    if (total_ == 0) return 0.0;
    const uint64_t rank = std::max<uint64_t>(1, (uint64_t)std::ceil(q * (double)total_));
    uint64_t seen = 0;
    for (int k = 0; k < kBuckets; ++k) {
        seen += n_[k];
        if (seen >= rank) return k == 0 ? 1e-3 : std::pow(10.0, (double)k / kPerDecade - 3.0);
    }
    return std::pow(10.0, (double)(kBuckets - 1) / kPerDecade - 3.0);
}

void latency_hist::clear() {
    std::memset(n_, 0, sizeof(n_));
    total_ = 0;
}

// ---------------------------------------------------------------------------
// scheduler

scheduler::scheduler(round_executor* ex, const sched_limits& lim)
    : ex_(ex), lim_(lim), slots_((size_t)std::max(1, ex->slot_count())) {
    worker_ = std::thread(&scheduler::worker_main, this);
}

scheduler::~scheduler() {
    stop();
    for (auto& kv : jobs_) {
        // every job is done once the worker has stopped; job_done was called
        delete kv.second;
    }
    jobs_.clear();
}

int scheduler::submit(job* j, uint64_t* ticket) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) {
            ex_->job_done(j);
            delete j;
            return kErrShutdown;
        }
        j->ticket = next_ticket_++;
        j->t_submit = now_ms();
        j->state = kQueued;
        j->status = kOk;
        jobs_[j->ticket] = j;
        queue_.push_back(j);
        st_.submitted += 1;
        *ticket = j->ticket;
    }
    cv_.notify_all();
    return kOk;
}

int scheduler::poll(uint64_t ticket, uint64_t counts[16], int* done) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return kErrNotFound;
    job* j = it->second;
    if (j->state != kDone) {
        *done = 0;
        return stop_ ? kErrShutdown : kOk;
    }
    const int st = j->status;
    if (st == kOk) std::memcpy(counts, j->counts, sizeof(j->counts));
    *done = 1;
    jobs_.erase(it);
    delete j;
    return st;
}

void scheduler::round_done(int slot) {
    if (slot >= 0 && slot < (int)slots_.size()) slots_[(size_t)slot].finished.store(true);
    cv_.notify_all();
}

void scheduler::stop() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
}

bool scheduler::stopped() {
    std::lock_guard<std::mutex> lk(mu_);
    return stop_;
}

sched_stats scheduler::stats() {
    std::lock_guard<std::mutex> lk(mu_);
    sched_stats s = st_;
    s.bytes_in_flight = bytes_in_flight_;
    s.p50_ms = lat_.percentile(0.50);
    s.p99_ms = lat_.percentile(0.99);
    s.mean_admission_ms = admitted_ ? admission_ms_sum_ / (double)admitted_ : 0.0;
    return s;
}

void scheduler::reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    st_ = sched_stats{};
    lat_.clear();
    admission_ms_sum_ = 0;
    admitted_ = 0;
}

void scheduler::set_watchdog_ms(double ms) {
    std::lock_guard<std::mutex> lk(mu_);
    lim_.watchdog_ms = ms;
}

// A job leaves the scheduler: its status is final and it can be polled.
void scheduler::complete_locked(job* j, int status, double t, std::vector<job*>& retired) {
    const bool ran = j->state == kRunning;
    if (ran) bytes_in_flight_ -= j->footprint;
    j->status = status;
    j->state = kDone;
    j->t_done = t;
    st_.completed += 1;
    if (ran) lat_.add(t - j->t_submit);   // latency of the jobs that were admitted
    ex_->job_done(j);
    retired.push_back(j);
}

// Moves queued jobs into slot s in arrival order while their footprint fits
// the budget (with what is in flight and what the executor still holds); a
// job larger than the whole budget fails with kErrNoMem.  A job that does not
// fit yet stops the admission (no overtaking: large jobs are not starved).
// A round holds jobs of one kind, that of the queue's first job: those whose
// graph is built first (`builds`) or resident ones, so that a resident job
// never waits for another job's build.  Jobs of the other kind keep their
// place (at most max_jobs_per_round of them are passed over per round).  The
// first queued job opens the next round, unless it builds and
// max_build_rounds rounds are building already: then the resident jobs
// behind it run meanwhile, and it opens the round after the next build ends.
void scheduler::admit_locked(slot_state& s, int si, double t, std::vector<job*>& retired) {
    (void)si;
    if (queue_.empty()) return;
    uint64_t round_entries = 0;
    const uint64_t held = ex_->held_bytes();
    size_t building = 0;
    for (const slot_state& o : slots_) building += o.busy && o.builds ? 1u : 0u;
    const bool builds = queue_.front()->builds &&
                        (lim_.max_build_rounds == 0 || building < lim_.max_build_rounds);
    s.builds = builds;
    size_t k = 0, passed = 0;
    while (k < queue_.size() && s.jobs.size() < lim_.max_jobs_per_round) {
        job* j = queue_[k];
        if (j->builds != builds) {
            if (++passed > lim_.max_jobs_per_round) break;
            ++k;
            continue;
        }
        if (!s.jobs.empty() && round_entries + j->entries > lim_.max_round_entries) break;
        if (j->footprint > lim_.budget) {
            queue_.erase(queue_.begin() + (std::ptrdiff_t)k);
            complete_locked(j, kErrNoMem, t, retired);
            continue;
        }
        if (bytes_in_flight_ + held + j->footprint > lim_.budget) break;
        queue_.erase(queue_.begin() + (std::ptrdiff_t)k);
        bytes_in_flight_ += j->footprint;
        round_entries += j->entries;
        j->state = kRunning;
        j->t_admit = t;
        admission_ms_sum_ += t - j->t_submit;
        admitted_ += 1;
        s.jobs.push_back(j);
    }
}

void scheduler::worker_main() {
    std::vector<job*> retired;
    std::vector<int> abandoned;
    bool idle_released = false;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        const double t = now_ms();
        // 1. rounds that finished
        for (size_t si = 0; si < slots_.size(); ++si) {
            slot_state& s = slots_[si];
            if (!s.busy || !s.finished.load()) continue;
            ex_->collect((int)si, s.jobs);
            for (job* j : s.jobs) complete_locked(j, j->status, t, retired);
            s.jobs.clear();
            s.busy = false;
            s.finished.store(false);
        }
        // 2. rounds past the watchdog: their jobs fail, the slot is retired
        for (size_t si = 0; si < slots_.size(); ++si) {
            slot_state& s = slots_[si];
            if (!s.busy || s.finished.load()) continue;
            if (!ex_->issued((int)si)) {
                s.t_launch = t;   // still being prepared: the clock starts once it runs
                continue;
            }
            if (t - s.t_launch <= lim_.watchdog_ms) continue;
            for (job* j : s.jobs) complete_locked(j, kErrDevice, t, retired);
            s.jobs.clear();
            s.busy = false;
            s.dead = true;
            st_.abandoned_rounds += 1;
            abandoned.push_back((int)si);
        }
        bool idle = true, any_live = false;
        for (const slot_state& s : slots_) {
            idle = idle && !s.busy;
            any_live = any_live || !s.dead;
        }
        // (an idle executor releases everything it holds: once per idle spell)
        const bool idle_release = idle && !idle_released && ex_->held_bytes() > 0;
        if (!retired.empty() || !abandoned.empty() || idle_release) {
            lk.unlock();
            for (int si : abandoned) ex_->abandon(si);
            ex_->release(idle);
            lk.lock();
            retired.clear();
            abandoned.clear();
            idle_released = idle;
            continue;   // new completions may have arrived meanwhile
        }
        if (stop_) break;
        // 3. no slot left (every round was abandoned): the device is lost
        if (!any_live) {
            while (!queue_.empty()) {
                job* j = queue_.front();
                queue_.pop_front();
                complete_locked(j, kErrDevice, t, retired);
            }
            if (!retired.empty()) continue;
        }
        // 4. admit queued jobs into a free slot and start the round
        int free_slot = -1;
        for (size_t k = 0; k < slots_.size(); ++k) {
            const int si = (int)((rotate_ + k) % slots_.size());
            if (!slots_[(size_t)si].busy && !slots_[(size_t)si].dead) {
                free_slot = si;
                break;
            }
        }
        if (free_slot >= 0 && !queue_.empty()) {
            slot_state& s = slots_[(size_t)free_slot];
            admit_locked(s, free_slot, t, retired);
            if (!s.jobs.empty()) {
                s.busy = true;
                s.finished.store(false);
                s.t_launch = t;
                idle_released = false;
                st_.rounds += 1;
                rotate_ = (free_slot + 1) % (int)slots_.size();
                lk.unlock();
                const int rc = ex_->launch(free_slot, s.jobs);   // only this thread touches s.jobs
                lk.lock();
                if (rc != kOk) {
                    const double t2 = now_ms();
                    for (job* j : s.jobs) complete_locked(j, j->status == kOk ? rc : j->status, t2, retired);
                    s.jobs.clear();
                    s.busy = false;
                    st_.failed_rounds += 1;
                }
                continue;
            }
            if (!retired.empty()) continue;
        }
        bool any_busy = false;
        for (const slot_state& s : slots_) any_busy = any_busy || s.busy;
        if (any_busy) cv_.wait_for(lk, std::chrono::milliseconds(1));
        else cv_.wait(lk);
    }
    // shutdown: the rounds in flight finish, queued jobs are cancelled
    lk.unlock();
    ex_->drain();
    lk.lock();
    const double t = now_ms();
    for (size_t si = 0; si < slots_.size(); ++si) {
        slot_state& s = slots_[si];
        if (!s.busy) continue;
        if (s.finished.load()) {
            ex_->collect((int)si, s.jobs);
            for (job* j : s.jobs) complete_locked(j, j->status, t, retired);
        } else {
            for (job* j : s.jobs) complete_locked(j, kErrShutdown, t, retired);
        }
        s.jobs.clear();
        s.busy = false;
    }
    while (!queue_.empty()) {
        job* j = queue_.front();
        queue_.pop_front();
        complete_locked(j, kErrShutdown, t, retired);
    }
    lk.unlock();
    ex_->release(true);
}

}  // namespace sched
}  // namespace tc
