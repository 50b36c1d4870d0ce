// Scheduler of the serving loop: a host queue of census jobs, admission by
// device footprint, rounds on a small pool of executor slots, completion,
// a watchdog on rounds and latency statistics.  It knows nothing of HIP: the
// device work of a round is done by a round_executor (tc_serve.cpp holds the
// HIP one), so the scheduler can be driven by other executors as well.
//
// Threads: any number of callers (submit, poll, stats, stop); one worker
// thread (admission, rounds, watchdog); the executor's completion callbacks
// (round_done), which take no lock.
#pragma once
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace tc {
namespace sched {

// Status codes (the values of include/tc.h).
enum : int { kOk = 0, kErrNoMem = -3, kErrDevice = -4, kErrNotFound = -6, kErrShutdown = -7 };

enum job_state { kQueued, kRunning, kDone };

// One census request.  Executors derive from it to carry their payload.
struct job {
    uint64_t ticket = 0;
    uint64_t footprint = 0;    // device bytes while the job is admitted
    uint64_t entries = 0;      // its share of a round (neighbour entries)
    bool builds = false;       // its round builds its graph first (the request brought its arcs)
    double t_submit = 0, t_admit = 0, t_done = 0;   // ms, steady clock
    int status = kOk;
    job_state state = kQueued;
    uint64_t counts[16] = {0};
    virtual ~job() = default;
};

// Submit-to-completion latencies in a fixed histogram: 64 buckets per decade
// from 1 microsecond up (bucket k >= 1 holds [10^((k-1)/64 - 3), 10^(k/64 - 3))
// ms, bucket 0 everything shorter, the last bucket everything from about 10^6
// ms on); a percentile is the upper edge of the bucket that holds it (relative
// error below 3.7 %).  Memory does not grow with the number of requests.
class latency_hist {
public:
    static constexpr int kPerDecade = 64, kDecades = 9, kBuckets = kPerDecade * kDecades + 2;
    void add(double ms);
    double percentile(double q) const;   // 0 when empty
    uint64_t count() const { return total_; }
    void clear();

private:
    uint64_t n_[kBuckets] = {0};
    uint64_t total_ = 0;
};

// The device side of the rounds.
struct round_executor {
    virtual ~round_executor() = default;
    // Number of rounds that may be in flight at once.
    virtual int slot_count() const = 0;
    // Worker thread, scheduler lock not held: starts the round of `jobs` on
    // `slot` and returns kOk, after which the executor calls
    // scheduler::round_done(slot) exactly once, from any thread, when the
    // round's results can be collected.  Any other return value: nothing is
    // running, and every job still kOk is given that status.  A job whose
    // status the executor sets (a build error) is completed with it.
    virtual int launch(int slot, std::vector<job*>& jobs) = 0;
    // Scheduler lock held, after round_done(slot): fill the counts of the
    // jobs whose status is kOk.  Must not block.
    virtual void collect(int slot, std::vector<job*>& jobs) = 0;
    // Scheduler lock held: j leaves the scheduler (done, failed or
    // cancelled); called once per job.  Must not block: device memory the job
    // held is moved to the executor's own list, released by release().
    virtual void job_done(job* j) = 0;
    // Worker thread, lock not held, after jobs were completed: release what
    // they held on the device (job objects may already be polled and gone).
    // `idle`: no round is in flight; then everything held is released.
    virtual void release(bool idle) = 0;
    // Device bytes the executor still holds for completed jobs (counted in
    // admission).  Any thread.
    virtual uint64_t held_bytes() const = 0;
    // Worker thread, lock not held: the round on `slot` outlived the watchdog;
    // its jobs have failed and the slot is never used again.
    virtual void abandon(int slot) = 0;
    // Lock not held, when the worker stops: wait for the rounds of every slot
    // that was not abandoned.
    virtual void drain() = 0;
    // Scheduler lock held, must not block: whether the round on `slot` has
    // issued its device work.  An executor that prepares a round on a thread
    // of its own (building graphs first) reports false until then; the
    // watchdog measures a round from the first check at which this holds.
    virtual bool issued(int slot) const {
        (void)slot;
        return true;
    }
};

struct sched_stats {
    uint64_t submitted = 0, completed = 0, rounds = 0, failed_rounds = 0, abandoned_rounds = 0;
    uint64_t bytes_in_flight = 0;
    double p50_ms = 0, p99_ms = 0, mean_admission_ms = 0;
};

struct sched_limits {
    uint64_t budget = 0;                    // device bytes admitted jobs may hold
    size_t max_jobs_per_round = 512;
    uint64_t max_round_entries = 64ull << 20;   // a round closes past this many entries
    double watchdog_ms = 60000.0;           // a round running longer fails its jobs
    size_t max_build_rounds = 0;            // rounds building graphs at once (0: no limit)
};

class scheduler {
public:
    scheduler(round_executor* ex, const sched_limits& lim);
    ~scheduler();   // stops the worker

    // Takes ownership of j (also on error).  kErrShutdown once stopped.
    int submit(job* j, uint64_t* ticket);
    // As tc_poll: done -> the ticket is retired and its status returned.
    int poll(uint64_t ticket, uint64_t counts[16], int* done);
    // Called by the executor when a round's results are ready.  Takes no lock.
    void round_done(int slot);
    // Stops the worker: running rounds finish, queued jobs end with
    // kErrShutdown, later submissions fail with kErrShutdown.
    void stop();
    bool stopped();
    sched_stats stats();
    void reset_stats();
    void set_watchdog_ms(double ms);

private:
    struct slot_state {
        bool busy = false, dead = false;
        bool builds = false;   // the round's jobs build their graphs
        std::atomic<bool> finished{false};
        double t_launch = 0;
        std::vector<job*> jobs;
    };
    void worker_main();
    void complete_locked(job* j, int status, double t, std::vector<job*>& retired);
    void admit_locked(slot_state& s, int si, double t, std::vector<job*>& retired);

    round_executor* ex_;
    sched_limits lim_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<job*> queue_;
    std::map<uint64_t, job*> jobs_;
    std::vector<slot_state> slots_;
    std::thread worker_;
    bool stop_ = false;
    uint64_t next_ticket_ = 1;
    uint64_t bytes_in_flight_ = 0;
    sched_stats st_;
    latency_hist lat_;
    double admission_ms_sum_ = 0;
    uint64_t admitted_ = 0;
    int rotate_ = 0;
};

double now_ms();

}  // namespace sched
}  // namespace tc
