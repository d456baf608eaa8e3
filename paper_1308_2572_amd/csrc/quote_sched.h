// Quote scheduler: the host-side core of the continuous-batching server,
// free of HIP so that it runs (and is tested under ThreadSanitizer) on the
// CPU with a stand-in executor.
//
// A quote is a candidate layer over a contiguous trial range.  Queued quotes
// are admitted in arrival order while a slot and arena memory are free.  The
// active quotes are served by a circular scan of the YET's trial blocks:
// every iteration takes a window of consecutive blocks from the scan
// position and, in ONE launch, every active quote's work item for each of
// those blocks that lies in its range and has not been served yet; then the
// position moves past the window.  A quote admitted mid-scan joins at the
// next iteration and is complete after one revolution over its range, so
// quotes that are active together read the same blocks in the same launch.
// The items of one block are dealt to one XCD one after another (the device
// deals workgroups to its XCDs round-robin by index), so the quotes sharing
// a block read its codes through one L2.  A quote whose blocks have all been
// launched is finished (metrics, backward, result copy); when the executor
// reports that work complete its results are collected and its memory and
// slot freed.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ara.h"
#include "arena.h"

namespace ara {

enum SchedStage { kQueued, kForward, kFinishing, kDone, kCancelled };

struct SchedJob {
    int64_t ticket = 0;
    ara_quote q{};                  // q.elt_ids is cleared: the list is elt_ids
    std::vector<int32_t> elt_ids;
    // Written under the scheduler's mutex only; the scheduler thread also
    // reads it without the mutex (no other thread writes an admitted job's
    // stage).
    int stage = kQueued;
    int slot = -1;
    size_t mem_off = 0, mem_bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t status = ARA_OK;
    // the quote's blocks [b_lo, b_hi) and which of them have been launched
    // (scheduler thread only)
    int b_lo = 0, b_hi = 0, launched = 0;
    std::vector<uint8_t> served;
    // results: 3 metrics, 3x4 layer gradients, 3 x J x 3 ELT gradients in the
    // quote's ELT order (filled by the executor's collect)
    std::vector<double> res;
    void *exec = nullptr;           // the executor's per-quote state
};

// One unit of forward work: a quote's layer over one block of trials; a null
// job is an empty slot of the launch (the workgroup exits at once).
struct SchedItem {
    SchedJob *job;
    int block;
};

// What the scheduler asks of the device side.  All calls come from the
// scheduler thread, except validate and job_bytes (submitting threads too).
class SchedExecutor {
   public:
    virtual ~SchedExecutor() = default;
    // quote checks that depend on the resident data; ARA_OK or a status with *err
    virtual int32_t validate(const ara_quote &q, std::string *err) = 0;
    // arena bytes the quote needs while active
    virtual size_t job_bytes(const SchedJob &j) = 0;
    // an admitted quote: set up its state in arena bytes [mem_off, mem_off + mem_bytes)
    virtual int32_t setup(SchedJob &j, std::string *err) = 0;
    // one launch over the items in slot order; shared: some block has several items
    virtual int32_t launch(const std::vector<SchedItem> &items, bool shared, std::string *err) = 0;
    // after the launch holding its last block: metrics, backward, result copy
    virtual int32_t finish(SchedJob &j, std::string *err) = 0;
    // every quote whose last block the launch held; one at a time unless the
    // executor does better (the device executor shares the metrics launches)
    virtual int32_t finish_all(const std::vector<SchedJob *> &jobs, std::string *err) {
        for (SchedJob *j : jobs) {
            const int32_t rc = finish(*j, err);
            if (rc) return rc;
        }
        return 0;
    }
    // has the quote's finishing work completed?
    virtual bool done(SchedJob &j) = 0;
    // fills j.res; returns the quote's device-side status (ARA_OK if none)
    virtual int32_t collect(SchedJob &j) = 0;
    // releases the quote's per-quote state (completion marker and the like)
    virtual void release(SchedJob &j) = 0;
    // after an iteration that launched: wait until that launch has run, so
    // that the quotes arriving meanwhile are packed into the next launch
    // instead of queueing behind it one launch each
    virtual void settle() = 0;
};

// Deals items sorted by block to n_xcd XCDs: the items of one block go to
// one XCD, consecutively; blocks go to the XCD with the fewest items so far
// (the lowest index on ties).  Returns the launch order: slot 8k + x is the
// k-th item of XCD x (n_xcd = 8), -1 for an empty slot; its length is a
// multiple of n_xcd.
std::vector<int> deal_to_xcds(const std::vector<int> &block_of_item, int n_xcd);

struct SchedConfig {
    int64_t n_trials = 0;
    int trials_per_block = 1;
    int n_blocks = 0;
    int32_t n_elts = 0;
    size_t arena_bytes = 0;
    int max_slots = 1;
    int max_items = 8192;          // slots of one launch
    int items_per_launch = 6144;   // the scan window is about this many items over the active quotes
    int min_window = 64;           // blocks
    int n_xcd = 8;
    // forward workgroups that run at once on one XCD (0: unknown).  A launch
    // whose last round of workgroups would be at most half full is cut back
    // by whole blocks to full rounds; the blocks cut go to the next launch.
    int xcd_slots = 0;
};

class Scheduler {
   public:
    Scheduler(SchedExecutor *ex, const SchedConfig &cfg);
    ~Scheduler();   // stops and joins (see stop)
    // starts the scheduler thread
    void start();
    int32_t submit(const ara_quote &q, int64_t *ticket, std::string *err);
    // ARA_OK and the job's results when done (the ticket is retired),
    // ARA_E_BUSY while not done; a cancelled quote retires with ARA_E_INVAL
    int32_t poll(int64_t ticket, std::shared_ptr<SchedJob> *out, std::string *err);
    int32_t wait(int64_t ticket, std::shared_ptr<SchedJob> *out, std::string *err);
    int32_t cancel(int64_t ticket, std::string *err);
    // iterations, launches, most quotes in one launch, queued, active, free
    // arena bytes, items launched, items of shared blocks, most quotes
    // finished after one launch
    void stats(int64_t *s9);
    // stops admitting, cancels what is queued, drains the active quotes and
    // joins the scheduler thread; idempotent
    void stop();

   private:
    static constexpr int kSpinPolls = 256;   // polls before the scheduler sleeps between them
    void loop();
    void admit(std::vector<std::shared_ptr<SchedJob>> *admitted);
    bool next_launch(std::vector<SchedItem> *slots, bool *shared, std::vector<SchedJob *> *completed);

    SchedExecutor *ex_;
    SchedConfig cfg_;
    Arena arena_;
    std::vector<int> free_slots_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<std::shared_ptr<SchedJob>> queue_;
    std::vector<std::shared_ptr<SchedJob>> active_;
    std::map<int64_t, std::shared_ptr<SchedJob>> jobs_;
    int64_t next_ticket_ = 1;
    bool stop_ = false, stopped_ = false;
    int32_t fatal_ = ARA_OK;
    std::string fatal_msg_;
    std::thread th_;
    int scan_pos_ = 0;   // scheduler thread only
    // statistics (under mu_)
    int64_t iterations_ = 0, launches_ = 0, max_quotes_ = 0, items_ = 0, shared_items_ = 0, max_finished_ = 0;
};

}  // namespace ara
