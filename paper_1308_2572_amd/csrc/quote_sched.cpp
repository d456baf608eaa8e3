// Quote scheduler (host side of the continuous-batching server); see quote_sched.h.
#include "quote_sched.h"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace ara {

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

std::vector<int> deal_to_xcds(const std::vector<int> &block_of_item, int n_xcd) {
    std::vector<std::vector<int>> lists(static_cast<size_t>(std::max(n_xcd, 1)));
    size_t i = 0;
    while (i < block_of_item.size()) {
        size_t e = i;
        while (e < block_of_item.size() && block_of_item[e] == block_of_item[i]) ++e;
        size_t best = 0;
        for (size_t x = 1; x < lists.size(); ++x)
            if (lists[x].size() < lists[best].size()) best = x;
        for (size_t k = i; k < e; ++k) lists[best].push_back(static_cast<int>(k));
        i = e;
    }
    size_t depth = 0;
    for (auto &l : lists) depth = std::max(depth, l.size());
    std::vector<int> out(depth * lists.size(), -1);
    for (size_t x = 0; x < lists.size(); ++x)
        for (size_t k = 0; k < lists[x].size(); ++k) out[k * lists.size() + x] = lists[x][k];
    return out;
}

Scheduler::Scheduler(SchedExecutor *ex, const SchedConfig &cfg) : ex_(ex), cfg_(cfg) {
    arena_.init(cfg_.arena_bytes);
    for (int i = cfg_.max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
}

Scheduler::~Scheduler() { stop(); }

void Scheduler::start() { th_ = std::thread([this] { loop(); }); }

int32_t Scheduler::submit(const ara_quote &q, int64_t *ticket, std::string *err) {
    if (q.n_elts < 0 || q.n_elts > ARA_MAX_ELTS_PER_LAYER) {
        *err = "quote ELT count out of range";
        return ARA_E_LIMIT;
    }
    if (q.n_elts > 0 && !q.elt_ids) {
        *err = "quote without ELT list";
        return ARA_E_INVAL;
    }
    for (int i = 0; i < q.n_elts; ++i)
        if (q.elt_ids[i] < 0 || q.elt_ids[i] >= cfg_.n_elts) {
            *err = "quote ELT index out of range";
            return ARA_E_RANGE;
        }
    if (q.trial_begin < 0 || q.trial_end < q.trial_begin || q.trial_end > cfg_.n_trials) {
        *err = "quote trial range outside the YET";
        return ARA_E_RANGE;
    }
    if (q.trial_end == q.trial_begin) {
        *err = "quote over an empty trial range";
        return ARA_E_INVAL;
    }
    if (!(q.p > 0.0 && q.p < 1.0)) {
        *err = "quote p must lie in (0, 1)";
        return ARA_E_INVAL;
    }
    const double *t = q.layer_terms;
    if (!(t[0] >= 0.0 && t[0] < INFINITY) || !(t[1] > 0.0) || !(t[2] >= 0.0 && t[2] < INFINITY) || !(t[3] > 0.0)) {
        *err = "quote layer terms invalid";
        return ARA_E_INVAL;
    }
    int32_t rc = ex_->validate(q, err);
    if (rc) return rc;
    auto j = std::make_shared<SchedJob>();
    j->q = q;
    j->elt_ids.assign(q.elt_ids, q.elt_ids + q.n_elts);
    j->q.elt_ids = nullptr;
    j->t_submit = now_ms();
    if (ex_->job_bytes(*j) > arena_.size()) {
        *err = "quote larger than the whole arena";
        return ARA_E_NOSPACE;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (fatal_) {
        *err = "server stopped after a device error: " + fatal_msg_;
        return fatal_;
    }
    if (stop_) {
        *err = "server is stopping";
        return ARA_E_INVAL;
    }
    j->ticket = next_ticket_++;
    jobs_[j->ticket] = j;
    queue_.push_back(j);
    *ticket = j->ticket;
    cv_work_.notify_all();
    return ARA_OK;
}

int32_t Scheduler::poll(int64_t ticket, std::shared_ptr<SchedJob> *out, std::string *err) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) {
        *err = "unknown ticket";
        return ARA_E_RANGE;
    }
    if (it->second->stage == kCancelled) {
        jobs_.erase(it);
        *err = "quote was cancelled";
        return ARA_E_INVAL;
    }
    if (it->second->stage != kDone) return ARA_E_BUSY;
    *out = it->second;
    jobs_.erase(it);
    return ARA_OK;
}

int32_t Scheduler::wait(int64_t ticket, std::shared_ptr<SchedJob> *out, std::string *err) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) {
        *err = "unknown ticket";
        return ARA_E_RANGE;
    }
    std::shared_ptr<SchedJob> j = it->second;
    cv_done_.wait(lk, [&] { return j->stage == kDone || j->stage == kCancelled; });
    jobs_.erase(j->ticket);
    if (j->stage == kCancelled) {
        *err = "quote was cancelled";
        return ARA_E_INVAL;
    }
    *out = j;
    return ARA_OK;
}

int32_t Scheduler::cancel(int64_t ticket, std::string *err) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) {
        *err = "unknown ticket";
        return ARA_E_RANGE;
    }
    std::shared_ptr<SchedJob> j = it->second;
    if (j->stage != kQueued) return ARA_E_BUSY;   // admitted: runs to completion
    j->stage = kCancelled;
    queue_.erase(std::find(queue_.begin(), queue_.end(), j));
    cv_done_.notify_all();
    return ARA_OK;
}

void Scheduler::stats(int64_t *s) {
    std::lock_guard<std::mutex> lk(mu_);
    s[0] = iterations_;
    s[1] = launches_;
    s[2] = max_quotes_;
    s[3] = static_cast<int64_t>(queue_.size());
    s[4] = static_cast<int64_t>(active_.size());
    s[5] = static_cast<int64_t>(arena_.free_bytes());
    s[6] = items_;
    s[7] = shared_items_;
    s[8] = max_finished_;
}

void Scheduler::stop() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stopped_) return;
        stop_ = true;
        for (auto &j : queue_) j->stage = kCancelled;
        queue_.clear();
        cv_work_.notify_all();
        cv_done_.notify_all();
    }
    if (th_.joinable()) th_.join();
    std::lock_guard<std::mutex> lk(mu_);
    stopped_ = true;
}

// Under mu_: queued quotes in arrival order while a slot and memory are free.
void Scheduler::admit(std::vector<std::shared_ptr<SchedJob>> *admitted) {
    while (!stop_ && !fatal_ && !queue_.empty() && !free_slots_.empty()) {
        std::shared_ptr<SchedJob> j = queue_.front();
        const size_t need = ex_->job_bytes(*j);
        size_t off = 0;
        if (!arena_.alloc(need, &off)) break;   // arrival order: wait for memory
        queue_.pop_front();
        j->mem_off = off;
        j->mem_bytes = need;
        j->slot = free_slots_.back();
        free_slots_.pop_back();
        j->t_admit = now_ms();
        j->stage = kForward;
        j->b_lo = static_cast<int>(j->q.trial_begin / cfg_.trials_per_block);
        j->b_hi = static_cast<int>((j->q.trial_end + cfg_.trials_per_block - 1) / cfg_.trials_per_block);
        j->served.assign(static_cast<size_t>(j->b_hi - j->b_lo), 0);
        j->launched = 0;
        active_.push_back(j);
        admitted->push_back(j);
    }
}

// Scheduler thread: the next window of the circular scan over the quotes in
// the forward stage.  Returns false when no quote has a block left.
bool Scheduler::next_launch(std::vector<SchedItem> *slots, bool *shared, std::vector<SchedJob *> *completed) {
    std::vector<SchedJob *> fw;
    for (auto &j : active_)
        if (j->stage == kForward && j->launched < j->b_hi - j->b_lo) fw.push_back(j.get());
    if (fw.empty()) return false;
    const int nb = cfg_.n_blocks;
    auto wanted = [](const SchedJob *j, int b) {
        return b >= j->b_lo && b < j->b_hi && !j->served[static_cast<size_t>(b - j->b_lo)];
    };
    // skip to the first block some quote still needs
    int p = scan_pos_, k = 0;
    for (; k < nb; ++k) {
        const int b = (p + k) % nb;
        bool any = false;
        for (SchedJob *j : fw) any = any || wanted(j, b);
        if (any) break;
    }
    p = (p + k) % nb;
    int W = std::max(cfg_.min_window, cfg_.items_per_launch / static_cast<int>(fw.size()));
    W = std::min(W, nb);
    std::vector<SchedItem> items;
    std::vector<int> order;
    // the items of the window's first w blocks, dealt to the XCDs
    auto window = [&](int w) {
        items.clear();
        std::vector<int> blk;
        for (int d = 0; d < w; ++d) {
            const int b = (p + d) % nb;
            for (SchedJob *j : fw)
                if (wanted(j, b)) {
                    items.push_back({j, b});
                    blk.push_back(b);
                }
        }
        order = deal_to_xcds(blk, cfg_.n_xcd);
        return static_cast<int>(order.size()) / std::max(cfg_.n_xcd, 1);   // workgroups per XCD
    };
    int depth = window(W);
    while (static_cast<int>(order.size()) > cfg_.max_items && W > 1) depth = window(W = std::max(1, W / 2));
    const int S = cfg_.xcd_slots;
    if (S > 0 && depth > S && depth % S != 0 && depth % S <= S / 2) {
        // the largest window whose XCDs run whole rounds (the depth grows with w)
        const int full = depth / S * S;
        int lo = 0, hi = W;   // window(lo) fits (or lo = 0), window(hi) does not
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (window(mid) <= full) lo = mid;
            else hi = mid;
        }
        if (lo >= 1) W = lo;
        depth = window(W);
    }
    slots->clear();
    *shared = false;
    for (int i : order) slots->push_back(i < 0 ? SchedItem{nullptr, -1} : items[static_cast<size_t>(i)]);
    for (size_t i = 1; i < items.size(); ++i) *shared = *shared || items[i].block == items[i - 1].block;
    for (auto &it : items) {
        it.job->served[static_cast<size_t>(it.block - it.job->b_lo)] = 1;
        ++it.job->launched;
    }
    completed->clear();
    for (SchedJob *j : fw)
        if (j->launched == j->b_hi - j->b_lo) completed->push_back(j);
    scan_pos_ = (p + W) % nb;
    return true;
}

void Scheduler::loop() {
    int idle_polls = 0;   // iterations in a row that only waited for finishing quotes
    for (;;) {
        std::vector<std::shared_ptr<SchedJob>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait(lk, [&] { return stop_ || !queue_.empty() || !active_.empty(); });
            if (stop_ && active_.empty()) break;
            admit(&admitted);
        }
        int32_t rc = ARA_OK;
        std::string err;
        for (auto &j : admitted)
            if ((rc = ex_->setup(*j, &err))) break;
        std::vector<SchedItem> slots;
        std::vector<SchedJob *> completed;
        bool shared = false, launched = false;
        if (!rc && next_launch(&slots, &shared, &completed)) {
            launched = true;
            rc = ex_->launch(slots, shared, &err);
            int64_t n_items = 0, n_shared = 0, n_quotes = 0;
            std::vector<const SchedJob *> seen;
            for (size_t i = 0; i < slots.size(); ++i) {
                if (!slots[i].job) continue;
                ++n_items;
                if (std::find(seen.begin(), seen.end(), slots[i].job) == seen.end()) seen.push_back(slots[i].job);
            }
            n_quotes = static_cast<int64_t>(seen.size());
            // items whose block another item of the launch shares
            std::map<int, int> per_block;
            for (auto &s : slots)
                if (s.job) ++per_block[s.block];
            for (auto &kv : per_block)
                if (kv.second > 1) n_shared += kv.second;
            if (!rc && !completed.empty()) rc = ex_->finish_all(completed, &err);
            const int64_t n_finished = static_cast<int64_t>(completed.size());
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (SchedJob *j : completed) j->stage = kFinishing;
            }
            std::lock_guard<std::mutex> lk(mu_);
            ++launches_;
            items_ += n_items;
            shared_items_ += n_shared;
            max_quotes_ = std::max(max_quotes_, n_quotes);
            max_finished_ = std::max(max_finished_, n_finished);
        }
        bool waiting = false, launchable = false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            ++iterations_;
            if (rc && !fatal_) {
                fatal_ = rc;
                fatal_msg_ = err;
            }
            for (auto it = active_.begin(); it != active_.end();) {
                SchedJob &j = **it;
                bool done = fatal_ != ARA_OK;
                if (!done && j.stage == kFinishing) done = ex_->done(j);
                if (done) {
                    j.t_done = now_ms();
                    j.status = fatal_ ? fatal_ : ex_->collect(j);
                    ex_->release(j);
                    arena_.release(j.mem_off, j.mem_bytes);
                    free_slots_.push_back(j.slot);
                    j.stage = kDone;
                    it = active_.erase(it);
                    cv_done_.notify_all();
                } else {
                    waiting = waiting || j.stage == kFinishing;
                    launchable = launchable || j.stage == kForward;
                    ++it;
                }
            }
            if (fatal_) {   // nothing more runs: the queued quotes fail too
                for (auto &j : queue_) {
                    j->status = fatal_;
                    j->stage = kDone;
                }
                queue_.clear();
                cv_done_.notify_all();
            }
            launchable = launchable || (!queue_.empty() && !free_slots_.empty());
        }
        if (launched && rc == ARA_OK) {
            idle_polls = 0;
            ex_->settle();
        } else if (waiting && !launchable) {
            // results pending and nothing to launch: poll again at once for a
            // while (a finishing quote's last kernels and copy take tens to
            // hundreds of microseconds, and a sleep overshoots by about as
            // much), then back off to short sleeps
            if (++idle_polls < kSpinPolls) std::this_thread::yield();
            else std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            idle_polls = 0;
        }
    }
}

}  // namespace ara
