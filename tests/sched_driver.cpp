// CPU driver of the quote scheduler (paper_1308_2572_amd/csrc/quote_sched.cpp)
// with a stand-in executor backed by the oracle: a "device" thread runs the
// launches and finishing work in order, as a stream would, computing each
// (quote, block) item's year losses with oracle_forward over the block's
// trials and each finished quote's metrics with oracle_metrics.  Built with
// -fsanitize=thread by tests/test_server_cpu.py; prints one line per check
// and exits non-zero on the first failure.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "quote_sched.h"

extern "C" {
int oracle_build_tables(int32_t n_elts, int32_t catalog, const int64_t *rec_off, const int32_t *rec_ids,
                        const float *rec_loss, float *tables);
int oracle_forward(int32_t n_elts, int32_t catalog, const float *tables, int64_t n_trials, const int64_t *offsets,
                   const int32_t *ids, int32_t n_layers, const int32_t *layer_off, const int32_t *layer_elts,
                   const double *elt_terms, const double *layer_terms, int64_t t0, int64_t t1, int32_t n_threads,
                   double *ylt, double *s_pre, int32_t *hits, double *ylt_closed, double *yelt, double *occ_max);
int oracle_metrics(const double *ylt, int32_t n_layers, int64_t n, double p, double *out);
}

using namespace ara;

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

// ------------------------------------------------------------------ inputs
struct World {
    int32_t catalog = 3000, n_elts = 12;
    int64_t n_trials = 1000;
    int tb = 64;
    std::vector<float> tables;
    std::vector<int64_t> off;
    std::vector<int32_t> ids;
    std::vector<double> elt_terms;
    int n_blocks() const { return static_cast<int>((n_trials + tb - 1) / tb); }
};

static World make_world(uint64_t seed) {
    World w;
    std::mt19937_64 g(seed);
    std::vector<int64_t> rec_off(1, 0);
    std::vector<int32_t> rec_ids;
    std::vector<float> rec_loss;
    std::lognormal_distribution<double> ln(9.0, 1.2);
    for (int k = 0; k < w.n_elts; ++k) {
        std::vector<int32_t> all(static_cast<size_t>(w.catalog));
        for (int i = 0; i < w.catalog; ++i) all[static_cast<size_t>(i)] = i;
        std::shuffle(all.begin(), all.end(), g);
        const int sz = 100 + static_cast<int>(g() % 400);
        for (int i = 0; i < sz; ++i) {
            rec_ids.push_back(all[static_cast<size_t>(i)]);
            rec_loss.push_back(static_cast<float>(ln(g)));
        }
        rec_off.push_back(static_cast<int64_t>(rec_ids.size()));
        w.elt_terms.push_back(0.5 + (g() % 1000) / 1000.0);
        w.elt_terms.push_back(static_cast<double>(g() % 2000));
        w.elt_terms.push_back(2e4 + static_cast<double>(g() % 50000));
    }
    w.tables.assign(static_cast<size_t>(w.n_elts) * w.catalog, 0.0f);
    CHECK(oracle_build_tables(w.n_elts, w.catalog, rec_off.data(), rec_ids.data(), rec_loss.data(), w.tables.data()) == 0);
    w.off.push_back(0);
    for (int64_t t = 0; t < w.n_trials; ++t) {
        const int len = static_cast<int>(g() % 60);
        for (int i = 0; i < len; ++i) w.ids.push_back(static_cast<int32_t>(g() % static_cast<uint64_t>(w.catalog)));
        w.off.push_back(static_cast<int64_t>(w.ids.size()));
    }
    return w;
}

struct Quote {
    std::vector<int32_t> elts;
    double terms[4];
    int64_t t0, t1;
    double p;
};

static std::vector<Quote> make_quotes(const World &w, uint64_t seed, int n) {
    std::mt19937_64 g(seed);
    std::vector<Quote> out;
    for (int i = 0; i < n; ++i) {
        Quote q;
        std::vector<int32_t> all(static_cast<size_t>(w.n_elts));
        for (int k = 0; k < w.n_elts; ++k) all[static_cast<size_t>(k)] = k;
        std::shuffle(all.begin(), all.end(), g);
        q.elts.assign(all.begin(), all.begin() + 1 + static_cast<long>(g() % 8));
        q.terms[0] = static_cast<double>(g() % 3000);
        q.terms[1] = 1e4 + static_cast<double>(g() % 100000);
        q.terms[2] = static_cast<double>(g() % 20000);
        q.terms[3] = 1e5 + static_cast<double>(g() % 1000000);
        const int64_t n_tr = 1 + static_cast<int64_t>(g() % static_cast<uint64_t>(w.n_trials));
        q.t0 = static_cast<int64_t>(g() % static_cast<uint64_t>(w.n_trials - n_tr + 1));
        q.t1 = q.t0 + n_tr;
        q.p = 0.9;
        out.push_back(q);
    }
    return out;
}

static ara_quote to_abi(const Quote &q) {
    ara_quote a{};
    a.n_elts = static_cast<int32_t>(q.elts.size());
    a.want_grad = 0;
    a.elt_ids = q.elts.data();
    for (int i = 0; i < 4; ++i) a.layer_terms[i] = q.terms[i];
    a.trial_begin = q.t0;
    a.trial_end = q.t1;
    a.p = q.p;
    return a;
}

// year losses of one quote's layer over trials [a, b)
static void oracle_ylt(const World &w, const std::vector<int32_t> &elts, const double *terms, int64_t a, int64_t b,
                       double *ylt) {
    const int64_t n = b - a;
    if (n <= 0) return;
    std::vector<double> s(static_cast<size_t>(n)), closed(static_cast<size_t>(n));
    std::vector<int32_t> hits(static_cast<size_t>(n));
    const int32_t lo[2] = {0, static_cast<int32_t>(elts.size())};
    CHECK(oracle_forward(w.n_elts, w.catalog, w.tables.data(), w.n_trials, w.off.data(), w.ids.data(), 1, lo,
                         elts.data(), w.elt_terms.data(), terms, a, b, 1, ylt, s.data(), hits.data(), closed.data(),
                         nullptr, nullptr) == 0);
}

static void direct_metrics(const World &w, const Quote &q, double out[3]) {
    std::vector<double> y(static_cast<size_t>(q.t1 - q.t0));
    oracle_ylt(w, q.elts, q.terms, q.t0, q.t1, y.data());
    CHECK(oracle_metrics(y.data(), 1, q.t1 - q.t0, q.p, out) == 0);
}

// ------------------------------------------------------------------ executor
class FakeExec final : public SchedExecutor {
   public:
    struct FJob {
        int64_t ticket;
        Quote q;
        std::vector<double> ylt, res;
        std::atomic<bool> finished{false};
    };
    struct Logged {
        int64_t ticket;
        int block;
    };

    explicit FakeExec(const World &w, int launch_us = 100) : w_(w), launch_us_(launch_us) {
        dev_ = std::thread([this] { run(); });
    }
    ~FakeExec() override {
        {
            std::lock_guard<std::mutex> lk(m_);
            quit_ = true;
        }
        cv_.notify_all();
        dev_.join();
    }

    int32_t validate(const ara_quote &q, std::string *err) override {
        if (q.want_grad) {
            *err = "no gradients here";
            return ARA_E_INVAL;
        }
        return ARA_OK;
    }
    size_t job_bytes(const SchedJob &j) override { return 1024 + 8 * static_cast<size_t>(j.q.trial_end - j.q.trial_begin); }
    int32_t setup(SchedJob &j, std::string *) override {
        auto *f = new FJob();
        f->ticket = j.ticket;
        f->q.elts = j.elt_ids;
        for (int i = 0; i < 4; ++i) f->q.terms[i] = j.q.layer_terms[i];
        f->q.t0 = j.q.trial_begin;
        f->q.t1 = j.q.trial_end;
        f->q.p = j.q.p;
        f->ylt.assign(static_cast<size_t>(f->q.t1 - f->q.t0), -1.0);
        j.exec = f;
        ++created;
        const int now = ++live;
        int m = max_live.load();
        while (now > m && !max_live.compare_exchange_weak(m, now)) {
        }
        return ARA_OK;
    }
    int32_t launch(const std::vector<SchedItem> &items, bool shared, std::string *) override {
        std::vector<std::pair<FJob *, int>> work;
        std::vector<Logged> rec;
        for (const SchedItem &it : items) {
            if (!it.job) {
                rec.push_back({-1, -1});
                continue;
            }
            work.push_back({static_cast<FJob *>(it.job->exec), it.block});
            rec.push_back({it.job->ticket, it.block});
        }
        {
            std::lock_guard<std::mutex> lk(log_mu_);
            log_.push_back(rec);
            shared_flags_.push_back(shared);
        }
        {   // at most two launches in flight, as the device executor's item ring allows
            std::unique_lock<std::mutex> lk(m_);
            cv_.wait(lk, [&] { return in_flight_ < 2; });
            ++in_flight_;
        }
        enqueue([this, work] {
            std::this_thread::sleep_for(std::chrono::microseconds(launch_us_));
            for (auto &wk : work) {
                FJob *f = wk.first;
                const int64_t a = std::max<int64_t>(f->q.t0, static_cast<int64_t>(wk.second) * w_.tb);
                const int64_t b = std::min<int64_t>(f->q.t1, static_cast<int64_t>(wk.second + 1) * w_.tb);
                oracle_ylt(w_, f->q.elts, f->q.terms, a, b, f->ylt.data() + (a - f->q.t0));
            }
            {
                std::lock_guard<std::mutex> lk(m_);
                --in_flight_;
            }
            cv_.notify_all();
        });
        return ARA_OK;
    }
    int32_t finish(SchedJob &j, std::string *) override {
        FJob *f = static_cast<FJob *>(j.exec);
        enqueue([f] {
            f->res.assign(3, 0.0);
            CHECK(oracle_metrics(f->ylt.data(), 1, f->q.t1 - f->q.t0, f->q.p, f->res.data()) == 0);
            f->finished.store(true, std::memory_order_release);
        });
        return ARA_OK;
    }
    // the quotes a launch finished, handed over together: each must have had
    // every one of its blocks launched; their metrics run as one device task
    int32_t finish_all(const std::vector<SchedJob *> &jobs, std::string *) override {
        std::vector<FJob *> fs;
        std::vector<int64_t> tickets;
        {
            std::lock_guard<std::mutex> lk(log_mu_);
            for (SchedJob *j : jobs) {
                const int b0 = static_cast<int>(j->q.trial_begin / w_.tb);
                const int b1 = static_cast<int>((j->q.trial_end + w_.tb - 1) / w_.tb);
                std::set<int> seen;
                for (auto &l : log_)
                    for (auto &x : l)
                        if (x.ticket == j->ticket) seen.insert(x.block);
                CHECK(static_cast<int>(seen.size()) == b1 - b0 && *seen.begin() == b0 && *seen.rbegin() == b1 - 1);
                fs.push_back(static_cast<FJob *>(j->exec));
                tickets.push_back(j->ticket);
            }
            batches_.push_back(tickets);
        }
        enqueue([fs] {
            for (FJob *f : fs) {
                f->res.assign(3, 0.0);
                CHECK(oracle_metrics(f->ylt.data(), 1, f->q.t1 - f->q.t0, f->q.p, f->res.data()) == 0);
            }
            for (FJob *f : fs) f->finished.store(true, std::memory_order_release);
        });
        return ARA_OK;
    }
    bool done(SchedJob &j) override { return static_cast<FJob *>(j.exec)->finished.load(std::memory_order_acquire); }
    int32_t collect(SchedJob &j) override {
        FJob *f = static_cast<FJob *>(j.exec);
        j.res.assign(15 + 9 * j.elt_ids.size(), 0.0);
        std::copy(f->res.begin(), f->res.end(), j.res.begin());
        return ARA_OK;
    }
    void release(SchedJob &j) override {
        delete static_cast<FJob *>(j.exec);
        j.exec = nullptr;
        ++destroyed;
        --live;
    }

    void settle() override {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return in_flight_ == 0; });
    }

    std::vector<std::vector<Logged>> log() {
        std::lock_guard<std::mutex> lk(log_mu_);
        return log_;
    }
    std::vector<bool> shared_flags() {
        std::lock_guard<std::mutex> lk(log_mu_);
        return shared_flags_;
    }
    std::vector<std::vector<int64_t>> batches() {
        std::lock_guard<std::mutex> lk(log_mu_);
        return batches_;
    }

    std::atomic<int64_t> created{0}, destroyed{0};
    std::atomic<int> live{0}, max_live{0};

   private:
    void enqueue(std::function<void()> f) {
        {
            std::lock_guard<std::mutex> lk(m_);
            q_.push_back(std::move(f));
        }
        cv_.notify_all();
    }
    void run() {
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return quit_ || !q_.empty(); });
                if (q_.empty()) return;
                f = std::move(q_.front());
                q_.pop_front();
            }
            f();
        }
    }

    const World &w_;
    int launch_us_;
    std::thread dev_;
    std::mutex m_, log_mu_;
    std::condition_variable cv_;
    std::deque<std::function<void()>> q_;
    bool quit_ = false;
    int in_flight_ = 0;
    std::vector<std::vector<Logged>> log_;
    std::vector<bool> shared_flags_;
    std::vector<std::vector<int64_t>> batches_;
};

static SchedConfig config_for(const World &w, size_t arena, int slots) {
    SchedConfig c;
    c.n_trials = w.n_trials;
    c.trials_per_block = w.tb;
    c.n_blocks = w.n_blocks();
    c.n_elts = w.n_elts;
    c.arena_bytes = arena;
    c.max_slots = slots;
    c.max_items = 256;
    c.items_per_launch = 48;
    c.min_window = 4;
    c.n_xcd = 8;
    return c;
}

static bool same_bits(const double *a, const double *b, int n) { return std::memcmp(a, b, sizeof(double) * n) == 0; }

// every block with several items in one launch: its items on one XCD, back to back
static void check_grouping(const std::vector<FakeExec::Logged> &launch, int n_xcd) {
    std::map<int, std::vector<size_t>> where;
    for (size_t i = 0; i < launch.size(); ++i)
        if (launch[i].ticket >= 0) where[launch[i].block].push_back(i);
    CHECK(launch.size() % static_cast<size_t>(n_xcd) == 0);
    for (auto &kv : where) {
        const auto &v = kv.second;
        for (size_t i = 1; i < v.size(); ++i) {
            CHECK(v[i] % n_xcd == v[0] % n_xcd);
            CHECK(v[i] == v[i - 1] + static_cast<size_t>(n_xcd));
        }
    }
}

// ------------------------------------------------------------------ checks
static void alone_vs_mix(const World &w) {
    const auto quotes = make_quotes(w, 11, 14);
    std::vector<std::array<double, 3>> direct(quotes.size()), alone(quotes.size()), mix(quotes.size());
    for (size_t i = 0; i < quotes.size(); ++i) direct_metrics(w, quotes[i], direct[i].data());
    FakeExec ex(w);
    {
        Scheduler s(&ex, config_for(w, 1 << 30, 8));
        s.start();
        std::string err;
        for (size_t i = 0; i < quotes.size(); ++i) {
            ara_quote a = to_abi(quotes[i]);
            int64_t t = 0;
            CHECK(s.submit(a, &t, &err) == ARA_OK);
            std::shared_ptr<SchedJob> j;
            CHECK(s.wait(t, &j, &err) == ARA_OK);
            CHECK(j->status == ARA_OK);
            std::copy(j->res.begin(), j->res.begin() + 3, alone[i].begin());
        }
        std::vector<int64_t> tk(quotes.size());
        for (size_t i = 0; i < quotes.size(); ++i) {
            ara_quote a = to_abi(quotes[i]);
            CHECK(s.submit(a, &tk[i], &err) == ARA_OK);
        }
        for (size_t i = 0; i < quotes.size(); ++i) {
            std::shared_ptr<SchedJob> j;
            CHECK(s.wait(tk[i], &j, &err) == ARA_OK);
            std::copy(j->res.begin(), j->res.begin() + 3, mix[i].begin());
        }
        int64_t st[9];
        s.stats(st);
        CHECK(st[2] >= 2);           // several quotes shared a launch
        CHECK(st[7] > 0);            // and some blocks
        CHECK(st[3] == 0 && st[4] == 0 && st[5] == static_cast<int64_t>(1 << 30));
        s.stop();
    }
    for (size_t i = 0; i < quotes.size(); ++i) {
        CHECK(same_bits(direct[i].data(), alone[i].data(), 3));
        CHECK(same_bits(direct[i].data(), mix[i].data(), 3));
    }
    bool some_shared = false;
    for (auto &l : ex.log()) check_grouping(l, 8);
    for (bool b : ex.shared_flags()) some_shared = some_shared || b;
    CHECK(some_shared);
    CHECK(ex.created == ex.destroyed && ex.created == static_cast<int64_t>(2 * quotes.size()));
    std::printf("ok alone == mix == direct for %zu quotes; %zu launches\n", quotes.size(), ex.log().size());
}

// Quotes queued before the scheduler starts are admitted in its first
// iteration; when their ranges all end in the last block they finish after
// the same launch and reach the executor in one batch.
static void finished_together(const World &w) {
    auto quotes = make_quotes(w, 16, 9);
    const int64_t starts[9] = {0, 1, 63, 64, 300, 511, 700, 960, 999};
    for (size_t i = 0; i < quotes.size(); ++i) {
        quotes[i].t0 = starts[i];
        quotes[i].t1 = w.n_trials;
    }
    FakeExec ex(w);
    Scheduler s(&ex, config_for(w, 1 << 30, 16));
    std::string err;
    std::vector<int64_t> tk(quotes.size());
    for (size_t i = 0; i < quotes.size(); ++i) {
        ara_quote a = to_abi(quotes[i]);
        CHECK(s.submit(a, &tk[i], &err) == ARA_OK);
    }
    s.start();
    for (size_t i = 0; i < quotes.size(); ++i) {
        std::shared_ptr<SchedJob> j;
        CHECK(s.wait(tk[i], &j, &err) == ARA_OK);
        double d[3];
        direct_metrics(w, quotes[i], d);
        CHECK(same_bits(d, j->res.data(), 3));
    }
    int64_t st[9];
    s.stats(st);
    s.stop();
    const auto b = ex.batches();
    size_t total = 0, most = 0;
    for (auto &x : b) {
        total += x.size();
        most = std::max(most, x.size());
    }
    CHECK(total == quotes.size());
    CHECK(most == quotes.size() && st[8] == static_cast<int64_t>(quotes.size()));
    std::printf("ok %zu quotes ending in the last block finished after one launch, in one batch\n", most);
}

// With the XCD's concurrent workgroups known, no launch ends in a round of
// workgroups that is at most half full, unless the window could not be cut
// back to whole rounds; the results do not change.
static void whole_rounds(const World &w) {
    auto quotes = make_quotes(w, 17, 12);
    FakeExec ex(w);
    SchedConfig cfg = config_for(w, 1 << 30, 16);
    cfg.xcd_slots = 3;
    cfg.items_per_launch = 60;
    cfg.min_window = 1;
    Scheduler s(&ex, cfg);
    std::string err;
    std::vector<int64_t> tk(quotes.size());
    for (size_t i = 0; i < quotes.size(); ++i) {
        ara_quote a = to_abi(quotes[i]);
        CHECK(s.submit(a, &tk[i], &err) == ARA_OK);
    }
    s.start();
    for (size_t i = 0; i < quotes.size(); ++i) {
        std::shared_ptr<SchedJob> j;
        CHECK(s.wait(tk[i], &j, &err) == ARA_OK);
        double d[3];
        direct_metrics(w, quotes[i], d);
        CHECK(same_bits(d, j->res.data(), 3));
    }
    s.stop();
    int cut = 0, ragged = 0;
    for (auto &l : ex.log()) {
        check_grouping(l, 8);
        const int depth = static_cast<int>(l.size()) / 8;
        if (depth > 3 && depth % 3 != 0 && depth % 3 <= 1) ++ragged;
        if (depth > 3 && depth % 3 == 0) ++cut;
    }
    CHECK(ragged == 0 && cut > 0);
    std::printf("ok launches in whole rounds of workgroups: %d of %zu launches at a multiple of the XCD's slots\n", cut,
                ex.log().size());
}

static void admission_by_memory(const World &w) {
    auto quotes = make_quotes(w, 12, 10);
    for (auto &q : quotes) {   // the same size, so the arena holds exactly two
        q.t0 = 100;
        q.t1 = 900;
    }
    FakeExec ex(w, 2000);
    const size_t one = 1024 + 8 * 800;
    Scheduler s(&ex, config_for(w, 2 * one + one / 2, 16));
    s.start();
    std::string err;
    std::vector<int64_t> tk(quotes.size());
    for (size_t i = 0; i < quotes.size(); ++i) {
        ara_quote a = to_abi(quotes[i]);
        CHECK(s.submit(a, &tk[i], &err) == ARA_OK);
    }
    for (size_t i = 0; i < quotes.size(); ++i) {
        std::shared_ptr<SchedJob> j;
        CHECK(s.wait(tk[i], &j, &err) == ARA_OK);
        double d[3];
        direct_metrics(w, quotes[i], d);
        CHECK(same_bits(d, j->res.data(), 3));
        if (i > 0) CHECK(j->t_admit >= 0.0);
    }
    s.stop();
    CHECK(ex.max_live == 2);
    // a quote that can never fit
    {
        Quote big = quotes[0];
        big.t0 = 0;
        big.t1 = w.n_trials;
        FakeExec ex2(w);
        Scheduler s2(&ex2, config_for(w, one, 4));
        s2.start();
        ara_quote a = to_abi(big);
        int64_t t;
        CHECK(s2.submit(a, &t, &err) == ARA_E_NOSPACE);
    }
    std::printf("ok admission by memory: at most %d quotes live in an arena for two\n", ex.max_live.load());
}

static void mid_flight_admission(const World &w) {
    auto quotes = make_quotes(w, 13, 2);
    quotes[0].t0 = 0;
    quotes[0].t1 = w.n_trials;
    quotes[1].t0 = 200;
    quotes[1].t1 = 700;
    FakeExec ex(w, 3000);
    SchedConfig cfg = config_for(w, 1 << 30, 8);
    cfg.items_per_launch = 3;   // small windows: the long quote takes many launches
    cfg.min_window = 2;
    Scheduler s(&ex, cfg);
    s.start();
    std::string err;
    int64_t ta, tb;
    ara_quote a = to_abi(quotes[0]);
    CHECK(s.submit(a, &ta, &err) == ARA_OK);
    for (int i = 0; i < 2000; ++i) {   // until the first launch of the long quote is out
        int64_t st[9];
        s.stats(st);
        if (st[1] >= 1) break;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    ara_quote b = to_abi(quotes[1]);
    CHECK(s.submit(b, &tb, &err) == ARA_OK);
    std::shared_ptr<SchedJob> ja, jb;
    CHECK(s.wait(ta, &ja, &err) == ARA_OK);
    CHECK(s.wait(tb, &jb, &err) == ARA_OK);
    s.stop();
    CHECK(jb->t_admit < ja->t_done);
    bool together = false;
    for (auto &l : ex.log()) {
        std::set<int64_t> t;
        for (auto &x : l)
            if (x.ticket >= 0) t.insert(x.ticket);
        together = together || t.size() == 2;
        check_grouping(l, 8);
    }
    CHECK(together);
    for (int i = 0; i < 2; ++i) {
        double d[3];
        direct_metrics(w, quotes[static_cast<size_t>(i)], d);
        CHECK(same_bits(d, (i ? jb : ja)->res.data(), 3));
    }
    std::printf("ok mid-flight admission: the second quote joined the first one's launches\n");
}

static void cancellation(const World &w) {
    auto quotes = make_quotes(w, 14, 3);
    FakeExec ex(w, 3000);
    Scheduler s(&ex, config_for(w, 1 << 30, 1));   // one slot: B and C wait behind A
    s.start();
    std::string err;
    int64_t t[3];
    for (int i = 0; i < 3; ++i) {
        ara_quote a = to_abi(quotes[static_cast<size_t>(i)]);
        CHECK(s.submit(a, &t[i], &err) == ARA_OK);
    }
    for (int i = 0; i < 2000; ++i) {
        int64_t st[9];
        s.stats(st);
        if (st[4] == 1) break;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(s.cancel(t[0], &err) == ARA_E_BUSY);   // admitted: runs to completion
    CHECK(s.cancel(t[1], &err) == ARA_OK);
    CHECK(s.cancel(t[1], &err) == ARA_E_BUSY);   // already cancelled
    std::shared_ptr<SchedJob> j;
    CHECK(s.poll(t[1], &j, &err) == ARA_E_INVAL);
    CHECK(s.poll(t[1], &j, &err) == ARA_E_RANGE);   // retired
    for (int i : {0, 2}) {
        CHECK(s.wait(t[i], &j, &err) == ARA_OK);
        double d[3];
        direct_metrics(w, quotes[static_cast<size_t>(i)], d);
        CHECK(same_bits(d, j->res.data(), 3));
    }
    s.stop();
    CHECK(ex.created == 2 && ex.destroyed == 2);
    std::printf("ok cancellation: queued quote cancelled, admitted one busy\n");
}

static void stop_with_work_pending(const World &w) {
    auto quotes = make_quotes(w, 15, 12);
    FakeExec ex(w, 2000);
    std::vector<int64_t> t(quotes.size());
    {
        Scheduler s(&ex, config_for(w, 1 << 30, 2));
        s.start();
        std::string err;
        for (size_t i = 0; i < quotes.size(); ++i) {
            ara_quote a = to_abi(quotes[i]);
            CHECK(s.submit(a, &t[i], &err) == ARA_OK);
        }
        std::thread waiter([&] {
            std::shared_ptr<SchedJob> j;
            std::string e2;
            const int32_t rc = s.wait(t.back(), &j, &e2);
            CHECK(rc == ARA_OK || rc == ARA_E_INVAL);
        });
        s.stop();
        waiter.join();
        ara_quote a = to_abi(quotes[0]);
        int64_t tt;
        CHECK(s.submit(a, &tt, &err) == ARA_E_INVAL);   // stopping
    }
    CHECK(ex.created == ex.destroyed);
    std::printf("ok stop with quotes queued and active: drained, %lld set up and released\n",
                static_cast<long long>(ex.created.load()));
}

static void deal_property() {
    std::mt19937_64 g(5);
    for (int rep = 0; rep < 200; ++rep) {
        std::vector<int> blk;
        const int groups = 1 + static_cast<int>(g() % 40);
        for (int b = 0; b < groups; ++b)
            for (int k = 0, n = 1 + static_cast<int>(g() % 6); k < n; ++k) blk.push_back(b * 3);
        const auto order = deal_to_xcds(blk, 8);
        CHECK(order.size() % 8 == 0);
        std::vector<int> seen(blk.size(), 0);
        std::vector<FakeExec::Logged> l;
        for (int i : order) {
            if (i >= 0) ++seen[static_cast<size_t>(i)];
            l.push_back({i < 0 ? -1 : 0, i < 0 ? -1 : blk[static_cast<size_t>(i)]});
        }
        for (int c : seen) CHECK(c == 1);
        check_grouping(l, 8);
    }
    std::printf("ok dealing to XCDs: every item once, each block's items on one XCD back to back\n");
}

int main() {
    const World w = make_world(7);
    deal_property();
    alone_vs_mix(w);
    finished_together(w);
    whole_rounds(w);
    admission_by_memory(w);
    mid_flight_admission(w);
    cancellation(w);
    stop_with_work_pending(w);
    std::printf("all scheduler checks passed\n");
    return 0;
}
