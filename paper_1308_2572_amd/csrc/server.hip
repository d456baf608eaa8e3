// Quote server: continuous batching of pricing requests over the resident
// YET and ELT tables.
//
// A request ("quote") is a candidate layer -- a subset of the resident ELTs,
// its occurrence and aggregate terms -- over a contiguous trial range, with
// the tail probability for PML/TVaR and optionally the gradients of the three
// metrics.  A scheduler thread admits queued quotes in arrival order while a
// slot and arena memory are free, computes each admitted quote's occurrence
// table, and every iteration packs a share of the trial blocks of EVERY
// active quote into ONE launch of the forward streaming kernel, so quotes
// that arrive while others are on the GPU join at the next iteration and
// their work overlaps.  A quote whose blocks are all done gets its metrics
// (and backward) and its results are copied to host memory; completion is
// observed with an event and its arena memory is released.
//
// Per-quote results do not depend on what else is in flight: every block of
// a quote is computed by the same kernel in the same order, alone or packed.
#include "arena.h"
#include "occ.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace ara {

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum Stage { kQueued, kForward, kFinishing, kDone, kCancelled };

struct Job {
    int64_t ticket;
    ara_quote q;
    std::vector<int32_t> elt_ids, elt_off;
    int stage = kQueued;
    int slot = -1;
    size_t mem_off = 0, mem_bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t status = ARA_OK;
    // device memory carved from the arena
    char *base = nullptr;
    int32_t *d_off = nullptr, *d_ids = nullptr;
    double *d_lterm = nullptr;
    OccTables *d_tab = nullptr;
    OccTables tab{};
    double *ylt = nullptr, *s_pre = nullptr, *weights = nullptr, *d_res = nullptr;
    void *met_ws = nullptr, *bwd_ws = nullptr;
    size_t met_bytes = 0, bwd_bytes = 0;
    int b_lo = 0, b_hi = 0, next_block = 0;
    hipEvent_t done_ev = nullptr;
    bool finished_host = false;
    // the quote's results, copied out of its result slot when it completes
    // (the slot then serves the next quote): 3 metrics, 3x4 layer gradients,
    // 3 x J x 3 ELT gradients in the quote's ELT order
    std::vector<double> res;
};

struct ServerImpl {
    ara_tables tables{};
    ara_yet yet{};
    const double *elt_terms = nullptr;
    char *arena_base = nullptr;
    Arena arena;
    int max_slots = 0;
    size_t res_doubles = 0;            // per slot: 3 metrics + 3*4 layer grads + 3*n_elts*3 ELT grads
    double *h_res = nullptr;           // pinned host, [max_slots][res_doubles]
    std::vector<int> free_slots;
    hipStream_t st = nullptr;
    OccLayoutSizes z{};
    // forward work-item staging (two iterations in flight)
    static constexpr int kRing = 2;
    static constexpr int kMaxItems = 4096;
    FwdItem *d_items[kRing] = {nullptr, nullptr};
    FwdItem *h_items[kRing] = {nullptr, nullptr};
    hipEvent_t item_ev[kRing] = {nullptr, nullptr};
    bool item_used[kRing] = {false, false};
    int ring = 0;
    int blocks_per_iter = 1024;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> queue;
    std::vector<std::shared_ptr<Job>> active;
    std::map<int64_t, std::shared_ptr<Job>> jobs;
    int64_t next_ticket = 1;
    bool stop = false;
    int32_t fatal = ARA_OK;
    std::thread th;
    // statistics
    int64_t iterations = 0, packed_launches = 0, max_packed_quotes = 0;

    size_t job_bytes(const Job &j) const;
    int32_t setup(Job &j);
    int32_t finish(Job &j);
    void loop();
};

static ara_layers one_layer(const Job &j) {
    ara_layers L{};
    L.n_layers = 1;
    L.elt_off = j.elt_off.data();
    L.elt_ids = j.elt_ids.data();
    return L;
}

size_t ServerImpl::job_bytes(const Job &j) const {
    const int64_t n = j.q.trial_end - j.q.trial_begin;
    Carver c(nullptr);
    c.take<int32_t>(2);
    c.take<int32_t>(j.elt_ids.size() + 1);
    c.take<double>(4);
    c.take<OccTables>(1);
    size_t b = c.bytes() + z.per_layer;
    Carver d(nullptr);
    d.take<double>(static_cast<size_t>(n));   // ylt
    d.take<double>(static_cast<size_t>(n));   // s_pre
    size_t mb = 0;
    ara_metrics_workspace_bytes(1, n, &mb);
    d.take<char>(mb);
    d.take<double>(res_doubles);
    if (j.q.want_grad) {
        d.take<double>(static_cast<size_t>(3) * n);   // weights
        size_t bb = 0;
        ara_layers L = one_layer(j);
        ara_ylt_backward_workspace_bytes(&tables, &yet, &L, 3, &bb);
        d.take<char>(bb);
    }
    return align256(b + d.bytes());
}

int32_t ServerImpl::setup(Job &j) {
    const int64_t n = j.q.trial_end - j.q.trial_begin;
    j.base = arena_base + j.mem_off;
    Carver c(j.base);
    j.d_off = c.take<int32_t>(2);
    j.d_ids = c.take<int32_t>(j.elt_ids.size() + 1);
    j.d_lterm = c.take<double>(4);
    j.d_tab = c.take<OccTables>(1);
    j.tab = occ_carve(c, z, false);
    j.ylt = c.take<double>(static_cast<size_t>(n));
    j.s_pre = c.take<double>(static_cast<size_t>(n));
    ara_metrics_workspace_bytes(1, n, &j.met_bytes);
    j.met_ws = c.take<char>(j.met_bytes);
    j.d_res = c.take<double>(res_doubles);
    if (j.q.want_grad) {
        j.weights = c.take<double>(static_cast<size_t>(3) * n);
        ara_layers L = one_layer(j);
        ara_ylt_backward_workspace_bytes(&tables, &yet, &L, 3, &j.bwd_bytes);
        j.bwd_ws = c.take<char>(j.bwd_bytes);
    }
    ARA_HIP(hipMemcpyAsync(j.d_off, j.elt_off.data(), 2 * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!j.elt_ids.empty())
        ARA_HIP(hipMemcpyAsync(j.d_ids, j.elt_ids.data(), j.elt_ids.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(j.d_lterm, j.q.layer_terms, 4 * sizeof(double), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(j.d_tab, &j.tab, sizeof(OccTables), hipMemcpyHostToDevice, st));
    // the quote's occurrence table; device-side term errors land in the metric workspace header
    int32_t *d_err = static_cast<int32_t *>(j.met_ws);
    int32_t rc = launch_occ(&tables, j.d_off, j.d_ids, elt_terms, j.d_lterm, 1, false, false, j.d_tab, z.n_sr, d_err, st);
    if (rc) return rc;
    j.b_lo = static_cast<int>(j.q.trial_begin / yet.trials_per_block);
    j.b_hi = static_cast<int>((j.q.trial_end + yet.trials_per_block - 1) / yet.trials_per_block);
    j.next_block = j.b_lo;
    return ARA_OK;
}

int32_t ServerImpl::finish(Job &j) {
    const int64_t n = j.q.trial_end - j.q.trial_begin;
    int32_t rc;
    if (n > 0) {
        if ((rc = ara_metrics(j.ylt, 1, n, j.q.p, j.d_res, j.weights, j.met_ws, j.met_bytes, st))) return rc;
        if (j.q.want_grad) {
            ara_layers L = one_layer(j);
            double *ge = j.d_res + 3 + 12;
            double *gl = j.d_res + 3;
            if ((rc = ara_ylt_backward(&tables, &yet, &L, elt_terms, j.d_lterm, j.q.trial_begin, j.q.trial_end, j.s_pre,
                                       3, j.weights, ge, gl, j.bwd_ws, j.bwd_bytes, st)))
                return rc;
        }
    }
    ARA_HIP(hipMemcpyAsync(h_res + static_cast<size_t>(j.slot) * res_doubles, j.d_res, res_doubles * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    ARA_HIP(hipEventRecord(j.done_ev, st));
    return ARA_OK;
}

void ServerImpl::loop() {
    std::vector<std::shared_ptr<Job>> admitted;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop && active.empty()) break;
            admitted.clear();
            while (!stop && !queue.empty() && static_cast<int>(active.size()) < max_slots && !free_slots.empty()) {
                auto j = queue.front();
                if (j->stage == kCancelled) {
                    queue.pop_front();
                    continue;
                }
                const size_t need = job_bytes(*j);
                size_t off = 0;
                if (!arena.alloc(need, &off)) break;   // arrival order: wait for memory
                queue.pop_front();
                j->mem_off = off;
                j->mem_bytes = need;
                j->slot = free_slots.back();
                free_slots.pop_back();
                j->t_admit = now_ms();
                j->stage = kForward;
                active.push_back(j);
                admitted.push_back(j);
            }
        }
        int32_t rc = ARA_OK;
        for (auto &j : admitted) {
            if ((rc = setup(*j))) break;
            hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming);
        }
        // one packed forward launch over a share of every active quote's blocks
        std::vector<Job *> fwd;
        for (auto &j : active)
            if (j->stage == kForward) fwd.push_back(j.get());
        if (!rc && !fwd.empty()) {
            if (item_used[ring]) hipEventSynchronize(item_ev[ring]);
            FwdItem *hi = h_items[ring];
            int n_items = 0;
            const int share = std::max(16, blocks_per_iter / static_cast<int>(fwd.size()));
            for (Job *j : fwd) {
                const int take = std::min(share, j->b_hi - j->next_block);
                for (int k = 0; k < take && n_items < kMaxItems; ++k) {
                    FwdItem &it = hi[n_items++];
                    it.tab = j->d_tab;
                    it.lterm = j->d_lterm;
                    it.block = j->next_block++;
                    it.pad = 0;
                    it.t0 = j->q.trial_begin;
                    it.t1 = j->q.trial_end;
                    it.ylt = j->ylt;
                    it.s_pre = j->s_pre;
                    it.hits = nullptr;
                }
            }
            if (n_items > 0) {
                hipMemcpyAsync(d_items[ring], hi, n_items * sizeof(FwdItem), hipMemcpyHostToDevice, st);
                rc = launch_forward(&yet, z.n_sr, false, false, d_items[ring], n_items, st);
                hipEventRecord(item_ev[ring], st);
                item_used[ring] = true;
                ring = (ring + 1) % kRing;
                ++packed_launches;
                max_packed_quotes = std::max<int64_t>(max_packed_quotes, static_cast<int64_t>(fwd.size()));
            }
            for (Job *j : fwd) {
                if (!rc && j->next_block >= j->b_hi) {
                    j->stage = kFinishing;
                    rc = finish(*j);
                }
            }
        }
        ++iterations;
        // completions
        bool waiting = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (rc) fatal = rc;
            for (auto it = active.begin(); it != active.end();) {
                Job &j = **it;
                bool done = rc != ARA_OK;
                if (!done && j.stage == kFinishing) done = hipEventQuery(j.done_ev) == hipSuccess;
                if (done) {
                    j.t_done = now_ms();
                    j.status = rc;
                    j.stage = kDone;
                    if (rc == ARA_OK) {
                        const double *r = h_res + static_cast<size_t>(j.slot) * res_doubles;
                        const size_t J = j.elt_ids.size();
                        j.res.assign(15 + 9 * J, 0.0);
                        std::copy(r, r + 15, j.res.begin());
                        if (j.q.want_grad)
                            for (int c = 0; c < 3; ++c)
                                for (size_t q = 0; q < J; ++q)
                                    for (int m = 0; m < 3; ++m)
                                        j.res[15 + (c * J + q) * 3 + m] =
                                            r[15 + (static_cast<size_t>(c) * tables.n_elts + j.elt_ids[q]) * 3 + m];
                    }
                    arena.release(j.mem_off, j.mem_bytes);
                    free_slots.push_back(j.slot);
                    it = active.erase(it);
                    cv_done.notify_all();
                } else {
                    if (j.stage == kFinishing) waiting = true;
                    ++it;
                }
            }
            cv_work.notify_all();
        }
        // nothing left to launch: wait briefly for results instead of spinning
        bool any_fwd = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &j : active) any_fwd |= j->stage == kForward;
            any_fwd |= !queue.empty() && !free_slots.empty();
        }
        if (waiting && !any_fwd) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_server_create(const ara_tables *tables, const ara_yet *yet, const double *elt_terms, void *arena,
                                     size_t arena_bytes, int32_t max_slots, void **server) {
    if (!tables || !yet || !elt_terms || !arena || !server) return fail(ARA_E_INVAL, "ara_server_create: null pointer");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (max_slots < 1 || max_slots > 256) return fail(ARA_E_LIMIT, "max_slots must be 1..256");
    auto *S = new ServerImpl();
    S->tables = *tables;
    S->yet = *yet;
    S->elt_terms = elt_terms;
    S->max_slots = max_slots;
    S->z = occ_sizes(tables->catalog, false);
    S->res_doubles = 3 + 12 + static_cast<size_t>(3) * tables->n_elts * 3;
    // reserve the work-item ring at the start of the arena
    const size_t ring_bytes = align256(ServerImpl::kRing * ServerImpl::kMaxItems * sizeof(FwdItem));
    if (arena_bytes <= ring_bytes) {
        delete S;
        return fail(ARA_E_NOSPACE, "arena too small");
    }
    for (int r = 0; r < ServerImpl::kRing; ++r)
        S->d_items[r] = reinterpret_cast<FwdItem *>(static_cast<char *>(arena) + r * ServerImpl::kMaxItems * sizeof(FwdItem));
    S->arena_base = static_cast<char *>(arena) + ring_bytes;
    S->arena.init(arena_bytes - ring_bytes);
    hipError_t e = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&S->h_res), S->res_doubles * max_slots * sizeof(double),
                          hipHostMallocDefault);
    for (int r = 0; e == hipSuccess && r < ServerImpl::kRing; ++r) {
        e = hipHostMalloc(reinterpret_cast<void **>(&S->h_items[r]), ServerImpl::kMaxItems * sizeof(FwdItem),
                          hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->item_ev[r], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "ara_server_create");
    }
    for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->th = std::thread([S] { S->loop(); });
    *server = S;
    return ARA_OK;
}

extern "C" int32_t ara_server_submit(void *server, const ara_quote *q, int64_t *ticket) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S || !q || !ticket) return fail(ARA_E_INVAL, "ara_server_submit: null pointer");
    if (q->n_elts < 0 || q->n_elts > ARA_MAX_ELTS_PER_LAYER) return fail(ARA_E_LIMIT, "quote ELT count out of range");
    if (q->n_elts > 0 && !q->elt_ids) return fail(ARA_E_INVAL, "quote without ELT list");
    for (int i = 0; i < q->n_elts; ++i)
        if (q->elt_ids[i] < 0 || q->elt_ids[i] >= S->tables.n_elts) return fail(ARA_E_RANGE, "quote ELT index out of range");
    if (q->trial_begin < 0 || q->trial_end < q->trial_begin || q->trial_end > S->yet.n_trials)
        return fail(ARA_E_RANGE, "quote trial range outside the YET");
    if (q->trial_end == q->trial_begin) return fail(ARA_E_INVAL, "quote over an empty trial range");
    if (!(q->p > 0.0 && q->p < 1.0)) return fail(ARA_E_INVAL, "quote p must lie in (0, 1)");
    if (q->want_grad && S->yet.n_slices != kSlices)
        return fail(ARA_E_INVAL, "gradients need a resident YET prepared with ARA_PREP_TRANSPOSED");
    const double *t = q->layer_terms;
    if (!(t[0] >= 0.0 && t[0] < INFINITY) || !(t[1] > 0.0) || !(t[2] >= 0.0 && t[2] < INFINITY) || !(t[3] > 0.0))
        return fail(ARA_E_INVAL, "quote layer terms invalid");
    auto j = std::make_shared<Job>();
    j->q = *q;
    j->elt_ids.assign(q->elt_ids, q->elt_ids + q->n_elts);
    j->elt_off = {0, q->n_elts};
    j->q.elt_ids = nullptr;
    j->t_submit = now_ms();
    if (S->job_bytes(*j) > S->arena.size()) return fail(ARA_E_NOSPACE, "quote larger than the whole arena");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return fail(S->fatal, "server stopped after a device error");
    j->ticket = S->next_ticket++;
    S->jobs[j->ticket] = j;
    S->queue.push_back(j);
    *ticket = j->ticket;
    S->cv_work.notify_all();
    return ARA_OK;
}

static void fill_result(ServerImpl *S, const Job &j, ara_quote_result *out) {
    out->status = j.status;
    out->n_elts = static_cast<int32_t>(j.elt_ids.size());
    out->t_submit_ms = j.t_submit;
    out->t_admit_ms = j.t_admit;
    out->t_done_ms = j.t_done;
    (void)S;
    const size_t J = j.elt_ids.size();
    if (j.res.size() < 15 + 9 * J) {   // failed quote: no results
        for (int m = 0; m < 3; ++m) out->metrics[m] = 0.0;
        for (int m = 0; m < 12; ++m) out->grad_layer[m / 4][m % 4] = 0.0;
        return;
    }
    const double *r = j.res.data();
    for (int m = 0; m < 3; ++m) out->metrics[m] = r[m];
    if (j.q.want_grad) {
        for (int m = 0; m < 12; ++m) out->grad_layer[m / 4][m % 4] = r[3 + m];
        if (out->grad_elt)   // [3][J][3] in the quote's ELT order
            for (size_t i = 0; i < 9 * J; ++i) out->grad_elt[i] = r[15 + i];
    } else {
        for (int m = 0; m < 12; ++m) out->grad_layer[m / 4][m % 4] = 0.0;
    }
}

extern "C" int32_t ara_server_poll(void *server, int64_t ticket, ara_quote_result *out) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S || !out) return fail(ARA_E_INVAL, "ara_server_poll: null pointer");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(ARA_E_RANGE, "unknown ticket");
    const Job &j = *it->second;
    if (j.stage == kCancelled) {
        S->jobs.erase(it);
        return fail(ARA_E_INVAL, "quote was cancelled");
    }
    if (j.stage != kDone) return ARA_E_BUSY;
    fill_result(S, j, out);
    S->jobs.erase(it);
    return ARA_OK;
}

extern "C" int32_t ara_server_wait(void *server, int64_t ticket, ara_quote_result *out) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S || !out) return fail(ARA_E_INVAL, "ara_server_wait: null pointer");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(ARA_E_RANGE, "unknown ticket");
    std::shared_ptr<Job> j = it->second;
    S->cv_done.wait(lk, [&] { return j->stage == kDone || j->stage == kCancelled || S->fatal != ARA_OK; });
    if (j->stage == kCancelled) {
        S->jobs.erase(j->ticket);
        return fail(ARA_E_INVAL, "quote was cancelled");
    }
    if (j->stage != kDone) return fail(S->fatal, "server stopped after a device error");
    fill_result(S, *j, out);
    S->jobs.erase(j->ticket);
    return j->status;
}

extern "C" int32_t ara_server_cancel(void *server, int64_t ticket) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S) return fail(ARA_E_INVAL, "ara_server_cancel: null pointer");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(ARA_E_RANGE, "unknown ticket");
    if (it->second->stage != kQueued) return ARA_E_BUSY;   // already on the device: runs to completion
    it->second->stage = kCancelled;
    S->cv_done.notify_all();
    return ARA_OK;
}

extern "C" int32_t ara_server_stats(void *server, int64_t *stats) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S || !stats) return fail(ARA_E_INVAL, "ara_server_stats: null pointer");
    std::lock_guard<std::mutex> lk(S->mu);
    stats[0] = S->iterations;
    stats[1] = S->packed_launches;
    stats[2] = S->max_packed_quotes;
    stats[3] = static_cast<int64_t>(S->queue.size());
    stats[4] = static_cast<int64_t>(S->active.size());
    stats[5] = static_cast<int64_t>(S->arena.free_bytes());
    return ARA_OK;
}

extern "C" int32_t ara_server_destroy(void *server) {
    auto *S = static_cast<ServerImpl *>(server);
    if (!S) return ARA_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto &j : S->queue) j->stage = kCancelled;
        S->queue.clear();
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    hipStreamSynchronize(S->st);
    for (auto &kv : S->jobs)
        if (kv.second->done_ev) hipEventDestroy(kv.second->done_ev);
    for (int r = 0; r < ServerImpl::kRing; ++r) {
        if (S->item_ev[r]) hipEventDestroy(S->item_ev[r]);
        if (S->h_items[r]) hipHostFree(S->h_items[r]);
    }
    if (S->h_res) hipHostFree(S->h_res);
    if (S->st) hipStreamDestroy(S->st);
    delete S;
    return ARA_OK;
}

extern "C" int32_t ara_server_arena_bytes(const ara_tables *tables, const ara_yet *yet, int32_t quotes_with_grad,
                                          size_t *bytes) {
    if (!tables || !yet || !bytes || quotes_with_grad < 1) return fail(ARA_E_INVAL, "ara_server_arena_bytes: bad argument");
    ServerImpl tmp;
    tmp.tables = *tables;
    tmp.yet = *yet;
    tmp.z = occ_sizes(tables->catalog, false);
    tmp.res_doubles = 3 + 12 + static_cast<size_t>(3) * tables->n_elts * 3;
    Job j;
    j.q.trial_begin = 0;
    j.q.trial_end = yet->n_trials;
    j.q.want_grad = 1;
    j.elt_ids.assign(ARA_MAX_ELTS_PER_LAYER / 4, 0);
    j.elt_off = {0, static_cast<int32_t>(j.elt_ids.size())};
    *bytes = align256(ServerImpl::kRing * ServerImpl::kMaxItems * sizeof(FwdItem)) +
             static_cast<size_t>(quotes_with_grad) * tmp.job_bytes(j);
    return ARA_OK;
}
