// Quote server: continuous batching of pricing requests over the resident
// YET and ELT tables.
//
// A request ("quote") is a candidate layer -- a subset of the resident ELTs,
// its occurrence and aggregate terms -- over a contiguous trial range, with
// the tail probability for PML/TVaR and optionally the gradients of the three
// metrics.  The scheduling (admission by slot and memory, the circular scan
// of the trial blocks that packs every active quote's items into one launch
// of the forward kernel, completion and retirement) is the HIP-free core in
// quote_sched.cpp; this file is its executor on the device: each admitted quote's
// occurrence table, the packed forward launches (the items of one block dealt
// to one XCD, their codes loaded through its L2), the metrics of the quotes
// that a launch finishes (one row each, all in one set of launches), and each
// finished quote's backward and result copy, observed with an event.
//
// Per-quote results do not depend on what else is in flight: every block of
// a quote is computed by the same kernel in the same order, alone or packed.
#include "occ.h"
#include "quote_sched.h"

#include <algorithm>
#include <memory>
#include <vector>

namespace ara {

static ara_layers one_layer(const int32_t *off, const int32_t *ids) {
    ara_layers L{};
    L.n_layers = 1;
    L.elt_off = off;
    L.elt_ids = ids;
    return L;
}

// The device side of one admitted quote, carved from its arena range.
struct DevJob {
    int32_t h_off[2] = {0, 0};
    int32_t *d_off = nullptr, *d_ids = nullptr, *d_err = nullptr;
    double *d_lterm = nullptr;
    OccTables *d_tab = nullptr;
    OccTables tab{};
    double *ylt = nullptr, *s_pre = nullptr, *weights = nullptr, *d_res = nullptr;
    void *met_ws = nullptr, *bwd_ws = nullptr;
    size_t met_bytes = 0, bwd_bytes = 0;
    MetRow row{};                          // its metrics row over ylt, met_ws, d_res and weights
    hipEvent_t done_ev = nullptr;
};

class HipExecutor final : public SchedExecutor {
   public:
    static constexpr int kRing = 2;        // forward launches whose item lists may be in flight
    static constexpr int kMaxItems = 8192;
    static constexpr int kMaxRows = 256;   // quotes finishing together: at most one per slot

    ara_tables tables{};
    ara_yet yet{};
    const double *elt_terms = nullptr;
    char *arena_base = nullptr;
    OccLayoutSizes z{};
    size_t res_doubles = 0;                // per slot: 3 metrics + 3*4 layer grads + 3*n_elts*3 ELT grads
    // A quote's status word and its results sit side by side in its arena
    // range (the status first, kResOff bytes before the results) and come back
    // in one copy into its slot of the pinned host stage.
    static constexpr size_t kResOff = 256;
    size_t stage_bytes = 0;                // kResOff + res_doubles * 8
    char *h_stage = nullptr;               // pinned host, [max_slots][stage_bytes]
    hipStream_t st = nullptr;
    // Gradient quotes' backward passes (short chains of small kernels) run on
    // a few streams of their own after the metrics, so that those of the
    // quotes finishing together overlap; default priority like st.
    static constexpr int kFinStreams = 4;
    hipStream_t fst[kFinStreams] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t met_ev = nullptr;           // the metrics of the latest finishing set are done
    int fin_next = 0;
    FwdItem *d_items[kRing] = {nullptr, nullptr};
    FwdItem *h_items[kRing] = {nullptr, nullptr};
    hipEvent_t item_ev[kRing] = {nullptr, nullptr};
    bool item_used[kRing] = {false, false};
    int ring = 0;
    // the metrics rows of the quotes finishing after one launch, same ring scheme
    MetRow *d_rows[kRing] = {nullptr, nullptr};
    MetRow *h_rows[kRing] = {nullptr, nullptr};
    hipEvent_t row_ev[kRing] = {nullptr, nullptr};
    bool row_used[kRing] = {false, false};
    int row_ring = 0;
    int64_t events_created = 0, events_destroyed = 0;

    size_t bytes_of(const SchedJob &j) const {
        const int64_t n = j.q.trial_end - j.q.trial_begin;
        Carver c(nullptr);
        c.take<int32_t>(2);
        c.take<int32_t>(j.elt_ids.size() + 1);
        c.take<double>(4);
        c.take<OccTables>(1);
        c.take<int32_t>(kResOff / sizeof(int32_t));   // the quote's device-side status word
        c.take<double>(res_doubles);
        size_t b = c.bytes() + z.per_layer;
        Carver d(nullptr);
        d.take<double>(static_cast<size_t>(n));   // ylt
        d.take<double>(static_cast<size_t>(n));   // s_pre
        size_t mb = 0;
        ara_metrics_workspace_bytes(1, n, &mb);
        d.take<char>(mb);
        if (j.q.want_grad) {
            d.take<double>(static_cast<size_t>(3) * n);   // weights
            size_t bb = 0;
            const int32_t off[2] = {0, static_cast<int32_t>(j.elt_ids.size())};
            ara_layers L = one_layer(off, j.elt_ids.data());
            ara_ylt_backward_workspace_bytes(&tables, &yet, &L, 3, &bb);
            d.take<char>(bb);
        }
        return align256(b + d.bytes());
    }

    int32_t validate(const ara_quote &q, std::string *err) override {
        if (q.want_grad && yet.n_slices != kSlices) {
            *err = "gradients need a resident YET prepared with ARA_PREP_TRANSPOSED";
            return ARA_E_INVAL;
        }
        return ARA_OK;
    }

    size_t job_bytes(const SchedJob &j) override { return bytes_of(j); }

    int32_t setup(SchedJob &j, std::string *err) override {
        auto *d = new DevJob();
        j.exec = d;
        const int64_t n = j.q.trial_end - j.q.trial_begin;
        Carver c(arena_base + j.mem_off);
        d->d_off = c.take<int32_t>(2);
        d->d_ids = c.take<int32_t>(j.elt_ids.size() + 1);
        d->d_lterm = c.take<double>(4);
        d->d_tab = c.take<OccTables>(1);
        d->d_err = c.take<int32_t>(kResOff / sizeof(int32_t));
        d->d_res = c.take<double>(res_doubles);
        d->tab = occ_carve(c, z, false);
        d->ylt = c.take<double>(static_cast<size_t>(n));
        d->s_pre = c.take<double>(static_cast<size_t>(n));
        ara_metrics_workspace_bytes(1, n, &d->met_bytes);
        d->met_ws = c.take<char>(d->met_bytes);
        d->h_off[1] = static_cast<int32_t>(j.elt_ids.size());
        if (j.q.want_grad) {
            d->weights = c.take<double>(static_cast<size_t>(3) * n);
            ara_layers L = one_layer(d->h_off, j.elt_ids.data());
            ara_ylt_backward_workspace_bytes(&tables, &yet, &L, 3, &d->bwd_bytes);
            d->bwd_ws = c.take<char>(d->bwd_bytes);
        }
        d->row = metrics_row(d->met_ws, d->ylt, n, j.q.p, d->d_res, d->weights);
        hipError_t e = hipEventCreateWithFlags(&d->done_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            d->done_ev = nullptr;
            *err = "hipEventCreateWithFlags failed";
            return ARA_E_HIP;
        }
        ++events_created;
        // the quote's lists, terms and table descriptor in one copy, which
        // also clears its status word and results
        HeadImage img(arena_base + j.mem_off);
        img.put(d->d_off, d->h_off, 2);
        img.put(d->d_ids, j.elt_ids.data(), j.elt_ids.size());
        img.put(d->d_lterm, j.q.layer_terms, 4);
        img.put(d->d_tab, &d->tab, 1);
        img.cover(d->d_res + res_doubles);
        int32_t rc = img.send(st);
        if (rc) *err = "copy of the quote's head failed";
        // the quote's occurrence table; invalid terms set its own status word
        if (!rc && (rc = launch_occ(&tables, d->d_off, d->d_ids, elt_terms, d->d_lterm, 1, false, false, d->d_tab, z.n_sr,
                                    d->d_err, st)))
            *err = "occurrence table launch failed";
        return rc;
    }

    int32_t launch(const std::vector<SchedItem> &items, bool shared, std::string *err) override {
        if (items.empty()) return ARA_OK;
        if (static_cast<int>(items.size()) > kMaxItems) {
            *err = "too many items in one launch";
            return ARA_E_LIMIT;
        }
        int32_t rc;
        if (item_used[ring] && (rc = hip_step(hipEventSynchronize(item_ev[ring]), err))) return rc;
        FwdItem *hi = h_items[ring];
        for (size_t i = 0; i < items.size(); ++i) {
            FwdItem &it = hi[i];
            it = FwdItem{};
            it.block = -1;
            const SchedJob *j = items[i].job;
            if (!j) continue;
            const DevJob *d = static_cast<const DevJob *>(j->exec);
            it.tab = d->d_tab;
            it.lterm = d->d_lterm;
            it.block = items[i].block;
            it.t0 = j->q.trial_begin;
            it.t1 = j->q.trial_end;
            it.ylt = d->ylt;
            it.s_pre = d->s_pre;
            it.hits = nullptr;
        }
        if ((rc = hip_step(hipMemcpyAsync(d_items[ring], hi, items.size() * sizeof(FwdItem), hipMemcpyHostToDevice, st),
                           err)))
            return rc;
        if ((rc = launch_forward(&yet, z.n_sr, false, false, d_items[ring], static_cast<int>(items.size()), st, nullptr,
                                 shared))) {
            *err = "forward launch failed";
            return rc;
        }
        if ((rc = hip_step(hipEventRecord(item_ev[ring], st), err))) return rc;
        item_used[ring] = true;
        ring = (ring + 1) % kRing;
        return ARA_OK;
    }

    int32_t finish(SchedJob &j, std::string *err) override {
        SchedJob *one = &j;
        return finish_all(std::vector<SchedJob *>(1, one), err);
    }

    // The metrics of all the quotes at once (one row each, in one set of
    // launches), then each quote's backward and its copy back.
    int32_t finish_all(const std::vector<SchedJob *> &jobs, std::string *err) override {
        if (jobs.empty()) return ARA_OK;
        if (static_cast<int>(jobs.size()) > kMaxRows) {
            *err = "too many quotes finishing at once";
            return ARA_E_LIMIT;
        }
        int32_t rc;
        if (row_used[row_ring] && (rc = hip_step(hipEventSynchronize(row_ev[row_ring]), err))) return rc;
        MetRow *hr = h_rows[row_ring];
        int max_nwg = 1;
        int64_t max_n = 1;
        bool any_w = false;
        for (size_t i = 0; i < jobs.size(); ++i) {
            const DevJob *d = static_cast<const DevJob *>(jobs[i]->exec);
            hr[i] = d->row;
            max_nwg = std::max(max_nwg, static_cast<int>(d->row.nwg));
            max_n = std::max(max_n, d->row.n);
            any_w = any_w || d->row.w != nullptr;
        }
        if ((rc = hip_step(hipMemcpyAsync(d_rows[row_ring], hr, jobs.size() * sizeof(MetRow), hipMemcpyHostToDevice, st),
                           err)))
            return rc;
        if ((rc = metrics_rows(d_rows[row_ring], static_cast<int>(jobs.size()), max_nwg, max_n, any_w, st))) {
            *err = "metrics failed";
            return rc;
        }
        if ((rc = hip_step(hipEventRecord(row_ev[row_ring], st), err))) return rc;
        row_used[row_ring] = true;
        row_ring = (row_ring + 1) % kRing;
        if ((rc = hip_step(hipEventRecord(met_ev, st), err))) return rc;
        for (SchedJob *jp : jobs) {
            SchedJob &j = *jp;
            DevJob *d = static_cast<DevJob *>(j.exec);
            hipStream_t s = st;   // a quote without gradients only copies its results back
            if (j.q.want_grad) {
                // after the metrics (its weights), on the next backward stream
                s = fst[fin_next];
                fin_next = (fin_next + 1) % kFinStreams;
                if ((rc = hip_step(hipStreamWaitEvent(s, met_ev, 0), err))) return rc;
                ara_layers L = one_layer(d->h_off, j.elt_ids.data());
                double *ge = d->d_res + 3 + 12;
                double *gl = d->d_res + 3;
                if ((rc = ara_ylt_backward(&tables, &yet, &L, elt_terms, d->d_lterm, j.q.trial_begin, j.q.trial_end,
                                           d->s_pre, 3, d->weights, ge, gl, d->bwd_ws, d->bwd_bytes, s))) {
                    *err = "backward failed";
                    return rc;
                }
            }
            const size_t slot = static_cast<size_t>(j.slot);
            if ((rc = hip_step(
                     hipMemcpyAsync(h_stage + slot * stage_bytes, d->d_err, stage_bytes, hipMemcpyDeviceToHost, s),
                     err)))
                return rc;
            if ((rc = hip_step(hipEventRecord(d->done_ev, s), err))) return rc;
        }
        return ARA_OK;
    }

    bool done(SchedJob &j) override {
        const DevJob *d = static_cast<const DevJob *>(j.exec);
        return hipEventQuery(d->done_ev) != hipErrorNotReady;
    }

    int32_t collect(SchedJob &j) override {
        const DevJob *d = static_cast<const DevJob *>(j.exec);
        if (hipEventQuery(d->done_ev) != hipSuccess) return ARA_E_HIP;
        const char *stage = h_stage + static_cast<size_t>(j.slot) * stage_bytes;
        const int32_t status = *reinterpret_cast<const int32_t *>(stage);
        if (status != ARA_OK) return status;
        const double *r = reinterpret_cast<const double *>(stage + kResOff);
        const size_t J = j.elt_ids.size();
        j.res.assign(15 + 9 * J, 0.0);
        std::copy(r, r + 15, j.res.begin());
        if (j.q.want_grad)
            for (int c = 0; c < 3; ++c)
                for (size_t q = 0; q < J; ++q)
                    for (int m = 0; m < 3; ++m)
                        j.res[15 + (c * J + q) * 3 + m] =
                            r[15 + (static_cast<size_t>(c) * tables.n_elts + j.elt_ids[q]) * 3 + m];
        return ARA_OK;
    }

    void release(SchedJob &j) override {
        DevJob *d = static_cast<DevJob *>(j.exec);
        if (!d) return;
        if (d->done_ev) {
            hipEventDestroy(d->done_ev);
            ++events_destroyed;
        }
        delete d;
        j.exec = nullptr;
    }

    void settle() override {
        const int last = (ring + kRing - 1) % kRing;
        if (item_used[last]) hipEventSynchronize(item_ev[last]);
        const int last_rows = (row_ring + kRing - 1) % kRing;
        if (row_used[last_rows]) hipEventSynchronize(row_ev[last_rows]);
    }

   private:
    static int32_t hip_step(hipError_t e, std::string *err) {
        if (e == hipSuccess) return ARA_OK;
        *err = hipGetErrorString(e);
        return ARA_E_HIP;
    }
};

struct Server {
    HipExecutor ex;
    std::unique_ptr<Scheduler> sched;
};

// The head of the arena: the two item lists, then the two row lists.
static size_t items_bytes() { return align256(HipExecutor::kRing * HipExecutor::kMaxItems * sizeof(FwdItem)); }
static size_t ring_bytes() {
    return items_bytes() + align256(HipExecutor::kRing * HipExecutor::kMaxRows * sizeof(MetRow));
}

static void free_host(Server *S) {
    for (int r = 0; r < HipExecutor::kRing; ++r) {
        if (S->ex.item_ev[r]) hipEventDestroy(S->ex.item_ev[r]);
        if (S->ex.h_items[r]) hipHostFree(S->ex.h_items[r]);
        if (S->ex.row_ev[r]) hipEventDestroy(S->ex.row_ev[r]);
        if (S->ex.h_rows[r]) hipHostFree(S->ex.h_rows[r]);
    }
    if (S->ex.h_stage) hipHostFree(S->ex.h_stage);
    for (int i = 0; i < HipExecutor::kFinStreams; ++i)
        if (S->ex.fst[i]) hipStreamDestroy(S->ex.fst[i]);
    if (S->ex.met_ev) hipEventDestroy(S->ex.met_ev);
    if (S->ex.st) hipStreamDestroy(S->ex.st);
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_server_create(const ara_tables *tables, const ara_yet *yet, const double *elt_terms, void *arena,
                                     size_t arena_bytes, int32_t max_slots, void **server) {
    if (!tables || !yet || !elt_terms || !arena || !server) return fail(ARA_E_INVAL, "ara_server_create: null pointer");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (max_slots < 1 || max_slots > 256) return fail(ARA_E_LIMIT, "max_slots must be 1..256");
    if (arena_bytes <= ring_bytes()) return fail(ARA_E_NOSPACE, "arena too small");
    // the resident ELT terms are checked once here: quotes read them on the device
    std::vector<double> et(static_cast<size_t>(tables->n_elts) * 3);
    if (!et.empty()) {
        ARA_HIP(hipMemcpy(et.data(), elt_terms, et.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int32_t k = 0; k < tables->n_elts; ++k) {
            const double s = et[3 * k], r = et[3 * k + 1], l = et[3 * k + 2];
            if (!(s > 0.0 && s < INFINITY) || !(r >= 0.0 && r < INFINITY) || !(l > 0.0))
                return fail(ARA_E_INVAL, "resident ELT " + std::to_string(k) + " has invalid terms");
        }
    }
    auto *S = new Server();
    HipExecutor &X = S->ex;
    X.tables = *tables;
    X.yet = *yet;
    X.elt_terms = elt_terms;
    X.z = occ_sizes(tables->catalog, false);
    X.res_doubles = 3 + 12 + static_cast<size_t>(3) * tables->n_elts * 3;
    X.stage_bytes = HipExecutor::kResOff + X.res_doubles * sizeof(double);
    for (int r = 0; r < HipExecutor::kRing; ++r)
        X.d_items[r] = reinterpret_cast<FwdItem *>(static_cast<char *>(arena) + r * HipExecutor::kMaxItems * sizeof(FwdItem));
    for (int r = 0; r < HipExecutor::kRing; ++r)
        X.d_rows[r] = reinterpret_cast<MetRow *>(static_cast<char *>(arena) + items_bytes() +
                                                 r * HipExecutor::kMaxRows * sizeof(MetRow));
    X.arena_base = static_cast<char *>(arena) + ring_bytes();
    hipError_t e = hipStreamCreateWithFlags(&X.st, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < HipExecutor::kFinStreams; ++i)
        e = hipStreamCreateWithFlags(&X.fst[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&X.met_ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&X.h_stage), X.stage_bytes * max_slots, hipHostMallocDefault);
    for (int r = 0; e == hipSuccess && r < HipExecutor::kRing; ++r) {
        e = hipHostMalloc(reinterpret_cast<void **>(&X.h_items[r]), HipExecutor::kMaxItems * sizeof(FwdItem),
                          hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&X.item_ev[r], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&X.h_rows[r]), HipExecutor::kMaxRows * sizeof(MetRow),
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&X.row_ev[r], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        free_host(S);
        delete S;
        return hip_fail(e, "ara_server_create");
    }
    SchedConfig cfg;
    cfg.n_trials = yet->n_trials;
    cfg.trials_per_block = yet->trials_per_block;
    cfg.n_blocks = yet->n_blocks;
    cfg.n_elts = tables->n_elts;
    cfg.arena_bytes = arena_bytes - ring_bytes();
    cfg.max_slots = max_slots;
    cfg.max_items = HipExecutor::kMaxItems;
    cfg.n_xcd = kXcds;
    cfg.xcd_slots = 2 * device_cu_count() / kXcds;   // two forward workgroups per CU
    S->sched.reset(new Scheduler(&S->ex, cfg));
    S->sched->start();
    *server = S;
    return ARA_OK;
}

extern "C" int32_t ara_server_submit(void *server, const ara_quote *q, int64_t *ticket) {
    auto *S = static_cast<Server *>(server);
    if (!S || !q || !ticket) return fail(ARA_E_INVAL, "ara_server_submit: null pointer");
    std::string err;
    const int32_t rc = S->sched->submit(*q, ticket, &err);
    return rc ? fail(rc, err) : ARA_OK;
}

static void fill_result(const SchedJob &j, ara_quote_result *out) {
    out->status = j.status;
    out->n_elts = static_cast<int32_t>(j.elt_ids.size());
    out->t_submit_ms = j.t_submit;
    out->t_admit_ms = j.t_admit;
    out->t_done_ms = j.t_done;
    const size_t J = j.elt_ids.size();
    for (int m = 0; m < 3; ++m) out->metrics[m] = 0.0;
    for (int m = 0; m < 12; ++m) out->grad_layer[m / 4][m % 4] = 0.0;
    if (j.status != ARA_OK || j.res.size() < 15 + 9 * J) return;   // failed quote: no results
    const double *r = j.res.data();
    for (int m = 0; m < 3; ++m) out->metrics[m] = r[m];
    if (j.q.want_grad) {
        for (int m = 0; m < 12; ++m) out->grad_layer[m / 4][m % 4] = r[3 + m];
        if (out->grad_elt)   // [3][J][3] in the quote's ELT order
            for (size_t i = 0; i < 9 * J; ++i) out->grad_elt[i] = r[15 + i];
    }
}

extern "C" int32_t ara_server_poll(void *server, int64_t ticket, ara_quote_result *out) {
    auto *S = static_cast<Server *>(server);
    if (!S || !out) return fail(ARA_E_INVAL, "ara_server_poll: null pointer");
    std::shared_ptr<SchedJob> j;
    std::string err;
    const int32_t rc = S->sched->poll(ticket, &j, &err);
    if (rc == ARA_E_BUSY) return rc;
    if (rc) return fail(rc, err);
    fill_result(*j, out);
    return j->status ? fail(j->status, "quote failed on the device") : ARA_OK;
}

extern "C" int32_t ara_server_wait(void *server, int64_t ticket, ara_quote_result *out) {
    auto *S = static_cast<Server *>(server);
    if (!S || !out) return fail(ARA_E_INVAL, "ara_server_wait: null pointer");
    std::shared_ptr<SchedJob> j;
    std::string err;
    const int32_t rc = S->sched->wait(ticket, &j, &err);
    if (rc) return fail(rc, err);
    fill_result(*j, out);
    return j->status ? fail(j->status, "quote failed on the device") : ARA_OK;
}

extern "C" int32_t ara_server_cancel(void *server, int64_t ticket) {
    auto *S = static_cast<Server *>(server);
    if (!S) return fail(ARA_E_INVAL, "ara_server_cancel: null pointer");
    std::string err;
    const int32_t rc = S->sched->cancel(ticket, &err);
    if (rc == ARA_E_BUSY) return rc;
    return rc ? fail(rc, err) : ARA_OK;
}

extern "C" int32_t ara_server_stats(void *server, int64_t *stats) {
    auto *S = static_cast<Server *>(server);
    if (!S || !stats) return fail(ARA_E_INVAL, "ara_server_stats: null pointer");
    S->sched->stats(stats);
    return ARA_OK;
}

extern "C" int32_t ara_server_destroy(void *server) {
    auto *S = static_cast<Server *>(server);
    if (!S) return ARA_OK;
    S->sched->stop();   // drains the active quotes: every event is destroyed by then
    hipStreamSynchronize(S->ex.st);
    free_host(S);
    delete S;
    return ARA_OK;
}

extern "C" int32_t ara_server_arena_bytes(const ara_tables *tables, const ara_yet *yet, int32_t quotes_with_grad,
                                          size_t *bytes) {
    if (!tables || !yet || !bytes || quotes_with_grad < 1) return fail(ARA_E_INVAL, "ara_server_arena_bytes: bad argument");
    HipExecutor tmp;
    tmp.tables = *tables;
    tmp.yet = *yet;
    tmp.z = occ_sizes(tables->catalog, false);
    tmp.res_doubles = 3 + 12 + static_cast<size_t>(3) * tables->n_elts * 3;
    SchedJob j;
    j.q.trial_begin = 0;
    j.q.trial_end = yet->n_trials;
    j.q.want_grad = 1;
    j.elt_ids.assign(ARA_MAX_ELTS_PER_LAYER / 4, 0);
    *bytes = ring_bytes() + static_cast<size_t>(quotes_with_grad) * tmp.bytes_of(j);
    return ARA_OK;
}
