// Per-occurrence losses (the event-level YLT) and the per-year maximum
// occurrence loss: step four of Algorithm 1 taken literally, in storage
// order -- running total of the occurrence losses, aggregate retention and
// limit on each running total, then each occurrence's increment.  The sum
// of a trial's increments is its year loss; their maximum is the occurrence
// loss behind occurrence-exceedance metrics.
//
// One wavefront per trial, 1024 consecutive occurrences per step: the event
// IDs stream from the caller's trial-major YET (storage order is needed
// here, so the bucketed layout cannot serve).  Each workgroup first loads a
// 1-Mbit filter of the layer's set events into LDS (the set-event bitmap
// folded onto 2^20 bits by OR); only occurrences whose filter bit is set
// (the set events plus a few that share a bit) read the bitmap word with its
// rank, and only set events read their value, from the cache-resident
// occurrence table.  The address unit serves the active lanes of a gather
// one at a time, so these reads stay masked to the lanes that need them.
// The running total is formed on a transposed copy of four 64-occurrence
// slices (staged in LDS, each lane then holding four consecutive
// occurrences): a prefix inside the lane, one wavefront scan (DPP) across
// lanes, the previous slices' total carried in.
#include "occ.h"
#include "wave.h"

#include <algorithm>
#include <vector>

namespace ara {

constexpr int kYeltThreads = 1024;
constexpr int kYeltSteps = 16;          // 64-occurrence slices per step (8 and 20 measured slower)
constexpr int kYeltGroup = 4;           // slices per transposed scan

struct YeltParams {
    const int64_t *off;
    const int32_t *ids;
    int32_t catalog;
    int32_t pad;
    int64_t t0, t1;
    int64_t occ_begin, occ_count;
    const OccTables *tabs;
    const uint32_t *filter;   // [n_layers][kFilterWords]
    const double *lterms;
    double *yelt;       // [n_layers][occ_count]
    double *occ_max;    // [n_layers][t1 - t0]
    int32_t *err;
};

// One step: 64 * kYeltSteps consecutive occurrences of one trial.  The next
// step's event IDs are loaded (streaming, past the cache) before the current
// step's table lookups, so the ID stream's latency hides behind them; the
// occurrence table stays cache-resident because neither the ID stream nor the
// output stream allocates in the cache.
// The layer's set-event bitmap folded onto kFilterWords words by OR.
__global__ __launch_bounds__(256) void k_yelt_filter(const OccTables *__restrict__ tabs, int n_words,
                                                     uint32_t *__restrict__ filter) {
    const int j = blockIdx.y;
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kFilterWords) return;
    const OccTables T = tabs[j];
    uint32_t f = 0;
    for (int i = w; i < n_words; i += kFilterWords) f |= T.br[i].x;
    filter[static_cast<size_t>(j) * kFilterWords + w] = f;
}

// Global-memory views of the occurrence table: pointers loaded from memory
// are generic, and generic loads are waited for together with LDS traffic.
template <typename T>
using gmem = const __attribute__((address_space(1))) T *;

__global__ __launch_bounds__(kYeltThreads) void k_yelt(YeltParams P) {
    __shared__ uint32_t filt[kFilterWords];
    __shared__ double stage[kYeltThreads / kWave][kYeltGroup * kWave];   // one wavefront's transposed slices
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kFilterWords; i += blockDim.x)
        filt[i] = P.filter[static_cast<size_t>(j) * kFilterWords + i];
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *st = stage[wv];
    const int64_t gw = static_cast<int64_t>(blockIdx.x) * (kYeltThreads / kWave) + wv;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (kYeltThreads / kWave);
    const OccTables T = P.tabs[j];
    const gmem<unsigned long long> gbr = (gmem<unsigned long long>)T.br;   // (bits, rank) words, one per 32 events
    const gmem<double> gvals = (gmem<double>)T.vals;
    const gmem<int32_t> gids = (gmem<int32_t>)P.ids;
    const gmem<int32_t> gdummy = (gmem<int32_t>)(P.filter + static_cast<size_t>(j) * kFilterWords);
    const gmem<int64_t> goff = (gmem<int64_t>)P.off;
    const double aggR = P.lterms[4 * j + 2], aggL = P.lterms[4 * j + 3];
    double *Y = P.yelt + static_cast<size_t>(j) * P.occ_count;
    double *M = P.occ_max + static_cast<size_t>(j) * (P.t1 - P.t0);
    constexpr int kStep = kWave * kYeltSteps;

    // occurrences [lo, hi) of a trial, empty (and flagged) if they fall
    // outside the caller's occurrence range
    auto checked = [&](int64_t lo, int64_t hi, int64_t &a, int64_t &b) {
        a = lo;
        b = hi;
        if (a < P.occ_begin || b > P.occ_begin + P.occ_count || b < a) {
            if (lane == 0) atomicCAS(P.err, 0, ARA_E_RANGE);
            b = a;   // nothing of this trial is read or written
        }
    };
    // cursor (uniform over the wavefront): trial t, its occurrences [a, b),
    // step start base; na, nb: the offsets of trial t + nw (when it exists),
    // loaded a trial ahead
    int64_t t = P.t0 + gw;
    if (t >= P.t1) return;
    int64_t a, b;
    checked(goff[t], goff[t + 1], a, b);
    int64_t base = a, na = 0, nb = 0;
    if (t + nw < P.t1) {
        na = goff[t + nw];
        nb = goff[t + nw + 1];
    }
    // IDs [from, from + kStep) capped at end, lanes past it re-reading the
    // last one; a wavefront with none reads its filter words instead.  The
    // loads carry no branch.
    int32_t en[kYeltSteps];
    auto fetch = [&](int64_t from, int64_t end) {
        const int64_t n = min<int64_t>(end - from, kStep);
        const gmem<int32_t> src = n > 0 ? gids + from : gdummy;
        const int last = n > 0 ? static_cast<int>(n) - 1 : 0;
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) en[k] = __builtin_nontemporal_load(src + min(k * kWave + lane, last));
    };
    // Waiting for the IDs where they are consumed: at the top of the loop
    // they are then complete on every path, and the previous step's stores
    // (issued after them) are not waited for there.
    auto consume_ids = [&]() {
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) asm volatile("" ::"v"(en[k]));
    };
    fetch(base, b);
    consume_ids();
    double carry = 0.0, mx = 0.0;
    bool first = true;   // the next slice group opens its trial
    while (true) {
        const int64_t ct = t, cbase = base;
        const int crem = static_cast<int>(min<int64_t>(b - base, kStep));   // occurrences in this step
        int32_t e[kYeltSteps];
        bool in[kYeltSteps];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            in[k] = k * kWave + lane < crem;
            const bool ok = static_cast<uint32_t>(en[k]) < static_cast<uint32_t>(P.catalog);
            bad = bad || (in[k] && !ok);
            in[k] = in[k] && ok;
            e[k] = in[k] ? en[k] : 0;
        }
        if (__ballot(bad) != 0 && lane == 0) atomicCAS(P.err, 0, ARA_E_RANGE);
        // filter; the bitmap word (with its rank) of each maybe-set event,
        // word e/32 of the table
        bool maybe[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const uint32_t f = filt[(static_cast<uint32_t>(e[k]) >> 5) & (kFilterWords - 1)];
            maybe[k] = in[k] & (__builtin_amdgcn_ubfe(f, static_cast<uint32_t>(e[k]), 1) != 0u);
        }
        unsigned long long wq[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            wq[k] = 0ull;
            if (maybe[k]) wq[k] = gbr[static_cast<uint32_t>(e[k]) >> 5];
        }
        // the value of each set event: super-range base plus rank
        bool hit[kYeltSteps];
        double ov[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const uint32_t ue = static_cast<uint32_t>(e[k]);
            const uint32_t wx = static_cast<uint32_t>(wq[k]), wr = static_cast<uint32_t>(wq[k] >> 32);
            hit[k] = maybe[k] & (__builtin_amdgcn_ubfe(wx, ue, 1) != 0u);
            ov[k] = 0.0;
            if (hit[k]) ov[k] = gvals[(ue & ~static_cast<uint32_t>(kSr - 1)) + wr + __popc(__builtin_amdgcn_ubfe(wx, 0, ue))];
        }
        // the next step (the rest of this trial, or the next trial, whose
        // offsets are at hand): its IDs are fetched now, to arrive with the
        // values
        base += kStep;
        const bool last_step = base >= b;
        bool more = true;
        if (last_step) {
            t += nw;
            more = t < P.t1;
            if (more) {
                checked(na, nb, a, b);
                base = a;
            }
        }
        fetch(more ? base : 0, more ? b : 0);
        if (last_step && more && t + nw < P.t1) {
            na = goff[t + nw];
            nb = goff[t + nw + 1];
        }

        // step four on each group of kYeltGroup slices (256 occurrences):
        // lane l takes occurrences 4l .. 4l+3 of the group
#pragma unroll
        for (int g = 0; g < kYeltSteps / kYeltGroup; ++g) {
#pragma unroll
            for (int kk = 0; kk < kYeltGroup; ++kk) st[kk * kWave + lane] = hit[g * kYeltGroup + kk] ? ov[g * kYeltGroup + kk] : 0.0;
            if (g == 0) consume_ids();
            __builtin_amdgcn_wave_barrier();
            double p[kYeltGroup];
#pragma unroll
            for (int i = 0; i < kYeltGroup; ++i) p[i] = st[kYeltGroup * lane + i];
#pragma unroll
            for (int i = 1; i < kYeltGroup; ++i) p[i] = p[i - 1] + p[i];   // running total inside the lane
            const double incl = wave_inclusive_sum(p[kYeltGroup - 1]);
            const double excl = dpp_f64<0x138, 0xf>(incl);   // wave_shr:1, lane 0 reads 0
            const double bl = carry + excl;                   // total before the lane's first occurrence
            // the aggregate terms on each running total, then the increments;
            // the trial's first occurrence starts from 0, as the
            // differencing pass defines it
            double cprev = (first && lane == 0) ? 0.0 : xl(bl, aggR, aggL);
            double inc[kYeltGroup];
#pragma unroll
            for (int i = 0; i < kYeltGroup; ++i) {
                const double c = xl(bl + p[i], aggR, aggL);
                inc[i] = c - cprev;
                cprev = c;
                mx = fmax(mx, inc[i]);   // occurrences past the end add nothing: their increment is exactly 0
            }
            carry = lane63(bl + p[kYeltGroup - 1]);
            first = false;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < kYeltGroup; ++i) st[kYeltGroup * lane + i] = inc[i];
            __builtin_amdgcn_wave_barrier();
            double v[kYeltGroup];
#pragma unroll
            for (int kk = 0; kk < kYeltGroup; ++kk) v[kk] = st[kk * kWave + lane];
            static_assert(kYeltGroup == 4, "the read fence below names four values");
            asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));   // all reads before the (masked) stores
#pragma unroll
            for (int kk = 0; kk < kYeltGroup; ++kk) {
                const int k = g * kYeltGroup + kk;
                if (in[k]) __builtin_nontemporal_store(v[kk], Y + (cbase + k * kWave + lane - P.occ_begin));
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (last_step) {
            for (int sh = 32; sh > 0; sh >>= 1) mx = fmax(mx, __shfl_xor(mx, sh));
            if (lane == 0) M[ct - P.t0] = mx;
            carry = 0.0;
            mx = 0.0;
            first = true;
        }
        if (!more) break;
    }
}

int32_t launch_set_filter(const OccTables *d_tabs, int n_words, uint32_t *filter, int n_layers, hipStream_t st) {
    if (n_layers <= 0) return ARA_OK;
    k_yelt_filter<<<dim3(kFilterWords / 256, n_layers), 256, 0, st>>>(d_tabs, n_words, filter);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

static size_t yelt_workspace(const ara_tables *tables, const ara_layers *layers) {
    const OccLayoutSizes z = occ_sizes(tables->catalog, false);
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    size_t b = kWsHeaderBytes;
    b += align256(static_cast<size_t>(L + 1) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(nJ, 1)) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(L, 1)) * sizeof(OccTables));
    b += align256(static_cast<size_t>(std::max(L, 1)) * kFilterWords * sizeof(uint32_t));
    b += static_cast<size_t>(L) * z.per_layer;
    return b;
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_yelt_workspace_bytes(const ara_tables *tables, const ara_layers *layers, size_t *bytes) {
    if (!bytes || !tables) return fail(ARA_E_INVAL, "null argument");
    int32_t rc = check_layers(layers, tables->n_elts);
    if (rc) return rc;
    *bytes = yelt_workspace(tables, layers);
    return ARA_OK;
}

extern "C" int32_t ara_yelt_forward(const ara_tables *tables, const int64_t *offsets, const int32_t *ids,
                                    int64_t n_trials, const ara_layers *layers, const double *elt_terms,
                                    const double *layer_terms, int64_t trial_begin, int64_t trial_end,
                                    int64_t occ_begin, int64_t occ_count, double *yelt, double *occ_max, void *ws,
                                    size_t ws_bytes, void *stream) {
    if (!tables) return fail(ARA_E_INVAL, "null tables");
    int32_t rc = check_layers(layers, tables->n_elts);
    if (rc) return rc;
    if (trial_begin < 0 || trial_end < trial_begin || trial_end > n_trials)
        return fail(ARA_E_RANGE, "trial range outside the YET");
    if (occ_begin < 0 || occ_count < 0) return fail(ARA_E_RANGE, "negative occurrence range");
    if (!ws) return fail(ARA_E_INVAL, "null workspace");
    const int L = layers->n_layers;
    const int64_t n = trial_end - trial_begin;
    if (L > 0 && n > 0 && (!offsets || !elt_terms || !layer_terms || !occ_max || (occ_count > 0 && (!ids || !yelt))))
        return fail(ARA_E_INVAL, "null input or output");
    if (ws_bytes < yelt_workspace(tables, layers)) return fail(ARA_E_NOSPACE, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L == 0 || n == 0) {
        ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
        return ARA_OK;
    }

    const OccLayoutSizes z = occ_sizes(tables->catalog, false);
    const int nJ = layers->elt_off[L];
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / sizeof(int32_t));
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    uint32_t *d_filter = c.take<uint32_t>(static_cast<size_t>(L) * kFilterWords);
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, z, false);
    HeadImage img(ws);
    img.cover(d_err + kWsHeaderBytes / sizeof(int32_t));
    img.put(d_off, layers->elt_off, static_cast<size_t>(L + 1));
    img.put(d_ids, layers->elt_ids, static_cast<size_t>(nJ));
    img.put(d_tabs, tabs.data(), tabs.size());
    if ((rc = img.send(st))) return rc;
    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, false, false, d_tabs, z.n_sr, d_err, st)))
            return rc;
    }
    if ((rc = launch_set_filter(d_tabs, z.n_sr * kSrWords, d_filter, L, st))) return rc;
    YeltParams P{};
    P.off = offsets;
    P.ids = ids;
    P.catalog = tables->catalog;
    P.t0 = trial_begin;
    P.t1 = trial_end;
    P.occ_begin = occ_begin;
    P.occ_count = occ_count;
    P.tabs = d_tabs;
    P.filter = d_filter;
    P.lterms = layer_terms;
    P.yelt = yelt;
    P.occ_max = occ_max;
    P.err = d_err;
    // one workgroup per CU (the filter takes most of its LDS)
    const int waves_per_wg = kYeltThreads / kWave;
    const int64_t want = (n + waves_per_wg - 1) / waves_per_wg;
    const unsigned gx = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(want, device_cu_count())));
    ProfScope prof(ARA_PROF_YELT, st);
    k_yelt<<<dim3(gx, L), kYeltThreads, 0, st>>>(P);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}
