// Per-occurrence losses (the event-level YLT) and the per-year maximum
// occurrence loss: step four of Algorithm 1 taken literally, in storage
// order -- running total of the occurrence losses, aggregate retention and
// limit on each running total, then each occurrence's increment.  The sum
// of a trial's increments is its year loss; their maximum is the occurrence
// loss behind occurrence-exceedance metrics.
//
// One wavefront per trial, 256 consecutive occurrences per step: the event
// IDs stream from the caller's trial-major YET (storage order is needed
// here, so the bucketed layout cannot serve).  A lookup per occurrence in
// the cache would be bound by its request rate, so each workgroup first
// loads a 1-Mbit filter of the layer's set events into LDS (the set-event
// bitmap folded onto 2^20 bits by OR); only occurrences whose filter bit is
// set (the set events plus a few that share a bit) read the bitmap word
// with its rank and then the value from the cache-resident occurrence table.
// The running total is a wavefront inclusive scan (DPP, no LDS traffic) with
// the previous step's total carried in.
#include "occ.h"

#include <algorithm>
#include <vector>

namespace ara {

constexpr int kYeltThreads = 1024;
constexpr int kYeltSteps = 8;
constexpr int kFilterWords = 1 << 15;   // 2^20 bits = 128 KB of LDS

// Cross-lane moves of a binary64 value by DPP (no LDS traffic): CTRL is the
// DPP control, lanes whose source is outside the pattern (or whose row is
// masked off) read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) |
                                                       static_cast<uint32_t>(lo)));
}

// Inclusive prefix sum over the 64 lanes: shifts of 1, 2, 4, 8 inside each
// row of 16 lanes, then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then the first two rows' total into rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ double wave_inclusive_sum(double x) {
    x += dpp_f64<0x111, 0xf>(x);   // row_shr:1
    x += dpp_f64<0x112, 0xf>(x);   // row_shr:2
    x += dpp_f64<0x114, 0xf>(x);   // row_shr:4
    x += dpp_f64<0x118, 0xf>(x);   // row_shr:8
    x += dpp_f64<0x142, 0xa>(x);   // row_bcast:15
    x += dpp_f64<0x143, 0xc>(x);   // row_bcast:31
    return x;
}

__device__ __forceinline__ double lane63(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(b), 63);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(b >> 32), 63);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

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

__global__ __launch_bounds__(kYeltThreads) void k_yelt(YeltParams P) {
    __shared__ uint32_t filt[kFilterWords];
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kFilterWords; i += blockDim.x)
        filt[i] = P.filter[static_cast<size_t>(j) * kFilterWords + i];
    __syncthreads();
    const int64_t gw = static_cast<int64_t>(blockIdx.x) * (kYeltThreads / kWave) + (threadIdx.x >> 6);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (kYeltThreads / kWave);
    const OccTables T = P.tabs[j];
    const double aggR = P.lterms[4 * j + 2], aggL = P.lterms[4 * j + 3];
    double *Y = P.yelt + static_cast<size_t>(j) * P.occ_count;
    double *M = P.occ_max + static_cast<size_t>(j) * (P.t1 - P.t0);
    constexpr int kStep = kWave * kYeltSteps;

    // cursor: trial t, its occurrence range [a, b) (empty if invalid), step start
    int64_t t = P.t0 + gw, a = 0, b = 0, base = 0;
    auto open_trial = [&]() {
        a = P.off[t];
        b = P.off[t + 1];
        if (a < P.occ_begin || b > P.occ_begin + P.occ_count || b < a) {
            if (lane == 0) atomicCAS(P.err, 0, ARA_E_RANGE);
            b = a;   // nothing of this trial is read or written
        }
        base = a;
    };
    int32_t en[kYeltSteps];
    auto fetch = [&]() {   // IDs of the step at (t, base)
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const int64_t i = base + k * kWave + lane;
            en[k] = (i < b) ? __builtin_nontemporal_load(P.ids + i) : 0;
        }
    };
    if (t >= P.t1) return;
    open_trial();
    fetch();
    double carry = 0.0, cprev = 0.0, mx = 0.0;
    while (true) {
        const int64_t ct = t, cbase = base, cb = b;
        int32_t e[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) e[k] = en[k];
        // advance the cursor and prefetch the next step's IDs
        base += kStep;
        const bool last_step = base >= b;
        bool more = true;
        if (last_step) {
            t += nw;
            more = t < P.t1;
            if (more) open_trial();
        }
        if (more) fetch();

        bool in[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            in[k] = cbase + k * kWave + lane < cb;
            if (in[k] && (e[k] < 0 || e[k] >= P.catalog)) {
                atomicCAS(P.err, 0, ARA_E_RANGE);
                in[k] = false;
            }
            if (!in[k]) e[k] = 0;
        }
        uint2 q[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const bool maybe = in[k] && ((filt[(e[k] >> 5) & (kFilterWords - 1)] >> (e[k] & 31)) & 1u);
            q[k] = maybe ? T.br[static_cast<size_t>(e[k] >> kSrBits) * kSrWords + ((e[k] & (kSr - 1)) >> 5)]
                         : make_uint2(0u, 0u);
        }
        double o[kYeltSteps];
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const uint32_t bit = e[k] & 31;
            const bool hit = in[k] && ((q[k].x >> bit) & 1u);
            const uint32_t rank = q[k].y + __popc(q[k].x & ((1u << bit) - 1u));
            o[k] = hit ? T.vals[static_cast<size_t>(e[k] >> kSrBits) * kSr + rank] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kYeltSteps; ++k) {
            const double x = wave_inclusive_sum(o[k]);
            const double run = carry + x;                 // running total after this occurrence
            const double c = xl(run, aggR, aggL);
            double cl = dpp_f64<0x138, 0xf>(c);           // wave_shr:1, the previous lane's value
            if (lane == 0) cl = cprev;
            const double inc = c - cl;
            if (in[k]) {
                __builtin_nontemporal_store(inc, Y + (cbase + k * kWave + lane - P.occ_begin));
                mx = fmax(mx, inc);
            }
            carry = lane63(run);   // lanes past the end add 0
            cprev = lane63(c);
        }
        if (last_step) {
            for (int sh = 32; sh > 0; sh >>= 1) mx = fmax(mx, __shfl_xor(mx, sh));
            if (lane == 0) M[ct - P.t0] = mx;
            carry = 0.0;
            cprev = 0.0;
            mx = 0.0;
        }
        if (!more) break;
    }
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
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, false, d_tabs, z.n_sr, d_err, st)))
            return rc;
    }
    k_yelt_filter<<<dim3(kFilterWords / 256, L), 256, 0, st>>>(d_tabs, z.n_sr * kSrWords, d_filter);
    ARA_HIP(hipGetLastError());
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
