// Per-occurrence losses (the event-level YLT) and the per-year maximum
// occurrence loss: step four of Algorithm 1 taken literally, in storage
// order -- running total of the occurrence losses, aggregate retention and
// limit on each running total, then each occurrence's increment.  The sum
// of a trial's increments is its year loss; their maximum is the occurrence
// loss behind occurrence-exceedance metrics.
//
// One wavefront per trial, 64 consecutive occurrences per step with four
// steps' loads in flight: the event IDs stream from the caller's trial-major
// YET (storage order is needed here, so the bucketed layout cannot serve),
// O(e) comes from the occurrence table in global memory (bitmap word, then
// value: L2-resident), the running total is a wavefront inclusive scan with
// the previous step's total carried in.
#include "occ.h"

#include <algorithm>
#include <vector>

namespace ara {

constexpr int kYeltThreads = 256;
constexpr int kYeltSteps = 4;

struct YeltParams {
    const int64_t *off;
    const int32_t *ids;
    int32_t catalog;
    int32_t pad;
    int64_t t0, t1;
    int64_t occ_begin, occ_count;
    const OccTables *tabs;
    const double *lterms;
    double *yelt;       // [n_layers][occ_count]
    double *occ_max;    // [n_layers][t1 - t0]
    int32_t *err;
};

__global__ __launch_bounds__(kYeltThreads) void k_yelt(YeltParams P) {
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    const int64_t gw = static_cast<int64_t>(blockIdx.x) * (kYeltThreads / kWave) + (threadIdx.x >> 6);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (kYeltThreads / kWave);
    const OccTables T = P.tabs[j];
    const double aggR = P.lterms[4 * j + 2], aggL = P.lterms[4 * j + 3];
    double *Y = P.yelt + static_cast<size_t>(j) * P.occ_count;
    double *M = P.occ_max + static_cast<size_t>(j) * (P.t1 - P.t0);
    for (int64_t t = P.t0 + gw; t < P.t1; t += nw) {
        const int64_t a = P.off[t], b = P.off[t + 1];
        if (a < P.occ_begin || b > P.occ_begin + P.occ_count || b < a) {
            if (lane == 0) atomicCAS(P.err, 0, ARA_E_RANGE);
            continue;
        }
        double carry = 0.0, cprev = 0.0, mx = 0.0;
        for (int64_t base = a; base < b; base += kWave * kYeltSteps) {
            int32_t e[kYeltSteps];
            bool in[kYeltSteps];
#pragma unroll
            for (int k = 0; k < kYeltSteps; ++k) {
                const int64_t i = base + k * kWave + lane;
                in[k] = i < b;
                e[k] = in[k] ? P.ids[i] : 0;
                if (in[k] && (e[k] < 0 || e[k] >= P.catalog)) {
                    atomicCAS(P.err, 0, ARA_E_RANGE);
                    e[k] = 0;
                    in[k] = false;
                }
            }
            uint2 q[kYeltSteps];
#pragma unroll
            for (int k = 0; k < kYeltSteps; ++k)
                q[k] = T.br[static_cast<size_t>(e[k] >> kSrBits) * kSrWords + ((e[k] & (kSr - 1)) >> 5)];
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
                double x = o[k];
                for (int s = 1; s < kWave; s <<= 1) {
                    const double v = __shfl_up(x, s);
                    if (lane >= s) x += v;
                }
                const double run = carry + x;                 // running total after this occurrence
                const double c = xl(run, aggR, aggL);
                double cl = __shfl_up(c, 1);
                if (lane == 0) cl = cprev;
                const double inc = c - cl;
                const int64_t i = base + k * kWave + lane;
                if (in[k]) {
                    Y[i - P.occ_begin] = inc;
                    mx = fmax(mx, inc);
                }
                carry = __shfl(run, kWave - 1);   // lanes past the end add 0
                cprev = __shfl(c, kWave - 1);
            }
        }
        for (int s = 32; s > 0; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s));
        if (lane == 0) M[t - P.t0] = mx;
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
    ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
    if (L == 0 || n == 0) return ARA_OK;

    const OccLayoutSizes z = occ_sizes(tables->catalog, false);
    const int nJ = layers->elt_off[L];
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / sizeof(int32_t));
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, z, false);
    ARA_HIP(hipMemcpyAsync(d_off, layers->elt_off, (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (nJ > 0) ARA_HIP(hipMemcpyAsync(d_ids, layers->elt_ids, nJ * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(d_tabs, tabs.data(), L * sizeof(OccTables), hipMemcpyHostToDevice, st));
    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, false, d_tabs, z.n_sr, d_err, st)))
            return rc;
    }
    YeltParams P{};
    P.off = offsets;
    P.ids = ids;
    P.catalog = tables->catalog;
    P.t0 = trial_begin;
    P.t1 = trial_end;
    P.occ_begin = occ_begin;
    P.occ_count = occ_count;
    P.tabs = d_tabs;
    P.lterms = layer_terms;
    P.yelt = yelt;
    P.occ_max = occ_max;
    P.err = d_err;
    const int waves_per_wg = kYeltThreads / kWave;
    const int64_t want = (n + waves_per_wg - 1) / waves_per_wg;
    const unsigned gx = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(want, 8 * device_cu_count())));
    ProfScope prof(ARA_PROF_YELT, st);
    k_yelt<<<dim3(gx, L), kYeltThreads, 0, st>>>(P);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}
