// Occurrence-table kernel: per (super-range, layer) workgroup, evaluate the
// per-event steps of Algorithm 1 (lookup, financial terms, sum over the
// layer's ELTs, occurrence terms) and store the non-zero results compactly.
#include "occ.h"

#include <cmath>
#include <string>

namespace ara {

constexpr int kPassWords = 128;                 // 4096 events per pass
constexpr int kPasses = kSrWords / kPassWords;  // 16

__device__ __forceinline__ bool bad_scale(double s) { return !(s > 0.0) || !(s < INFINITY); }
__device__ __forceinline__ bool bad_retention(double r) { return !(r >= 0.0) || !(r < INFINITY); }
__device__ __forceinline__ bool bad_limit(double l) { return !(l > 0.0); }

template <bool UNION>
__global__ __launch_bounds__(1024) void k_occ(const float *__restrict__ loss, const uint32_t *__restrict__ present,
                                              int32_t catalog, int32_t words, const int32_t *__restrict__ elt_off,
                                              const int32_t *__restrict__ elt_ids, const double *__restrict__ elt_terms,
                                              const double *__restrict__ layer_terms, const OccTables *__restrict__ tabs,
                                              int32_t *__restrict__ err) {
    __shared__ uint32_t stage[kMaxJ * kPassWords];
    __shared__ uint32_t wbits[kSrWords];
    __shared__ uint32_t wrank[kSrWords];
    __shared__ int32_t lk[kMaxJ];
    __shared__ double ls[kMaxJ], lr[kMaxJ], ll[kMaxJ];
    __shared__ double lterm[4];
    __shared__ uint32_t wsum[16];

    const int s = blockIdx.x, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int a = elt_off[j];
    const int J = elt_off[j + 1] - a;
    for (int q = tid; q < J; q += blockDim.x) {
        const int k = elt_ids[a + q];
        lk[q] = k;
        ls[q] = elt_terms[3 * k + 0];
        lr[q] = elt_terms[3 * k + 1];
        ll[q] = elt_terms[3 * k + 2];
        if (s == 0 && (bad_scale(ls[q]) || bad_retention(lr[q]) || bad_limit(ll[q]))) atomicCAS(err, 0, ARA_E_INVAL);
    }
    if (tid < 4) {
        lterm[tid] = layer_terms[4 * j + tid];
        const bool bad = (tid & 1) ? bad_limit(lterm[tid]) : bad_retention(lterm[tid]);
        if (s == 0 && bad) atomicCAS(err, 0, ARA_E_INVAL);
    }
    __syncthreads();
    const double occR = lterm[0], occL = lterm[1];
    const OccTables T = tabs[j];
    const int64_t ev_base = static_cast<int64_t>(s) * kSr;

    // evaluate event `local` (0..4095) of pass p; returns O and the ELT count
    auto eval = [&](int p, int local, double &O, int &nb) {
        const int wip = local >> 5, bit = local & 31;
        const int64_t ev = ev_base + p * (kPassWords * 32) + local;
        double x = 0.0;
        nb = 0;
        for (int q = 0; q < J; ++q) {
            if ((stage[q * kPassWords + wip] >> bit) & 1u) {
                const double l = static_cast<double>(loss[static_cast<size_t>(lk[q]) * catalog + ev]);
                const double scaled = ls[q] * l;
                x = x + xl(scaled, lr[q], ll[q]);
                ++nb;
            }
        }
        O = xl(x, occR, occL);
    };
    auto stage_pass = [&](int p) {
        for (int idx = tid; idx < J * kPassWords; idx += blockDim.x) {
            const int q = idx / kPassWords, ww = idx % kPassWords;
            const int64_t gw = static_cast<int64_t>(s) * kSrWords + p * kPassWords + ww;
            stage[idx] = (gw < words) ? present[static_cast<size_t>(lk[q]) * words + gw] : 0u;
        }
    };

    // phase A: which events are set
    for (int p = 0; p < kPasses; ++p) {
        stage_pass(p);
        __syncthreads();
        for (int it = 0; it < 4; ++it) {
            const int local = it * 1024 + tid;
            double O;
            int nb;
            eval(p, local, O, nb);
            const bool flag = UNION ? (nb > 0) : (O != 0.0);
            const uint64_t m = __ballot(flag);
            if (lane == 0) {
                const int wi = p * kPassWords + (it * 1024 + w * 64) / 32;
                wbits[wi] = static_cast<uint32_t>(m);
                wbits[wi + 1] = static_cast<uint32_t>(m >> 32);
            }
        }
        __syncthreads();
    }

    // exclusive prefix of the per-word counts
    const uint32_t c0 = __popc(wbits[2 * tid]), c1 = __popc(wbits[2 * tid + 1]);
    uint32_t incl = c0 + c1;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    const uint32_t excl = before + incl - (c0 + c1);
    wrank[2 * tid] = excl;
    wrank[2 * tid + 1] = excl + c0;
    if (tid == 1023) T.count[s] = static_cast<int32_t>(excl + c0 + c1);
    __syncthreads();
    for (int i = tid; i < kSrWords; i += blockDim.x) T.br[static_cast<size_t>(s) * kSrWords + i] = make_uint2(wbits[i], wrank[i]);

    // phase B: store the values of the set events in rank order
    double *vals = T.vals + static_cast<size_t>(s) * kSr;
    uint8_t *cnt = UNION ? T.cnt + static_cast<size_t>(s) * kSr : nullptr;
    for (int p = 0; p < kPasses; ++p) {
        __syncthreads();
        stage_pass(p);
        __syncthreads();
        for (int it = 0; it < 4; ++it) {
            const int local = it * 1024 + tid;
            const int wi = p * kPassWords + (local >> 5), bit = local & 31;
            const uint32_t wb = wbits[wi];
            if ((wb >> bit) & 1u) {
                double O;
                int nb;
                eval(p, local, O, nb);
                const uint32_t rank = wrank[wi] + __popc(wb & ((1u << bit) - 1u));
                vals[rank] = O;
                if (UNION) cnt[rank] = static_cast<uint8_t>(nb > 255 ? 255 : nb);
            }
        }
    }
}

int32_t check_layers(const ara_layers *layers, int32_t n_elts) {
    if (!layers) return fail(ARA_E_INVAL, "null layers");
    if (layers->n_layers < 0) return fail(ARA_E_INVAL, "negative layer count");
    if (layers->n_layers == 0) return ARA_OK;
    if (!layers->elt_off || !layers->elt_ids) return fail(ARA_E_INVAL, "null layer arrays");
    if (layers->elt_off[0] != 0) return fail(ARA_E_RANGE, "elt_off[0] must be 0");
    for (int32_t j = 0; j < layers->n_layers; ++j) {
        const int32_t J = layers->elt_off[j + 1] - layers->elt_off[j];
        if (J < 0) return fail(ARA_E_RANGE, "elt_off must be non-decreasing");
        if (J > kMaxJ) return fail(ARA_E_LIMIT, "layer covers more than ARA_MAX_ELTS_PER_LAYER ELTs");
        for (int32_t q = layers->elt_off[j]; q < layers->elt_off[j + 1]; ++q)
            if (layers->elt_ids[q] < 0 || layers->elt_ids[q] >= n_elts)
                return fail(ARA_E_RANGE, "layer refers to an ELT index out of range");
    }
    return ARA_OK;
}

int32_t launch_occ(const ara_tables *tables, const int32_t *d_elt_off, const int32_t *d_elt_ids,
                   const double *elt_terms, const double *layer_terms, int32_t n_layers, bool union_mode,
                   OccTables *d_tabs, int n_sr, int32_t *d_err, hipStream_t st) {
    if (n_layers == 0 || n_sr == 0) return ARA_OK;
    dim3 grid(static_cast<unsigned>(n_sr), static_cast<unsigned>(n_layers));
    if (union_mode)
        k_occ<true><<<grid, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words, d_elt_off,
                                           d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
    else
        k_occ<false><<<grid, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words, d_elt_off,
                                            d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

}  // namespace ara
