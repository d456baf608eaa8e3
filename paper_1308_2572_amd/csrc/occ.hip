// Occurrence-table kernels: evaluate the per-event steps of Algorithm 1
// (lookup, financial terms, sum over the layer's ELTs, occurrence terms) once
// per catalogue event, then store the set events compactly in rank order.
#include "occ.h"

#include <cmath>
#include <string>

namespace ara {

constexpr int kPassWords = 128;                 // 4096 events per pass
constexpr int kPasses = kSrWords / kPassWords;  // 16

__device__ __forceinline__ bool bad_scale(double s) { return !(s > 0.0) || !(s < INFINITY); }
__device__ __forceinline__ bool bad_retention(double r) { return !(r >= 0.0) || !(r < INFINITY); }
__device__ __forceinline__ bool bad_limit(double l) { return !(l > 0.0); }

// Phase one: one workgroup per (4096-event chunk, layer).  For every event,
// sum g_k over the layer's ELTs in listed order (losses of 8 ELTs are loaded
// together so their latencies overlap), apply the occurrence terms, mark the
// set events in a bitmap and keep O (and the ELT count) densely.
template <bool UNION>
__global__ __launch_bounds__(1024) void k_occ_eval(const float *__restrict__ loss, const uint32_t *__restrict__ present,
                                                   int32_t catalog, int32_t words, const int32_t *__restrict__ elt_off,
                                                   const int32_t *__restrict__ elt_ids,
                                                   const double *__restrict__ elt_terms,
                                                   const double *__restrict__ layer_terms,
                                                   const OccTables *__restrict__ tabs, int32_t *__restrict__ err) {
    __shared__ uint32_t stage[kMaxJ * kPassWords];
    __shared__ int32_t lk[kMaxJ];
    __shared__ double ls[kMaxJ], lr[kMaxJ], ll[kMaxJ];
    __shared__ double lterm[4];

    const int s = blockIdx.x / kPasses, p = blockIdx.x % kPasses, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int a = elt_off[j];
    const int J = elt_off[j + 1] - a;
    const bool checker = blockIdx.x == 0;
    for (int q = tid; q < J; q += blockDim.x) {
        const int k = elt_ids[a + q];
        lk[q] = k;
        ls[q] = elt_terms[3 * k + 0];
        lr[q] = elt_terms[3 * k + 1];
        ll[q] = elt_terms[3 * k + 2];
        if (checker && (bad_scale(ls[q]) || bad_retention(lr[q]) || bad_limit(ll[q]))) atomicCAS(err, 0, ARA_E_INVAL);
    }
    if (tid < 4) {
        lterm[tid] = layer_terms[4 * j + tid];
        const bool bad = (tid & 1) ? bad_limit(lterm[tid]) : bad_retention(lterm[tid]);
        if (checker && bad) atomicCAS(err, 0, ARA_E_INVAL);
    }
    __syncthreads();
    for (int idx = tid; idx < J * kPassWords; idx += blockDim.x) {
        const int q = idx / kPassWords, ww = idx % kPassWords;
        const int64_t gw = static_cast<int64_t>(s) * kSrWords + p * kPassWords + ww;
        stage[idx] = (gw < words) ? present[static_cast<size_t>(lk[q]) * words + gw] : 0u;
    }
    __syncthreads();
    const double occR = lterm[0], occL = lterm[1];
    const OccTables T = tabs[j];
    const int64_t ev0 = static_cast<int64_t>(s) * kSr + p * (kPassWords * 32);
    for (int it = 0; it < 4; ++it) {
        const int local = it * 1024 + tid;
        const int wip = local >> 5, bit = local & 31;
        const int64_t ev = ev0 + local;
        uint32_t any = 0;
        for (int q = 0; q < J; ++q) any |= stage[q * kPassWords + wip];
        double x = 0.0;
        int nb = 0;
        if ((any >> bit) & 1u) {
            for (int q0 = 0; q0 < J; q0 += 8) {
                float v[8];
                bool on[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + u;
                    on[u] = q < J && ((stage[q * kPassWords + wip] >> bit) & 1u);
                    // lanes without the event read element 0 (always valid) and ignore it,
                    // so the eight loads are issued back to back
                    const size_t idx = on[u] ? static_cast<size_t>(lk[q]) * catalog + ev : 0;
                    v[u] = loss[idx];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (on[u]) {
                        const int q = q0 + u;
                        const double scaled = ls[q] * static_cast<double>(v[u]);
                        x = x + xl(scaled, lr[q], ll[q]);
                        ++nb;
                    }
                }
            }
        }
        const double O = xl(x, occR, occL);
        const bool flag = UNION ? (nb > 0) : (O != 0.0);
        const uint64_t m = __ballot(flag);
        if (lane == 0) {
            const size_t wi = static_cast<size_t>(s) * kSrWords + p * kPassWords + (it * 1024 + w * 64) / 32;
            T.bits[wi] = static_cast<uint32_t>(m);
            T.bits[wi + 1] = static_cast<uint32_t>(m >> 32);
        }
        if (flag) {
            T.dense[ev] = O;
            if (UNION) T.dense_nb[ev] = static_cast<uint8_t>(nb > 255 ? 255 : nb);
        }
    }
}

// Phase two: one workgroup per (super-range, layer): rank of every set event
// (prefix count of the bitmap) and compaction of O into rank order.
template <bool UNION>
__global__ __launch_bounds__(1024) void k_occ_rank(const OccTables *__restrict__ tabs) {
    __shared__ uint32_t wsum[16];
    const int s = blockIdx.x, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const OccTables T = tabs[j];
    const uint32_t b0 = T.bits[static_cast<size_t>(s) * kSrWords + 2 * tid];
    const uint32_t b1 = T.bits[static_cast<size_t>(s) * kSrWords + 2 * tid + 1];
    const uint32_t c0 = __popc(b0), c1 = __popc(b1);
    uint32_t incl = c0 + c1;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    const uint32_t r0 = before + incl - (c0 + c1), r1 = r0 + c0;
    T.br[static_cast<size_t>(s) * kSrWords + 2 * tid] = make_uint2(b0, r0);
    T.br[static_cast<size_t>(s) * kSrWords + 2 * tid + 1] = make_uint2(b1, r1);
    if (tid == 1023) T.count[s] = static_cast<int32_t>(r1 + c1);
    double *vals = T.vals + static_cast<size_t>(s) * kSr;
    uint8_t *cnt = UNION ? T.cnt + static_cast<size_t>(s) * kSr : nullptr;
    const int64_t ev0 = static_cast<int64_t>(s) * kSr + 64 * tid;
    uint32_t rank = r0;
    for (int h = 0; h < 2; ++h) {
        uint32_t b = h ? b1 : b0;
        while (b) {
            const int bit = __ffs(b) - 1;
            b &= b - 1;
            const int64_t ev = ev0 + 32 * h + bit;
            vals[rank] = T.dense[ev];
            if (UNION) cnt[rank] = T.dense_nb[ev];
            ++rank;
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
    dim3 grid_a(static_cast<unsigned>(n_sr * kPasses), static_cast<unsigned>(n_layers));
    dim3 grid_b(static_cast<unsigned>(n_sr), static_cast<unsigned>(n_layers));
    if (union_mode) {
        k_occ_eval<true><<<grid_a, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words,
                                                  d_elt_off, d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
        k_occ_rank<true><<<grid_b, 1024, 0, st>>>(d_tabs);
    } else {
        k_occ_eval<false><<<grid_a, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words,
                                                   d_elt_off, d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
        k_occ_rank<false><<<grid_b, 1024, 0, st>>>(d_tabs);
    }
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

}  // namespace ara
