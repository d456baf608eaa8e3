// Occurrence-table kernels: evaluate the per-event steps of Algorithm 1
// (lookup, financial terms, sum over the layer's ELTs, occurrence terms) once
// per catalogue event, then store the set events compactly in rank order.
#include "occ.h"

#include <cmath>
#include <string>

namespace ara {

constexpr int kPassWords = kOccChunkWords;      // 4096 events per chunk
constexpr int kPasses = kOccChunks;             // 16 chunks per super-range
constexpr int kLossBatch = 16;                  // ELT losses of one event loaded together

__device__ __forceinline__ bool bad_scale(double s) { return !(s > 0.0) || !(s < INFINITY); }
__device__ __forceinline__ bool bad_retention(double r) { return !(r >= 0.0) || !(r < INFINITY); }
__device__ __forceinline__ bool bad_limit(double l) { return !(l > 0.0); }

// Exclusive prefix sum of v over the first 128 threads (two wavefronts);
// *total receives the sum.  Every thread of the block must call it.
__device__ __forceinline__ uint32_t scan128(uint32_t v, uint32_t *wtot, uint32_t *total) {
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t incl = v;
    if (tid < 128) {
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(incl, o);
            if (lane >= o) incl += x;
        }
        if (lane == 63) wtot[tid >> 6] = incl;
    }
    __syncthreads();
    const uint32_t before = (tid >= 64 && tid < 128) ? wtot[0] : 0u;
    if (tid == 0) *total = wtot[0] + wtot[1];
    __syncthreads();
    return before + incl - v;
}

// Phase one: one workgroup per (4096-event chunk, layer).  The events held
// by at least one of the layer's ELTs are listed in event order; each is
// evaluated once: g_k summed over the layer's ELTs in listed order (losses of
// up to 16 ELTs are loaded together so their latencies overlap), then the occurrence
// terms.  The set events are compacted in event order: the chunk's bitmap
// words, its count, and O (and the ELT count) at the start of the chunk's
// slice of the staging arrays.
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
    __shared__ uint32_t anyw[kPassWords], cbase[kPassWords], fbits[kPassWords];
    __shared__ uint16_t cand[kPassWords * 32];
    __shared__ uint32_t wtot[16], wtot2[2], n_cand;

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
    for (int idx = tid; idx < J * kPassWords; idx += blockDim.x) {
        const int q = idx / kPassWords, ww = idx % kPassWords;
        const int64_t gw = static_cast<int64_t>(s) * kSrWords + p * kPassWords + ww;
        stage[idx] = (gw < words) ? present[static_cast<size_t>(elt_ids[a + q]) * words + gw] : 0u;
    }
    __syncthreads();
    // events held by any of the layer's ELTs, word by word, and where each
    // word's events start in the candidate list
    uint32_t any = 0;
    if (tid < kPassWords) {
        for (int q = 0; q < J; ++q) any |= stage[q * kPassWords + tid];
        anyw[tid] = any;
        fbits[tid] = 0u;
    }
    const uint32_t cb = scan128(__popc(any), wtot2, &n_cand);
    if (tid < kPassWords) cbase[tid] = cb;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int local = it * 1024 + tid;
        const uint32_t m = anyw[local >> 5];
        const uint32_t bit = static_cast<uint32_t>(local & 31);
        if ((m >> bit) & 1u) cand[cbase[local >> 5] + __popc(m & ((1u << bit) - 1u))] = static_cast<uint16_t>(local);
    }
    __syncthreads();
    const int nc = static_cast<int>(n_cand);
    const double occR = lterm[0], occL = lterm[1];
    const OccTables T = tabs[j];
    const int64_t ev0 = static_cast<int64_t>(s) * kSr + p * (kPassWords * 32);
    double *ov = T.dense + ev0;                           // the chunk's compacted O
    uint8_t *onb = UNION ? T.dense_nb + ev0 : nullptr;    // and ELT counts
    uint32_t run = 0;                                     // set events before this pass
    for (int i0 = 0; i0 < nc; i0 += 1024) {   // uniform trip count: every thread reaches the barriers
        const int i = i0 + tid;
        const int local = i < nc ? cand[i] : 0;
        const int wip = local >> 5, bit = local & 31;
        const int64_t ev = ev0 + local;
        double x = 0.0;
        int nb = 0;
        if (i < nc) {
            for (int q0 = 0; q0 < J; q0 += kLossBatch) {
                float v[kLossBatch];
                bool on[kLossBatch];
#pragma unroll
                for (int u = 0; u < kLossBatch; ++u) {
                    const int q = q0 + u;
                    on[u] = q < J && ((stage[q * kPassWords + wip] >> bit) & 1u);
                    // lanes without the event read element 0 (always valid) and ignore it,
                    // so the eight loads are issued back to back
                    const size_t idx = on[u] ? static_cast<size_t>(lk[q]) * catalog + ev : 0;
                    v[u] = loss[idx];
                }
#pragma unroll
                for (int u = 0; u < kLossBatch; ++u) {
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
        const bool flag = i < nc && (UNION ? (nb > 0) : (O != 0.0));
        // rank among this pass's set events: lanes below, then wavefronts below
        const uint64_t m = __ballot(flag);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
        if (lane == 0) wtot[w] = static_cast<uint32_t>(__popcll(m));
        __syncthreads();
        uint32_t wb = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            const uint32_t c = wtot[k];
            wb += (k < w) ? c : 0u;
            tot += c;
        }
        if (flag) {
            const uint32_t r = run + wb + below;
            ov[r] = O;
            if (UNION) onb[r] = static_cast<uint8_t>(nb > 255 ? 255 : nb);
            atomicOr(&fbits[wip], 1u << bit);
        }
        run += tot;
        __syncthreads();   // wtot is rewritten by the next pass
    }
    if (tid < kPassWords) T.bits[static_cast<size_t>(s) * kSrWords + p * kPassWords + tid] = fbits[tid];
    if (tid == 0) T.pcount[static_cast<size_t>(s) * kPasses + p] = static_cast<int32_t>(run);
}

// Phase two: one workgroup per (chunk, layer): the chunk's rank base (set
// events of the super-range's earlier chunks), the rank of every bitmap word,
// and the chunk's compacted values moved to their place in rank order.
template <bool UNION, bool F32>
__global__ __launch_bounds__(1024) void k_occ_rank(const OccTables *__restrict__ tabs) {
    __shared__ uint32_t wtot2[2], tot;
    const int s = blockIdx.x / kPasses, p = blockIdx.x % kPasses, j = blockIdx.y;
    const int tid = threadIdx.x;
    const OccTables T = tabs[j];
    const int32_t *pc = T.pcount + static_cast<size_t>(s) * kPasses;
    uint32_t base = 0;
    for (int k = 0; k < p; ++k) base += static_cast<uint32_t>(pc[k]);
    const uint32_t cnt = static_cast<uint32_t>(pc[p]);
    const size_t w0 = static_cast<size_t>(s) * kSrWords + p * kPassWords;
    const uint32_t b = tid < kPassWords ? T.bits[w0 + tid] : 0u;
    const uint32_t r = scan128(__popc(b), wtot2, &tot);
    if (tid < kPassWords) T.br[w0 + tid] = make_uint2(b, base + r);
    if (p == kPasses - 1 && tid == 0) T.count[s] = static_cast<int32_t>(base + cnt);
    const size_t src = static_cast<size_t>(s) * kSr + static_cast<size_t>(p) * (kPassWords * 32);
    const size_t dst = static_cast<size_t>(s) * kSr + base;
    for (uint32_t i = tid; i < cnt; i += blockDim.x) {
        if (F32) reinterpret_cast<float *>(T.vals)[dst + i] = static_cast<float>(T.dense[src + i]);
        else T.vals[dst + i] = T.dense[src + i];
        if (UNION) T.cnt[dst + i] = T.dense_nb[src + i];
    }
}

int32_t check_layers(const ara_layers *layers, int32_t n_elts) {
    if (!layers) return fail(ARA_E_INVAL, "null layers");
    if (layers->n_layers < 0) return fail(ARA_E_INVAL, "negative layer count");
    if (layers->n_layers > ARA_MAX_LAYERS) return fail(ARA_E_LIMIT, "more than ARA_MAX_LAYERS layers in one call");
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
                   bool f32_vals, OccTables *d_tabs, int n_sr, int32_t *d_err, hipStream_t st) {
    if (n_layers == 0 || n_sr == 0) return ARA_OK;
    dim3 grid_a(static_cast<unsigned>(n_sr * kPasses), static_cast<unsigned>(n_layers));
    dim3 grid_b(static_cast<unsigned>(n_sr * kPasses), static_cast<unsigned>(n_layers));
    if (union_mode) {
        k_occ_eval<true><<<grid_a, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words,
                                                  d_elt_off, d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
        if (f32_vals) k_occ_rank<true, true><<<grid_b, 1024, 0, st>>>(d_tabs);
        else k_occ_rank<true, false><<<grid_b, 1024, 0, st>>>(d_tabs);
    } else {
        k_occ_eval<false><<<grid_a, 1024, 0, st>>>(tables->loss, tables->present, tables->catalog, tables->words,
                                                   d_elt_off, d_elt_ids, elt_terms, layer_terms, d_tabs, d_err);
        if (f32_vals) k_occ_rank<false, true><<<grid_b, 1024, 0, st>>>(d_tabs);
        else k_occ_rank<false, false><<<grid_b, 1024, 0, st>>>(d_tabs);
    }
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

}  // namespace ara
