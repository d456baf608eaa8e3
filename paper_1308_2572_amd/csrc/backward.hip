// Backward: gradients of sum_t c_t * Y_t with respect to every ELT term
// (scale, retention, limit) and every layer term (OccR, OccL, AggR, AggL),
// for up to ARA_MAX_COTANGENTS cotangent rows c at once -- the reverse sweep
// of Algorithm 1.
//
// Chain rule through the forward (branch-following subgradients):
//   Y_t = f_agg(S_t),  S_t = sum over occurrences d of O(e_d),
//   O(e) = f_occ(x_e),  x_e = sum over the layer's ELTs k of g_k(l_k(e)).
//   dY_t/dS_t = a_t (aggregate clamp in its linear branch), so with
//   v_t = c_t * a_t and W(e) = sum_t v_t * (occurrences of e in trial t):
//     dAggR = -sum_t c_t a_t,  dAggL = sum_t c_t [aggregate limit binds]
//     dOccR = -sum_e W(e) b_e, dOccL = sum_e W(e) [occurrence limit binds]
//     ds_k  =  sum_e W(e) b_e lin_k(e) l_k(e)
//     dR_k  = -sum_e W(e) b_e lin_k(e),  dL_k = sum_e W(e) b_e [ELT limit binds]
//   (b_e: occurrence clamp linear; lin_k: ELT clamp linear).  Only events
//   with O(e) != 0 can have b_e or a binding occurrence limit, so W is kept
//   for those "hot" events only, indexed by the occurrence table's rank.
//
// Kernels: (1) the hot occurrence tables (shared with the forward);
// (2) v_t per cotangent row, its largest magnitude and the aggregate-term
// sums; (3) v_t in 64-bit fixed point, scaled so that no partial sum of W
// can overflow (|W| <= max|v| * largest occurrence count of one event);
// (4) a stream over the prepared YET, one workgroup per (catalogue range,
// part of the blocks), adding fixed-point v into LDS accumulators of W --
// integer addition, so the result does not depend on the order;
// (5) per 4096-event chunk, W times the per-event derivatives, reduced in a
// fixed order; (6) a fixed-order sum of the chunk partials into the outputs.
#include "occ.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace ara {

constexpr int kBwdThreads = 1024;
constexpr int kMaxCot = ARA_MAX_COTANGENTS;
constexpr int kChunkWords = 128;                  // 4096 events per reduction workgroup
constexpr int kChunks = kSrWords / kChunkWords;   // 16 per super-range
constexpr int kLds = 160 * 1024;

struct VScale {
    unsigned long long maxabs_bits;   // max |v| as binary64 bits (non-negative: order-preserving)
    int32_t sigma;                    // v is stored as round(v * 2^sigma)
    int32_t pad;
};

__device__ __forceinline__ bool agg_linear(double S, double aggR, double aggL) {
    const double y = S - aggR;
    const double a = (y > 0.0) ? y : 0.0;
    return (y > 0.0) && (a < aggL);
}

__device__ __forceinline__ bool agg_capped(double S, double aggR, double aggL) {
    const double y = S - aggR;
    const double a = (y > 0.0) ? y : 0.0;
    return a >= aggL;
}

__device__ double bsum(double v, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (tid == 0)
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void chunk_range(int64_t n, int nwg, int wg, int64_t &lo, int64_t &hi) {
    const int64_t c = (n + nwg - 1) / nwg;
    lo = std::min<int64_t>(n, static_cast<int64_t>(wg) * c);
    hi = std::min<int64_t>(n, lo + c);
}

// (2) largest |c_t a_t| per (layer, row); aggregate-term partial sums.
__global__ __launch_bounds__(kBwdThreads) void k_bwd_vmax(const double *__restrict__ cot, const double *__restrict__ s_pre,
                                                         const double *__restrict__ layer_terms, int64_t n, int n_layers,
                                                         int n_cot, int nwg, VScale *__restrict__ vs,
                                                         double *__restrict__ aggpart) {
    __shared__ double red[16];
    const int wg = blockIdx.x, j = blockIdx.y;
    const double aggR = layer_terms[4 * j + 2], aggL = layer_terms[4 * j + 3];
    int64_t lo, hi;
    chunk_range(n, nwg, wg, lo, hi);
    const double *S = s_pre + static_cast<size_t>(j) * n;
    for (int c = 0; c < n_cot; ++c) {
        const double *g = cot + (static_cast<size_t>(c) * n_layers + j) * n;
        double m = 0.0, sr = 0.0, sl = 0.0;
        for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
            const double w = g[t], st = S[t];
            const bool lin = agg_linear(st, aggR, aggL);
            if (lin) {
                sr += w;
                m = fmax(m, fabs(w));
            }
            if (agg_capped(st, aggR, aggL)) sl += w;
        }
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
        if ((threadIdx.x & 63) == 0 && m > 0.0)
            atomicMax(&vs[j * n_cot + c].maxabs_bits, static_cast<unsigned long long>(__double_as_longlong(m)));
        const double tr = bsum(sr, red);
        const double tl = bsum(sl, red);
        if (threadIdx.x == 0) {
            double *ap = aggpart + ((static_cast<size_t>(j) * n_cot + c) * nwg + wg) * 2;
            ap[0] = -tr;
            ap[1] = tl;
        }
    }
}

__device__ __forceinline__ int sigma_of(const VScale &v, int max_occ) {
    const double m = __longlong_as_double(static_cast<long long>(v.maxabs_bits));
    if (!(m > 0.0)) return 0;
    int e;
    frexp(m * static_cast<double>(max_occ > 0 ? max_occ : 1), &e);   // m*max_occ < 2^e
    return 62 - e;
}

// (3) fixed-point weights vq[c][j][t] = round(c_t a_t 2^sigma).
__global__ void k_bwd_vq(const double *__restrict__ cot, const double *__restrict__ s_pre,
                         const double *__restrict__ layer_terms, int64_t n, int n_layers, int n_cot, int max_occ,
                         VScale *__restrict__ vs, int64_t *__restrict__ vq) {
    const int j = blockIdx.y;
    const double aggR = layer_terms[4 * j + 2], aggL = layer_terms[4 * j + 3];
    const double *S = s_pre + static_cast<size_t>(j) * n;
    for (int c = 0; c < n_cot; ++c) {
        const int sg = sigma_of(vs[j * n_cot + c], max_occ);
        if (blockIdx.x == 0 && threadIdx.x == 0) vs[j * n_cot + c].sigma = sg;
        const double *g = cot + (static_cast<size_t>(c) * n_layers + j) * n;
        int64_t *q = vq + (static_cast<size_t>(c) * n_layers + j) * n;
        for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n;
             t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
            const double v = agg_linear(S[t], aggR, aggL) ? g[t] : 0.0;
            q[t] = (v == 0.0) ? 0 : static_cast<int64_t>(__double2ll_rn(ldexp(v, sg)));
        }
    }
}

struct BwdStream {
    const uint32_t *ent;
    const int64_t *seg_base;
    const int32_t *seg_run;
    int64_t t0, t1, n;
    int32_t tg, tb, n_ranges, n_parts, n_cot, n_layers;
    int32_t b_lo, b_hi;
    int32_t capw;                 // W accumulators per row held in LDS
    const OccTables *tabs;        // hot tables per layer
    const int64_t *vq;            // [n_cot][n_layers][n]
    int64_t *wg;                  // [n_layers][n_cot][n_parts][n_sr * kSr]
    size_t wg_stride;             // n_sr * kSr
};

// (4) W(e) += v_t for every occurrence (t, e) of a hot event.  The blocks of
// one part are processed in phases of half a block (8 trial groups): the
// weights of the next phase are loaded into registers while the current one
// streams, and each wavefront prefetches the first entries of its next
// segment before the phase barrier.
constexpr int kBwdUnroll = 16;
constexpr int kVqRegs = 8;   // n_cot * 8 * tg / 1024 <= 4 * 2048 / 1024

__global__ __launch_bounds__(kBwdThreads) void k_bwd_stream(BwdStream P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int half_trials = 8 * P.tg;
    uint2 *tbr = reinterpret_cast<uint2 *>(smem);                                       // [1024]
    int64_t *vql = reinterpret_cast<int64_t *>(smem + 1024 * sizeof(uint2));           // [n_cot][half_trials]
    unsigned long long *wl = reinterpret_cast<unsigned long long *>(
        smem + 1024 * sizeof(uint2) + static_cast<size_t>(P.n_cot) * half_trials * sizeof(int64_t));   // [n_cot][capw]

    const int r = blockIdx.x / P.n_parts, part = blockIdx.x % P.n_parts, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = r >> 1, hf = r & 1;
    const OccTables T = P.tabs[j];
    const uint2 *gbr = T.br + static_cast<size_t>(s) * kSrWords + hf * 1024;
    const uint32_t base = gbr[0].y;
    const uint32_t end = hf ? static_cast<uint32_t>(T.count[s]) : T.br[static_cast<size_t>(s) * kSrWords + 1024].y;
    const uint32_t hot = end - base;
    for (int i = tid; i < 1024; i += blockDim.x) {
        const uint2 q = gbr[i];
        tbr[i] = make_uint2(q.x, q.y - base);
    }
    const uint32_t inl = min(hot, static_cast<uint32_t>(P.capw));
    for (int c = 0; c < P.n_cot; ++c)
        for (uint32_t i = tid; i < inl; i += blockDim.x) wl[c * P.capw + i] = 0ull;
    int64_t *wgp = P.wg + (static_cast<size_t>(j) * P.n_cot * P.n_parts + part) * P.wg_stride +
                   static_cast<size_t>(s) * kSr + base;
    const size_t cstride = static_cast<size_t>(P.n_parts) * P.wg_stride;
    for (int c = 0; c < P.n_cot; ++c)
        for (uint32_t i = inl + tid; i < hot; i += blockDim.x) wgp[c * cstride + i] = 0;

    const int nb = P.b_hi - P.b_lo;
    const int per = (nb + P.n_parts - 1) / P.n_parts;
    const int pb0 = P.b_lo + part * per, pb1 = min(P.b_hi, pb0 + per);
    const int nph = 2 * max(0, pb1 - pb0);
    const int G = P.n_ranges;
    const int nv = P.n_cot * half_trials;

    // weights of phase q into registers
    int64_t vreg[kVqRegs];
    auto load_vq = [&](int q) {
        const int64_t tfirst = static_cast<int64_t>(pb0 + q / 2) * P.tb + static_cast<int64_t>(8 * (q & 1)) * P.tg;
#pragma unroll
        for (int k = 0; k < kVqRegs; ++k) {
            const int idx = tid + k * kBwdThreads;
            int64_t v = 0;
            if (idx < nv) {
                const int c = idx / half_trials, i = idx - c * half_trials;
                const int64_t t = tfirst + i;
                if (t >= P.t0 && t < P.t1) v = P.vq[(static_cast<size_t>(c) * P.n_layers + j) * P.n + (t - P.t0)];
            }
            vreg[k] = v;
        }
    };
    // this wavefront's share of phase q: half the steps of one segment
    auto meta = [&](int q, int64_t &sbq, int &a, int &bnd) {
        const int bq = pb0 + q / 2, g = 8 * (q & 1) + (w >> 1);
        const size_t si = (static_cast<size_t>(bq) * G + r) * kGroups + g;
        const int R = P.seg_run[si];
        sbq = P.seg_base[si];
        const int mid = (R + 1) >> 1;
        a = (w & 1) ? mid : 0;
        bnd = (w & 1) ? R : mid;
    };
    const uint32_t pad = pad_entry(P.tb);
    uint32_t X[kBwdUnroll];
    auto chunk = [&](int64_t sbq, int from, int to) {
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u)
            X[u] = (from + u < to) ? __builtin_nontemporal_load(P.ent + sbq + static_cast<int64_t>(from + u) * kWave + lane)
                                   : pad;
    };
    const bool all_lds = hot <= static_cast<uint32_t>(P.capw);   // uniform over the workgroup

    int64_t sb_c = 0, sb_n = 0;
    int a_c = 0, b_c = 0, a_n = 0, b_n = 0;
    if (nph > 0) {
        meta(0, sb_c, a_c, b_c);
        chunk(sb_c, a_c, b_c);
        load_vq(0);
    }
    for (int ph = 0; ph < nph; ++ph) {
        if (ph + 1 < nph) meta(ph + 1, sb_n, a_n, b_n);
        __syncthreads();   // every wave is done with the previous phase's weights
#pragma unroll
        for (int k = 0; k < kVqRegs; ++k) {
            const int idx = tid + k * kBwdThreads;
            if (idx < nv) vql[idx] = vreg[k];
        }
        __syncthreads();
        if (ph + 1 < nph) load_vq(ph + 1);
        const uint32_t tl0 = static_cast<uint32_t>(8 * (ph & 1)) * P.tg;
        int st = a_c;
        bool prefetched_next = false;
        while (st < b_c) {
            uint32_t Y[kBwdUnroll];
#pragma unroll
            for (int u = 0; u < kBwdUnroll; ++u) Y[u] = X[u];
            const int nst = st + kBwdUnroll;
            if (nst < b_c) {
                chunk(sb_c, nst, b_c);
            } else if (ph + 1 < nph) {
                chunk(sb_n, a_n, b_n);
                prefetched_next = true;
            }
            // branch-free lookups of all entries, then the masked accumulation
            uint2 q[kBwdUnroll];
#pragma unroll
            for (int u = 0; u < kBwdUnroll; ++u) q[u] = tbr[(Y[u] & (kRange - 1)) >> 5];
            uint32_t rk[kBwdUnroll], ti[kBwdUnroll];
            bool on[kBwdUnroll];
#pragma unroll
            for (int u = 0; u < kBwdUnroll; ++u) {
                const uint32_t bit = Y[u] & 31;
                ti[u] = (Y[u] >> kRangeBits) - tl0;
                on[u] = ((q[u].x >> bit) & 1u) && ti[u] < static_cast<uint32_t>(half_trials);   // padding is off
                rk[u] = q[u].y + __popc(q[u].x & ((1u << bit) - 1u));
            }
            for (int c = 0; c < P.n_cot; ++c) {
                int64_t v[kBwdUnroll];
#pragma unroll
                for (int u = 0; u < kBwdUnroll; ++u) v[u] = vql[c * half_trials + (on[u] ? ti[u] : 0)];
#pragma unroll
                for (int u = 0; u < kBwdUnroll; ++u) {
                    if (!(on[u] && v[u] != 0)) continue;
                    if (all_lds || rk[u] < static_cast<uint32_t>(P.capw))
                        atomicAdd(&wl[c * P.capw + rk[u]], static_cast<unsigned long long>(v[u]));
                    else
                        atomicAdd(reinterpret_cast<unsigned long long *>(&wgp[c * cstride + rk[u]]),
                                  static_cast<unsigned long long>(v[u]));
                }
            }
            st = nst;
        }
        if (!prefetched_next && ph + 1 < nph) chunk(sb_n, a_n, b_n);
        sb_c = sb_n;
        a_c = a_n;
        b_c = b_n;
    }
    __syncthreads();
    for (int c = 0; c < P.n_cot; ++c)
        for (uint32_t i = tid; i < inl; i += blockDim.x) wgp[c * cstride + i] = static_cast<int64_t>(wl[c * P.capw + i]);
}

struct BwdGrad {
    const float *loss;
    const uint32_t *present;
    int32_t catalog, words;
    const int32_t *elt_off, *elt_ids;
    const double *elt_terms, *layer_terms;
    const OccTables *tabs;
    const int64_t *wg;
    size_t wg_stride;
    int32_t n_parts, n_cot, n_chunks;   // chunks = n_sr * kChunks
    const VScale *vs;
    double *part_elt;    // [n_layers][n_chunks][kMaxJ][n_cot][3]
    double *part_occ;    // [n_layers][n_chunks][n_cot][2]
};

// (5) per 4096-event chunk: W(e) times the derivatives of O(e).
__global__ __launch_bounds__(kBwdThreads) void k_bwd_grad(BwdGrad P) {
    __shared__ uint32_t stage[kMaxJ * kChunkWords];
    __shared__ int32_t lk[kMaxJ];
    __shared__ double ls[kMaxJ], lr[kMaxJ], ll[kMaxJ];
    __shared__ double wpart[16][kMaxCot][3];
    __shared__ double opart[16][kMaxCot][2];
    const int s = blockIdx.x / kChunks, p = blockIdx.x % kChunks, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int a = P.elt_off[j];
    const int J = P.elt_off[j + 1] - a;
    for (int q = tid; q < J; q += blockDim.x) {
        const int k = P.elt_ids[a + q];
        lk[q] = k;
        ls[q] = P.elt_terms[3 * k + 0];
        lr[q] = P.elt_terms[3 * k + 1];
        ll[q] = P.elt_terms[3 * k + 2];
    }
    __syncthreads();
    for (int idx = tid; idx < J * kChunkWords; idx += blockDim.x) {
        const int q = idx / kChunkWords, ww = idx % kChunkWords;
        const int64_t gw = static_cast<int64_t>(s) * kSrWords + p * kChunkWords + ww;
        stage[idx] = (gw < P.words) ? P.present[static_cast<size_t>(lk[q]) * P.words + gw] : 0u;
    }
    const double occR = P.layer_terms[4 * j + 0], occL = P.layer_terms[4 * j + 1];
    const OccTables T = P.tabs[j];
    const int64_t ev0 = static_cast<int64_t>(s) * kSr + p * (kChunkWords * 32);
    __syncthreads();

    // the thread's four events: weight per row and occurrence-clamp branch.
    // O = min(max(x - OccR, 0), OccL) is non-zero for these events, and it is
    // below OccL exactly when the occurrence clamp is in its linear branch.
    double W[4][kMaxCot];
    bool lin_occ[4];
    int local[4];
    double po[kMaxCot][2];
    for (int c = 0; c < kMaxCot; ++c) po[c][0] = po[c][1] = 0.0;
    for (int it = 0; it < 4; ++it) {
        local[it] = it * 1024 + tid;
        const int wip = local[it] >> 5, bit = local[it] & 31;
        const uint2 q = T.br[static_cast<size_t>(s) * kSrWords + p * kChunkWords + wip];
        lin_occ[it] = false;
        for (int c = 0; c < kMaxCot; ++c) W[it][c] = 0.0;
        if (!((q.x >> bit) & 1u)) continue;
        const uint32_t rk = q.y + __popc(q.x & ((1u << bit) - 1u));
        const double O = T.vals[static_cast<size_t>(s) * kSr + rk];
        for (int c = 0; c < P.n_cot; ++c) {
            const int64_t *wc = P.wg + (static_cast<size_t>(j) * P.n_cot + c) * P.n_parts * P.wg_stride +
                                static_cast<size_t>(s) * kSr + rk;
            int64_t acc = 0;
            for (int pt = 0; pt < P.n_parts; ++pt) acc += wc[static_cast<size_t>(pt) * P.wg_stride];
            W[it][c] = ldexp(static_cast<double>(acc), -P.vs[j * P.n_cot + c].sigma);
        }
        lin_occ[it] = O < occL;
        for (int c = 0; c < P.n_cot; ++c) {
            if (lin_occ[it]) po[c][0] -= W[it][c];
            else po[c][1] += W[it][c];
        }
    }
    // occurrence-term partials
    for (int c = 0; c < P.n_cot; ++c)
        for (int m = 0; m < 2; ++m) {
            double v = po[c][m];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
            if (lane == 0) opart[w][c][m] = v;
        }
    __syncthreads();
    const size_t chunk = static_cast<size_t>(s) * kChunks + p;
    if (tid < P.n_cot * 2) {
        const int c = tid >> 1, m = tid & 1;
        double v = 0.0;
        for (int i = 0; i < 16; ++i) v += opart[i][c][m];
        P.part_occ[((static_cast<size_t>(j) * P.n_chunks + chunk) * P.n_cot + c) * 2 + m] = v;
    }
    // ELT-term partials, one ELT of the layer at a time
    for (int qq = 0; qq < J; ++qq) {
        double pe[kMaxCot][3];
        for (int c = 0; c < kMaxCot; ++c) pe[c][0] = pe[c][1] = pe[c][2] = 0.0;
        float lv[4];
        bool on[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int wip = local[it] >> 5, bit = local[it] & 31;
            on[it] = lin_occ[it] && ((stage[qq * kChunkWords + wip] >> bit) & 1u);
            const size_t idx = on[it] ? static_cast<size_t>(lk[qq]) * P.catalog + ev0 + local[it] : 0;
            lv[it] = P.loss[idx];   // element 0 (always valid) for events without the ELT
        }
        for (int it = 0; it < 4; ++it) {
            if (!on[it]) continue;
            const double l = static_cast<double>(lv[it]);
            const double scaled = ls[qq] * l;
            const double pre = scaled - lr[qq];
            const double av = (pre > 0.0) ? pre : 0.0;
            const bool lin = (pre > 0.0) && (av < ll[qq]);
            const bool cap = av >= ll[qq];
            for (int c = 0; c < P.n_cot; ++c) {
                if (lin) {
                    pe[c][0] += W[it][c] * l;
                    pe[c][1] -= W[it][c];
                }
                if (cap) pe[c][2] += W[it][c];
            }
        }
        __syncthreads();   // wpart is reused per ELT
        for (int c = 0; c < P.n_cot; ++c)
            for (int m = 0; m < 3; ++m) {
                double v = pe[c][m];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
                if (lane == 0) wpart[w][c][m] = v;
            }
        __syncthreads();
        if (tid < P.n_cot * 3) {
            const int c = tid / 3, m = tid % 3;
            double v = 0.0;
            for (int i = 0; i < 16; ++i) v += wpart[i][c][m];
            P.part_elt[(((static_cast<size_t>(j) * P.n_chunks + chunk) * kMaxJ + qq) * P.n_cot + c) * 3 + m] = v;
        }
    }
}

// (6) fixed-order sums into the outputs: one workgroup per output value,
// each thread a fixed stride of the partials, then a fixed-order tree.
__global__ __launch_bounds__(256) void k_bwd_final(const int32_t *__restrict__ elt_off, const int32_t *__restrict__ elt_ids,
                                                  int n_layers, int n_elts, int n_cot, int n_chunks, int nwg_v,
                                                  const double *__restrict__ part_elt, const double *__restrict__ part_occ,
                                                  const double *__restrict__ aggpart, double *__restrict__ grad_elt,
                                                  double *__restrict__ grad_layer) {
    __shared__ double red[256];
    const int o = blockIdx.x, tid = threadIdx.x;
    const int n_e = n_cot * n_elts * 3;
    double v = 0.0;
    if (o < n_e) {
        const int c = o / (n_elts * 3), k = (o / 3) % n_elts, m = o % 3;
        for (int j = 0; j < n_layers; ++j)
            for (int q = elt_off[j]; q < elt_off[j + 1]; ++q) {
                if (elt_ids[q] != k) continue;
                const int qq = q - elt_off[j];
                for (int ch = tid; ch < n_chunks; ch += blockDim.x)
                    v += part_elt[(((static_cast<size_t>(j) * n_chunks + ch) * kMaxJ + qq) * n_cot + c) * 3 + m];
            }
    } else {
        const int i = o - n_e;
        const int c = i / (n_layers * 4), j = (i / 4) % n_layers, m = i % 4;
        if (m < 2) {
            for (int ch = tid; ch < n_chunks; ch += blockDim.x)
                v += part_occ[((static_cast<size_t>(j) * n_chunks + ch) * n_cot + c) * 2 + m];
        } else {
            for (int wg = tid; wg < nwg_v; wg += blockDim.x)
                v += aggpart[((static_cast<size_t>(j) * n_cot + c) * nwg_v + wg) * 2 + (m - 2)];
        }
    }
    red[tid] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        if (o < n_e) grad_elt[o] = red[0];
        else {
            const int i = o - n_e;
            const int c = i / (n_layers * 4), j = (i / 4) % n_layers, m = i % 4;
            grad_layer[(static_cast<size_t>(c) * n_layers + j) * 4 + m] = red[0];
        }
    }
}

struct BwdLayout {
    OccLayoutSizes z;
    int n_parts, nwg_v, n_chunks;
    size_t wg_stride;
    size_t bytes;
};

static int bwd_nwg_v(int64_t n) {
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 8191) / 8192, 512)));
}

static BwdLayout bwd_layout(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, int n_cot,
                            int64_t n) {
    BwdLayout B{};
    B.z = occ_sizes(tables->catalog, false);
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    const int cu = device_cu_count();
    // one workgroup per CU at most (they need all of its LDS): parts = CUs / ranges
    B.n_parts = std::max(1, std::min(std::max(yet->n_blocks, 1), cu / std::max(yet->n_ranges, 1)));
    B.nwg_v = bwd_nwg_v(n);
    B.n_chunks = B.z.n_sr * kChunks;
    B.wg_stride = static_cast<size_t>(B.z.n_sr) * kSr;
    Carver c(nullptr);
    c.take<int32_t>(kWsHeaderBytes / 4);
    c.take<int32_t>(static_cast<size_t>(L + 1));
    c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    c.take<OccTables>(static_cast<size_t>(std::max(L, 1)));
    size_t b = c.bytes() + static_cast<size_t>(L) * B.z.per_layer;
    Carver d(nullptr);
    d.take<VScale>(static_cast<size_t>(std::max(L * n_cot, 1)));
    d.take<double>(static_cast<size_t>(L) * n_cot * B.nwg_v * 2);
    d.take<int64_t>(static_cast<size_t>(n_cot) * L * std::max<int64_t>(n, 1));
    d.take<int64_t>(static_cast<size_t>(L) * n_cot * B.n_parts * B.wg_stride);
    d.take<double>(static_cast<size_t>(L) * B.n_chunks * kMaxJ * n_cot * 3);
    d.take<double>(static_cast<size_t>(L) * B.n_chunks * n_cot * 2);
    B.bytes = b + d.bytes();
    return B;
}

static int32_t check_pair_b(const ara_tables *tables, const ara_yet *yet) {
    if (!tables || !yet) return fail(ARA_E_INVAL, "null tables or yet");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (yet->range_bits != kRangeBits || yet->groups != kGroups) return fail(ARA_E_INVAL, "YET not prepared by this library");
    return ARA_OK;
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_ylt_backward_workspace_bytes(const ara_tables *tables, const ara_yet *yet,
                                                    const ara_layers *layers, int32_t n_cot, size_t *bytes) {
    if (!bytes) return fail(ARA_E_INVAL, "null output");
    int32_t rc = check_pair_b(tables, yet);
    if (rc) return rc;
    if ((rc = check_layers(layers, tables->n_elts))) return rc;
    if (n_cot < 1 || n_cot > kMaxCot) return fail(ARA_E_LIMIT, "cotangent rows must be 1..ARA_MAX_COTANGENTS");
    *bytes = bwd_layout(tables, yet, layers, n_cot, yet->n_trials).bytes;
    return ARA_OK;
}

extern "C" int32_t ara_ylt_backward(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                    const double *elt_terms, const double *layer_terms, int64_t trial_begin,
                                    int64_t trial_end, const double *s_pre, int32_t n_cot, const double *grad_ylt,
                                    double *grad_elt, double *grad_layer, void *ws, size_t ws_bytes, void *stream) {
    int32_t rc = check_pair_b(tables, yet);
    if (rc) return rc;
    if ((rc = check_layers(layers, tables->n_elts))) return rc;
    if (n_cot < 1 || n_cot > kMaxCot) return fail(ARA_E_LIMIT, "cotangent rows must be 1..ARA_MAX_COTANGENTS");
    if (trial_begin < 0 || trial_end < trial_begin || trial_end > yet->n_trials)
        return fail(ARA_E_RANGE, "trial range outside the YET");
    if (!ws || !grad_elt || !grad_layer) return fail(ARA_E_INVAL, "null workspace or output");
    const int L = layers->n_layers;
    const int64_t n = trial_end - trial_begin;
    if (L > 0 && n > 0 && (!s_pre || !grad_ylt || !elt_terms || !layer_terms))
        return fail(ARA_E_INVAL, "null input");
    // workspace sized for the full trial range is valid for any sub-range
    const BwdLayout B = bwd_layout(tables, yet, layers, n_cot, yet->n_trials);
    if (ws_bytes < B.bytes) return fail(ARA_E_NOSPACE, "backward workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
    ARA_HIP(hipMemsetAsync(grad_elt, 0, static_cast<size_t>(n_cot) * tables->n_elts * 3 * sizeof(double), st));
    ARA_HIP(hipMemsetAsync(grad_layer, 0, static_cast<size_t>(n_cot) * L * 4 * sizeof(double), st));
    if (L == 0 || n == 0) return ARA_OK;

    const int nJ = layers->elt_off[L];
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / 4);
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, B.z, false);
    VScale *vs = c.take<VScale>(static_cast<size_t>(L * n_cot));
    double *aggpart = c.take<double>(static_cast<size_t>(L) * n_cot * bwd_nwg_v(n) * 2);
    int64_t *vq = c.take<int64_t>(static_cast<size_t>(n_cot) * L * n);
    int64_t *wgb = c.take<int64_t>(static_cast<size_t>(L) * n_cot * B.n_parts * B.wg_stride);
    double *part_elt = c.take<double>(static_cast<size_t>(L) * B.n_chunks * kMaxJ * n_cot * 3);
    double *part_occ = c.take<double>(static_cast<size_t>(L) * B.n_chunks * n_cot * 2);
    ARA_HIP(hipMemsetAsync(vs, 0, static_cast<size_t>(L * n_cot) * sizeof(VScale), st));
    ARA_HIP(hipMemcpyAsync(d_off, layers->elt_off, (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (nJ > 0) ARA_HIP(hipMemcpyAsync(d_ids, layers->elt_ids, nJ * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(d_tabs, tabs.data(), L * sizeof(OccTables), hipMemcpyHostToDevice, st));

    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, false, d_tabs, B.z.n_sr, d_err, st)))
            return rc;
    }
    const int nwg_v = bwd_nwg_v(n);
    {
        ProfScope prof(ARA_PROF_BWD_RED, st);
        k_bwd_vmax<<<dim3(nwg_v, L), kBwdThreads, 0, st>>>(grad_ylt, s_pre, layer_terms, n, L, n_cot, nwg_v, vs, aggpart);
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 2048));
        k_bwd_vq<<<dim3(gx, L), 256, 0, st>>>(grad_ylt, s_pre, layer_terms, n, L, n_cot, yet->max_occ, vs, vq);
        ARA_HIP(hipGetLastError());
    }
    BwdStream S{};
    S.ent = yet->ent;
    S.seg_base = yet->seg_base;
    S.seg_run = yet->seg_run;
    S.t0 = trial_begin;
    S.t1 = trial_end;
    S.n = n;
    S.tg = yet->trials_per_group;
    S.tb = yet->trials_per_block;
    S.n_ranges = yet->n_ranges;
    S.n_parts = B.n_parts;
    S.n_cot = n_cot;
    S.n_layers = L;
    S.b_lo = static_cast<int32_t>(trial_begin / yet->trials_per_block);
    S.b_hi = static_cast<int32_t>((trial_end + yet->trials_per_block - 1) / yet->trials_per_block);
    const size_t fixed = 1024 * sizeof(uint2) + static_cast<size_t>(n_cot) * 8 * yet->trials_per_group * sizeof(int64_t);
    S.capw = static_cast<int32_t>((kLds - fixed) / (static_cast<size_t>(n_cot) * sizeof(int64_t)));
    S.tabs = d_tabs;
    S.vq = vq;
    S.wg = wgb;
    S.wg_stride = B.wg_stride;
    {
        ProfScope prof(ARA_PROF_BWD, st);
        static bool attr = false;
        if (!attr) {
            ARA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bwd_stream),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, kLds));
            attr = true;
        }
        k_bwd_stream<<<dim3(yet->n_ranges * B.n_parts, L), kBwdThreads, kLds, st>>>(S);
        ARA_HIP(hipGetLastError());
    }
    BwdGrad Gp{};
    Gp.loss = tables->loss;
    Gp.present = tables->present;
    Gp.catalog = tables->catalog;
    Gp.words = tables->words;
    Gp.elt_off = d_off;
    Gp.elt_ids = d_ids;
    Gp.elt_terms = elt_terms;
    Gp.layer_terms = layer_terms;
    Gp.tabs = d_tabs;
    Gp.wg = wgb;
    Gp.wg_stride = B.wg_stride;
    Gp.n_parts = B.n_parts;
    Gp.n_cot = n_cot;
    Gp.n_chunks = B.n_chunks;
    Gp.vs = vs;
    Gp.part_elt = part_elt;
    Gp.part_occ = part_occ;
    {
        ProfScope prof(ARA_PROF_BWD_RED, st);
        k_bwd_grad<<<dim3(B.n_chunks, L), kBwdThreads, 0, st>>>(Gp);
        const int outs = n_cot * tables->n_elts * 3 + n_cot * L * 4;
        k_bwd_final<<<outs, 256, 0, st>>>(d_off, d_ids, L, tables->n_elts, n_cot, B.n_chunks, nwg_v, part_elt,
                                          part_occ, aggpart, grad_elt, grad_layer);
        ARA_HIP(hipGetLastError());
    }
    return ARA_OK;
}
