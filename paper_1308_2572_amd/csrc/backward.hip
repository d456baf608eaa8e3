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
// The forward gathers O(e) per trial; its adjoint scatters v_t per event.
// Read through the event-major copy of the YET the scatter is a gather
// again, and only the hot events' occurrence lists are read at all.
//
// Kernels: (1) the hot occurrence tables (shared with the forward);
// (2) v_t per cotangent row, its largest magnitude and the aggregate-term
// sums; (3) v_t in 64-bit fixed point, scaled so that no partial sum of W
// can overflow (|W| <= max|v| * largest occurrence count of one event);
// (4) the list of hot events; (5) W(e) per hot event, gathered per trial
// slice over the event-major YET and combined with integer atomics, so the
// result does not depend on the order; (6) over the hot events, W times
// the per-event derivatives, reduced in a fixed order; (7) a fixed-order sum
// of the chunk partials into the outputs.
//
// Step (5) has a second form for cotangents that take one value on most
// trials, as the metrics' do (AAL: the same weight wherever the aggregate
// clamp is linear; PML, TVaR: zero outside the tied or top trials).  With c
// that common fixed-point value and D the trials whose value differs,
//   W(e) = c * (occurrences of e in the call's trials)
//          + sum over t in D of (v_t - c) * (occurrences of e in t),
// integer arithmetic that gives the gather's result bit for bit.  The
// occurrence counts come from the event-major offsets: over all trials the
// per-event totals, over part of them the list lengths of the trial slices
// the range covers whole, plus a count of the in-range entries of the (at
// most two) slices it cuts; the second term comes from the trial-major copy
// of the deviating trials' events.  It is used when the trials to walk are
// at most a sixteenth of all (each walked trial costs about sixteen times
// its share of the gather's time); the decision is taken on the device from
// the counts, so both forms are enqueued and the one not chosen returns at
// once.
#include "occ.h"
#include "wave.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace ara {

constexpr int kBwdThreads = 1024;
constexpr int kMaxCot = ARA_MAX_COTANGENTS;

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

__device__ __forceinline__ void chunk_range(int64_t n, int nwg, int wg, int64_t &lo, int64_t &hi) {
    const int64_t c = (n + nwg - 1) / nwg;
    lo = std::min<int64_t>(n, static_cast<int64_t>(wg) * c);
    hi = std::min<int64_t>(n, lo + c);
}

// (2) largest |c_t a_t| per (layer, row); aggregate-term partial sums.  One
// pass over the trials of the workgroup's chunk reads S once for every row;
// the sums meet in fixed order (each thread's trials, DPP across the
// wavefront, the wavefronts in index order).
__global__ __launch_bounds__(kBwdThreads) void k_bwd_vmax(const double *__restrict__ cot, const double *__restrict__ s_pre,
                                                         const double *__restrict__ layer_terms, int64_t n, int n_layers,
                                                         int n_cot, int nwg, VScale *__restrict__ vs,
                                                         double *__restrict__ aggpart) {
    __shared__ double red[kBwdThreads / 64][kMaxCot][3];
    const int wg = blockIdx.x, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double aggR = layer_terms[4 * j + 2], aggL = layer_terms[4 * j + 3];
    int64_t lo, hi;
    chunk_range(n, nwg, wg, lo, hi);
    const double *S = s_pre + static_cast<size_t>(j) * n;
    double m[kMaxCot], sr[kMaxCot], sl[kMaxCot];
#pragma unroll
    for (int c = 0; c < kMaxCot; ++c) m[c] = sr[c] = sl[c] = 0.0;
    for (int64_t t = lo + tid; t < hi; t += blockDim.x) {
        const double st = S[t];
        const bool lin = agg_linear(st, aggR, aggL), cap = agg_capped(st, aggR, aggL);
#pragma unroll
        for (int c = 0; c < kMaxCot; ++c)
            if (c < n_cot) {
                const double g = cot[(static_cast<size_t>(c) * n_layers + j) * n + t];
                if (lin) {
                    sr[c] += g;
                    m[c] = fmax(m[c], fabs(g));
                }
                if (cap) sl[c] += g;
            }
    }
#pragma unroll
    for (int c = 0; c < kMaxCot; ++c)
        if (c < n_cot) {
            double mc = m[c];
            for (int o = 32; o > 0; o >>= 1) mc = fmax(mc, __shfl_down(mc, o));
            const double tr = wave_inclusive_sum(sr[c]), tl = wave_inclusive_sum(sl[c]);
            if (lane == 0) red[w][c][2] = mc;
            if (lane == 63) {
                red[w][c][0] = tr;
                red[w][c][1] = tl;
            }
        }
    __syncthreads();
    if (tid < n_cot * 2) {
        const int c = tid >> 1, h = tid & 1;
        double t = 0.0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += red[i][c][h];
        aggpart[((static_cast<size_t>(j) * n_cot + c) * nwg + wg) * 2 + h] = h ? t : -t;
    } else if (tid >= 64 && tid < 64 + n_cot) {   // one atomic per (workgroup, row)
        const int c = tid - 64;
        double mc = 0.0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) mc = fmax(mc, red[i][c][2]);
        if (mc > 0.0)
            atomicMax(&vs[j * n_cot + c].maxabs_bits, static_cast<unsigned long long>(__double_as_longlong(mc)));
    }
}

__device__ __forceinline__ int sigma_of(const VScale &v, int max_occ) {
    const double m = __longlong_as_double(static_cast<long long>(v.maxabs_bits));
    if (!(m > 0.0)) return 0;
    int e;
    frexp(m * static_cast<double>(max_occ > 0 ? max_occ : 1), &e);   // m*max_occ < 2^e
    return 62 - e;
}

// (3) fixed-point weights vq[j][t][c] = round(c_t a_t 2^sigma), the rows of
// one trial side by side (cs >= n_cot slots, the spare ones zero) so that one
// gather fetches every row.
__global__ void k_bwd_vq(const double *__restrict__ cot, const double *__restrict__ s_pre,
                         const double *__restrict__ layer_terms, int64_t n, int n_layers, int n_cot, int cs,
                         int max_occ, VScale *__restrict__ vs, int64_t *__restrict__ vq) {
    const int j = blockIdx.y;
    const double aggR = layer_terms[4 * j + 2], aggL = layer_terms[4 * j + 3];
    const double *S = s_pre + static_cast<size_t>(j) * n;
    int sg[kMaxCot];
    for (int c = 0; c < n_cot; ++c) {
        sg[c] = sigma_of(vs[j * n_cot + c], max_occ);
        if (blockIdx.x == 0 && threadIdx.x == 0) vs[j * n_cot + c].sigma = sg[c];
    }
    int64_t *q = vq + static_cast<size_t>(j) * n * cs;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool lin = agg_linear(S[t], aggR, aggL);
        for (int c = 0; c < cs; ++c) {
            int64_t r = 0;
            if (c < n_cot && lin) {
                const double v = cot[(static_cast<size_t>(c) * n_layers + j) * n + t];
                r = (v == 0.0) ? 0 : static_cast<int64_t>(__double2ll_rn(ldexp(v, sg[c])));
            }
            q[static_cast<size_t>(t) * cs + c] = r;
        }
    }
}

// (4) the layer's hot events (O(e) != 0) as one list, in (super-range,
// rank) order: hot_ev[g] is the event of hot index g = hot_base[s] + rank;
// the weight accumulators of every hot index start at zero.
__global__ __launch_bounds__(256) void k_bwd_hot(const OccTables *__restrict__ tabs, int n_sr, int n_cot,
                                                 int32_t catalog, int32_t *__restrict__ hot_ev,
                                                 int32_t *__restrict__ hot_base, int64_t *__restrict__ W) {
    __shared__ int32_t red[4];
    const int s = blockIdx.x, j = blockIdx.y, tid = threadIdx.x;
    const OccTables T = tabs[j];
    int32_t part = 0;
    for (int i = tid; i < s; i += blockDim.x) part += T.count[i];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o);
    if ((tid & 63) == 0) red[tid >> 6] = part;
    __syncthreads();
    const int32_t base = red[0] + red[1] + red[2] + red[3];
    int32_t *hb = hot_base + static_cast<size_t>(j) * (n_sr + 1);
    if (tid == 0) {
        hb[s] = base;
        if (s == n_sr - 1) hb[n_sr] = base + T.count[s];
    }
    int32_t *hev = hot_ev + static_cast<size_t>(j) * catalog;
    int64_t *Wj = W + static_cast<size_t>(j) * n_cot * catalog;
    for (int i = tid; i < kSrWords; i += blockDim.x) {
        const uint2 q = T.br[static_cast<size_t>(s) * kSrWords + i];
        uint32_t m = q.x;
        int32_t g = base + static_cast<int32_t>(q.y);
        while (m) {
            const int bit = __builtin_ctz(m);
            hev[g] = s * kSr + 32 * i + bit;
            for (int c = 0; c < n_cot; ++c) Wj[static_cast<size_t>(c) * catalog + g] = 0;
            ++g;
            m &= m - 1;
        }
    }
}

constexpr int kCand = 8;   // candidates for the common value of a row: 0 and seven sampled trials
constexpr int kDevChunk = 4096;   // trials per workgroup when counting and listing them

struct BwdSparse {
    const int64_t *vq;                 // [n_layers][n][cs]
    int64_t n, t0, n_trials;
    int32_t cs, n_cot, catalog, n_sr;
    int64_t slice_trials;              // trials of one slice of the event-major copy
    const int64_t *tr_off;             // event-major copy: list offsets per (slice, event)
    const uint32_t *tr_ent;            //   and the lists' slice-local trial indices
    unsigned long long *ndev;          // [n_layers] deviating trials
    int64_t *common;                   // [n_layers][kMaxCot] the chosen common value
    int32_t *dev;                      // [n_layers][n] deviating trials (call-relative)
    const int32_t *t_cnt;              // occurrences of each event
    const int64_t *t_off;              // trial-major copy
    const int32_t *t_ids;
    const OccTables *tabs;
    const int32_t *hot_ev, *hot_base;
    int64_t *W;                        // [n_layers][n_cot][catalog], by hot index
};

__device__ __forceinline__ int64_t cand_value(const BwdSparse &P, int j, int c, int k) {
    if (k == 0 || P.n == 0) return 0;
    const int64_t t = (static_cast<int64_t>(k) * P.n) / kCand;
    return P.vq[(static_cast<size_t>(j) * P.n + t) * P.cs + c];
}

// Whether some row's common value is non-zero (W then starts from c times
// the occurrence counts).
__device__ __forceinline__ bool common_nonzero(const BwdSparse &P, int j) {
    for (int c = 0; c < P.n_cot; ++c)
        if (P.common[static_cast<size_t>(j) * kMaxCot + c] != 0) return true;
    return false;
}

// Trial slice x of the event-major copy holds trials [x S, min((x + 1) S, N)).
__device__ __forceinline__ bool slice_inside(const BwdSparse &P, int x) {
    const int64_t lo = static_cast<int64_t>(x) * P.slice_trials;
    const int64_t hi = min(lo + P.slice_trials, P.n_trials);
    return lo >= P.t0 && hi <= P.t0 + P.n;
}

__device__ __forceinline__ bool slice_cut(const BwdSparse &P, int x) {
    const int64_t lo = static_cast<int64_t>(x) * P.slice_trials;
    const int64_t hi = min(lo + P.slice_trials, P.n_trials);
    return max(lo, P.t0) < min(hi, P.t0 + P.n) && !slice_inside(P, x);
}

// Deviating trials the second form walks: those of the range.
__device__ __forceinline__ int64_t sparse_walk(const BwdSparse &P, int j) { return static_cast<int64_t>(P.ndev[j]); }

// The second form's condition, the same in every kernel that reads it: at
// most a sixteenth of all the trials to walk.
constexpr int kWalkShare = 16;
__device__ __forceinline__ bool sparse_chosen(const BwdSparse &P, int j) {
    return sparse_walk(P, j) * kWalkShare <= P.n_trials;
}

struct BwdGather {
    const int64_t *tr_off;        // event-major YET
    const uint32_t *tr_ent;
    int32_t catalog, n_sr, n_cot, pad;
    int64_t slice_trials;
    int64_t t0, t1, n;            // trial range of the call
    const int32_t *hot_ev;        // [n_layers][catalog]
    const int32_t *hot_base;      // [n_layers][n_sr + 1]
    const int64_t *vq;            // [n_layers][n][CS]
    int64_t *W;                   // [n_layers][n_cot][catalog], by hot index
    BwdSparse sp;                 // the second form's state
    int32_t use_sp;               // 0 when the second form is not available (no trial-major copy)
    int32_t pad2;
};

// (5) W(e) = sum of v_t over the occurrences (t, e), per hot event, as a
// gather over the event-major YET.  Workgroup i works on trial slice i mod 8
// only, which keeps its gathers of v in the L2 of one XCD; a group of G
// lanes owns one hot event at a time, reads its list coalesced (G
// consecutive entries per step, streamed past the cache) and sums the
// trials' fixed-point weights; the group's sums meet in a lane reduction and
// the eight slice sums in one integer atomic add per (event, row) -- exact
// in any order.
template <int CS, int G>
__global__ __launch_bounds__(256) void k_bwd_w(BwdGather P) {
    constexpr int kU = 2;
    const int x = blockIdx.x % kSlices, wi = blockIdx.x / kSlices, nw = gridDim.x / kSlices, j = blockIdx.y;
    if (P.use_sp && sparse_chosen(P.sp, j)) return;   // W comes from the deviating trials instead
    const int64_t tx0 = static_cast<int64_t>(x) * P.slice_trials;
    const int64_t ulo = max<int64_t>(P.t0 - tx0, 0), uhi = min<int64_t>(P.t1 - tx0, P.slice_trials);
    if (uhi <= ulo) return;   // the slice lies outside the call's trials
    const uint32_t u0 = static_cast<uint32_t>(ulo), span = static_cast<uint32_t>(uhi - ulo);
    const int64_t *vq = P.vq + (static_cast<size_t>(j) * P.n + static_cast<size_t>(tx0 + ulo - P.t0)) * CS;
    const int H = P.hot_base[static_cast<size_t>(j) * (P.n_sr + 1) + P.n_sr];
    const int32_t *hev = P.hot_ev + static_cast<size_t>(j) * P.catalog;
    const int64_t *off = P.tr_off + static_cast<int64_t>(x) * P.catalog;
    int64_t *Wj = P.W + static_cast<size_t>(j) * P.n_cot * P.catalog;
    const int sub = threadIdx.x & (G - 1);
    const int ngrp = nw * static_cast<int>(blockDim.x) / G;
    for (int g = (wi * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) / G; g < H; g += ngrp) {
        const int e = hev[g];
        const int64_t o0 = off[e], o1 = off[e + 1];
        int64_t acc[CS];
#pragma unroll
        for (int c = 0; c < CS; ++c) acc[c] = 0;
        for (int64_t i = o0 + sub; i < o1; i += G * kU) {
            uint32_t d[kU];
#pragma unroll
            for (int v = 0; v < kU; ++v)
                d[v] = (i + v * G < o1) ? __builtin_nontemporal_load(P.tr_ent + i + v * G) - u0 : span;   // span = skip
#pragma unroll
            for (int v = 0; v < kU; ++v) {
                if (d[v] < span) {
                    const int64_t *q = vq + static_cast<size_t>(d[v]) * CS;
                    if constexpr (CS == 1) {
                        acc[0] += q[0];
                    } else {
#pragma unroll
                        for (int h = 0; h < CS; h += 2) {
                            const longlong2 t = *reinterpret_cast<const longlong2 *>(q + h);
                            acc[h] += t.x;
                            acc[h + 1] += t.y;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CS; ++c)
            for (int s = G / 2; s > 0; s >>= 1) acc[c] += __shfl_xor(acc[c], s, G);
        if (sub == 0) {
#pragma unroll
            for (int c = 0; c < CS; ++c)
                if (c < P.n_cot && acc[c] != 0)
                    atomicAdd(reinterpret_cast<unsigned long long *>(&Wj[static_cast<size_t>(c) * P.catalog + g]),
                              static_cast<unsigned long long>(acc[c]));
        }
    }
}

template <int G>
static void launch_bwd_w(int cs, dim3 grid, hipStream_t st, const BwdGather &S) {
    if (cs == 1) k_bwd_w<1, G><<<grid, 256, 0, st>>>(S);
    else if (cs == 2) k_bwd_w<2, G><<<grid, 256, 0, st>>>(S);
    else k_bwd_w<4, G><<<grid, 256, 0, st>>>(S);
}

// (5a) the common value of every row: of 0 and the values at seven sampled
// trials, the one held by most of 1024 evenly spaced trials (the first on
// ties).  Any choice gives the same W; a good one keeps the list of
// deviating trials short.  One workgroup per layer.
constexpr int kPickSamples = 1024;

__global__ __launch_bounds__(kPickSamples) void k_bwd_pick(BwdSparse P) {
    __shared__ uint32_t cnt[kMaxCot * kCand];
    const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    if (tid < kMaxCot * kCand) cnt[tid] = 0;
    __syncthreads();
    const int64_t t = (static_cast<int64_t>(tid) * P.n) / kPickSamples;
    const int64_t *q = P.vq + (static_cast<size_t>(j) * P.n + t) * P.cs;
    for (int c = 0; c < P.n_cot; ++c) {
        const int64_t v = q[c];
        for (int k = 0; k < kCand; ++k) {
            const uint64_t m = __ballot(v == cand_value(P, j, c, k));
            if (lane == 0 && m) atomicAdd(&cnt[c * kCand + k], static_cast<uint32_t>(__popcll(m)));
        }
    }
    __syncthreads();
    if (tid < kMaxCot) {
        int64_t cm = 0;
        if (tid < P.n_cot) {
            int best = 0;
            for (int k = 1; k < kCand; ++k)
                if (cnt[tid * kCand + k] > cnt[tid * kCand + best]) best = k;
            cm = cand_value(P, j, tid, best);
        }
        P.common[static_cast<size_t>(j) * kMaxCot + tid] = cm;
    }
}

// (5b) the list of trials where some row differs from its common value.
// A workgroup gathers the deviating trials of its chunk of kDevChunk trials
// in LDS and reserves their place in the list with one atomic.
__global__ __launch_bounds__(1024) void k_bwd_dev(BwdSparse P) {
    __shared__ int32_t buf[kDevChunk];
    __shared__ uint32_t nbuf;
    __shared__ unsigned long long base;
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    int64_t cm[kMaxCot];
#pragma unroll
    for (int c = 0; c < kMaxCot; ++c) cm[c] = P.common[static_cast<size_t>(j) * kMaxCot + c];
    if (threadIdx.x == 0) nbuf = 0;
    __syncthreads();
    const int64_t *q = P.vq + static_cast<size_t>(j) * P.n * P.cs;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kDevChunk;
    const int64_t c1 = min<int64_t>(c0 + kDevChunk, P.n);
    for (int64_t t0 = c0; t0 < c1; t0 += blockDim.x) {   // uniform
        const int64_t t = t0 + threadIdx.x;
        bool d = false;
        if (t < c1)
#pragma unroll
            for (int c = 0; c < kMaxCot; ++c)
                if (c < P.n_cot) d = d || (q[static_cast<size_t>(t) * P.cs + c] != cm[c]);
        const uint64_t m = __ballot(d);
        if (m) {
            uint32_t wb = 0;
            if (lane == 0) wb = atomicAdd(&nbuf, static_cast<uint32_t>(__popcll(m)));
            wb = __shfl(wb, 0);
            if (d) {
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
                buf[wb + pos] = static_cast<int32_t>(t);
            }
        }
    }
    __syncthreads();
    const uint32_t nb = nbuf;
    if (nb == 0) return;   // uniform
    if (threadIdx.x == 0) base = atomicAdd(&P.ndev[j], static_cast<unsigned long long>(nb));
    __syncthreads();
    int32_t *dv = P.dev + static_cast<size_t>(j) * P.n + base;
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) dv[i] = buf[i];
}

// (5c) W(e) = c * (occurrences of e in the trial slices the call covers
// whole; all trials: the per-event totals) for every hot event (when the
// second form is chosen and c is not zero; the accumulators are zero from
// step 4 otherwise)
__global__ __launch_bounds__(256) void k_bwd_winit(BwdSparse P) {
    const int j = blockIdx.y;
    if (!sparse_chosen(P, j) || !common_nonzero(P, j)) return;   // c = 0: W starts at zero
    const int H = P.hot_base[static_cast<size_t>(j) * (P.n_sr + 1) + P.n_sr];
    const int32_t *hev = P.hot_ev + static_cast<size_t>(j) * P.catalog;
    int64_t *Wj = P.W + static_cast<size_t>(j) * P.n_cot * P.catalog;
    const bool all = P.t0 == 0 && P.n == P.n_trials;   // uniform
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < H; g += gridDim.x * blockDim.x) {
        const int e = hev[g];
        int64_t cnt = 0;
        if (all) {
            cnt = P.t_cnt[e];
        } else {
#pragma unroll
            for (int x = 0; x < kSlices; ++x)
                if (slice_inside(P, x)) {
                    const int64_t *off = P.tr_off + static_cast<int64_t>(x) * P.catalog;
                    cnt += off[e + 1] - off[e];
                }
        }
#pragma unroll
        for (int c = 0; c < kMaxCot; ++c)
            if (c < P.n_cot)
                Wj[static_cast<size_t>(c) * P.catalog + g] = static_cast<int64_t>(
                    static_cast<unsigned long long>(P.common[static_cast<size_t>(j) * kMaxCot + c]) *
                    static_cast<unsigned long long>(cnt));   // exact modulo 2^64, like every sum below
    }
}

// (5c') the slices the call's range cuts (cut[0 .. ncut), at most two): for
// every hot event, c times the entries of its list in the slice that lie in
// the range.  Workgroup i works on cut slice i mod ncut, so that every
// workgroup has work; G lanes per hot event read its list coalesced and
// count, and the count meets W in one integer atomic per row.
template <int G>
__global__ __launch_bounds__(256) void k_bwd_wcut(BwdSparse P, int2 cut, int ncut) {
    constexpr int kU = 4;
    const int k = blockIdx.x % ncut, wi = blockIdx.x / ncut, nw = gridDim.x / ncut, j = blockIdx.y;
    const int x = k == 0 ? cut.x : cut.y;
    if (!sparse_chosen(P, j) || !common_nonzero(P, j) || !slice_cut(P, x)) return;   // uniform
    const int64_t tx0 = static_cast<int64_t>(x) * P.slice_trials;
    const int64_t ulo = max<int64_t>(P.t0 - tx0, 0), uhi = min<int64_t>(P.t0 + P.n - tx0, P.slice_trials);
    const uint32_t u0 = static_cast<uint32_t>(ulo), span = static_cast<uint32_t>(uhi - ulo);
    const int H = P.hot_base[static_cast<size_t>(j) * (P.n_sr + 1) + P.n_sr];
    const int32_t *hev = P.hot_ev + static_cast<size_t>(j) * P.catalog;
    const int64_t *off = P.tr_off + static_cast<int64_t>(x) * P.catalog;
    int64_t *Wj = P.W + static_cast<size_t>(j) * P.n_cot * P.catalog;
    const int sub = threadIdx.x & (G - 1);
    const int ngrp = nw * static_cast<int>(blockDim.x) / G;
    for (int g = (wi * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x)) / G; g < H; g += ngrp) {
        const int e = hev[g];
        const int64_t o0 = off[e], o1 = off[e + 1];
        uint32_t cnt = 0;
        for (int64_t i = o0 + sub; i < o1; i += G * kU) {
            uint32_t d[kU];
#pragma unroll
            for (int v = 0; v < kU; ++v)
                d[v] = (i + v * G < o1) ? __builtin_nontemporal_load(P.tr_ent + i + v * G) - u0 : span;   // span = skip
#pragma unroll
            for (int v = 0; v < kU; ++v) cnt += d[v] < span ? 1u : 0u;
        }
        for (int s2 = G / 2; s2 > 0; s2 >>= 1) cnt += static_cast<uint32_t>(__shfl_xor(static_cast<int>(cnt), s2, G));
        if (sub == 0 && cnt != 0) {
#pragma unroll
            for (int c = 0; c < kMaxCot; ++c)
                if (c < P.n_cot)
                    atomicAdd(reinterpret_cast<unsigned long long *>(&Wj[static_cast<size_t>(c) * P.catalog + g]),
                              static_cast<unsigned long long>(P.common[static_cast<size_t>(j) * kMaxCot + c]) *
                                  static_cast<unsigned long long>(cnt));
        }
    }
}

// (5d) the deviating trials of the range: a wavefront per trial adds
// v_t - c to W of each hot event of the trial, one integer atomic per
// (occurrence, row)
__global__ __launch_bounds__(256) void k_bwd_wsparse(BwdSparse P) {
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    if (!sparse_chosen(P, j)) return;
    const int64_t nwalk = sparse_walk(P, j);
    const OccTables T = P.tabs[j];
    const int32_t *hb = P.hot_base + static_cast<size_t>(j) * (P.n_sr + 1);
    const int64_t *q = P.vq + static_cast<size_t>(j) * P.n * P.cs;
    int64_t *Wj = P.W + static_cast<size_t>(j) * P.n_cot * P.catalog;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int64_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < nwalk; i += waves) {
        unsigned long long dl[kMaxCot];
        const int32_t u = P.dev[static_cast<size_t>(j) * P.n + i];
#pragma unroll
        for (int c = 0; c < kMaxCot; ++c)
            dl[c] = c < P.n_cot ? static_cast<unsigned long long>(q[static_cast<size_t>(u) * P.cs + c]) -
                                      static_cast<unsigned long long>(P.common[static_cast<size_t>(j) * kMaxCot + c])
                                : 0ull;
        const int64_t t = P.t0 + u;
        const int64_t a = P.t_off[t], b = P.t_off[t + 1];
        constexpr int kU = 16;   // events per lane in flight: a 1000-event trial in one round
        for (int64_t k0 = a; k0 < b; k0 += 64 * kU) {
            int e[kU];
#pragma unroll
            for (int v = 0; v < kU; ++v) {
                const int64_t k = k0 + v * 64 + lane;
                e[v] = k < b ? P.t_ids[k] : -1;
            }
            uint2 w[kU];
#pragma unroll
            for (int v = 0; v < kU; ++v) {
                const int ev = e[v] < 0 ? 0 : e[v];
                w[v] = T.br[static_cast<size_t>(ev >> kSrBits) * kSrWords + ((ev & (kSr - 1)) >> 5)];
            }
#pragma unroll
            for (int v = 0; v < kU; ++v) {
                if (e[v] < 0) continue;
                const int s = e[v] >> kSrBits;
                const uint32_t bit = static_cast<uint32_t>(e[v] & 31);
                if ((w[v].x >> bit) & 1u) {
                    const int g = hb[s] + static_cast<int>(w[v].y + __popc(w[v].x & ((1u << bit) - 1u)));
#pragma unroll
                    for (int c = 0; c < kMaxCot; ++c)
                        if (dl[c])
                            atomicAdd(reinterpret_cast<unsigned long long *>(&Wj[static_cast<size_t>(c) * P.catalog + g]), dl[c]);
                }
            }
        }
    }
}

struct BwdGrad {
    const float *loss;
    const uint32_t *present;
    int32_t catalog, words;
    const int32_t *elt_off, *elt_ids;
    const double *elt_terms, *layer_terms;
    const OccTables *tabs;
    const int64_t *W;              // [n_layers][n_cot][catalog] by hot index
    const int32_t *hot_base;       // [n_layers][n_sr + 1]
    const int32_t *hot_ev;         // [n_layers][catalog]
    int32_t n_sr, n_cot, n_cw, n_elt_slots;   // cw = (workgroup, wavefront) slots; slots = ELT positions of all layers
    const VScale *vs;
    double *part_elt;    // [n_cw][n_elt_slots][n_cot][3]
    double *part_occ;    // [n_layers][n_cw][n_cot][2]
};

constexpr int kGradThreads = 256;
constexpr int kGradWaves = kGradThreads / kWave;   // 4
constexpr int kGradHot = 4 * kGradThreads;         // hot events per workgroup
constexpr int kGradBatch = 4;                      // ELTs whose presence words and losses are loaded together

// (6) W(e) times the derivatives of O(e), over the layer's hot events
// (the only ones with W): workgroup i takes hot indices 1024 i .. 1024 i +
// 1023, each thread four of them.  Each wavefront reduces its lanes in a
// fixed tree and writes its own partials, so no workgroup barrier sits in
// the ELT loop and the final sums (a fixed order over workgroups and
// wavefronts) are deterministic.  Every per-row array is indexed by
// compile-time constants (rows beyond n_cot are zero), so nothing leaves
// registers.
__global__ __launch_bounds__(kGradThreads) void k_bwd_grad(BwdGrad P) {
    __shared__ int32_t lk[kMaxJ];
    __shared__ double ls[kMaxJ], lr[kMaxJ], ll[kMaxJ];
    const int hb = blockIdx.x, j = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t *hbase = P.hot_base + static_cast<size_t>(j) * (P.n_sr + 1);
    const int H = hbase[P.n_sr];
    const int g0 = hb * kGradHot;
    if (g0 >= H) return;   // uniform; the final sums read only the slots of workgroups with hot events
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
    const double occL = P.layer_terms[4 * j + 1];
    const OccTables T = P.tabs[j];
    const int32_t *hev = P.hot_ev + static_cast<size_t>(j) * P.catalog;

    // the thread's four hot events: weight per row and occurrence-clamp
    // branch.  O = min(max(x - OccR, 0), OccL) is non-zero for these events,
    // and it is below OccL exactly when the occurrence clamp is linear.
    double W[4][kMaxCot];
    bool lin_occ[4];
    int ev[4];
    double po[kMaxCot][2];
#pragma unroll
    for (int c = 0; c < kMaxCot; ++c) po[c][0] = po[c][1] = 0.0;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int g = g0 + it * kGradThreads + tid;
        const bool valid = g < H;
        const int e = valid ? hev[g] : 0;
        ev[it] = e;
        const int sr = e >> kSrBits;
        const double O = valid ? T.vals[static_cast<size_t>(sr) * kSr + (g - hbase[sr])] : 0.0;
        lin_occ[it] = valid && (O < occL);
#pragma unroll
        for (int c = 0; c < kMaxCot; ++c) {
            double wv = 0.0;
            if (valid && c < P.n_cot) {
                const int64_t acc = P.W[(static_cast<size_t>(j) * P.n_cot + c) * P.catalog + g];
                wv = ldexp(static_cast<double>(acc), -P.vs[j * P.n_cot + c].sigma);
            }
            W[it][c] = wv;
            if (valid) {
                if (lin_occ[it]) po[c][0] -= wv;
                else po[c][1] += wv;
            }
        }
    }
    const size_t cw = static_cast<size_t>(hb) * kGradWaves + w;   // (workgroup, wave) partial slot
    // occurrence-term partials of this wavefront
    // (wavefront sums by DPP: lane 63 holds the total, in a fixed order)
#pragma unroll
    for (int c = 0; c < kMaxCot; ++c)
        if (c < P.n_cot) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const double v = wave_inclusive_sum(po[c][m]);
                if (lane == 63)
                    P.part_occ[((static_cast<size_t>(j) * P.n_cw + cw) * P.n_cot + c) * 2 + m] = v;
            }
        }
    // ELT-term partials, kGradBatch ELTs' presence words and losses in flight at a time
    for (int q0 = 0; q0 < J; q0 += kGradBatch) {
        uint32_t pw[kGradBatch][4];
#pragma unroll
        for (int b = 0; b < kGradBatch; ++b) {
            const int qq = q0 + b;
#pragma unroll
            for (int it = 0; it < 4; ++it)
                pw[b][it] = (qq < J && lin_occ[it]) ? P.present[static_cast<size_t>(lk[qq]) * P.words + (ev[it] >> 5)] : 0u;
        }
        float lv[kGradBatch][4];
        bool on[kGradBatch][4];
#pragma unroll
        for (int b = 0; b < kGradBatch; ++b) {
            const int qq = q0 + b;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                on[b][it] = (pw[b][it] >> (ev[it] & 31)) & 1u;
                const size_t idx = on[b][it] ? static_cast<size_t>(lk[qq]) * P.catalog + ev[it] : 0;
                lv[b][it] = P.loss[idx];   // element 0 (always valid) for events without the ELT
            }
        }
#pragma unroll
        for (int b = 0; b < kGradBatch; ++b) {
            const int qq = q0 + b;
            if (qq >= J) break;
            double pe[kMaxCot][3];
#pragma unroll
            for (int c = 0; c < kMaxCot; ++c) pe[c][0] = pe[c][1] = pe[c][2] = 0.0;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                if (!on[b][it]) continue;
                const double l = static_cast<double>(lv[b][it]);
                const double scaled = ls[qq] * l;
                const double pre = scaled - lr[qq];
                const double av = (pre > 0.0) ? pre : 0.0;
                const bool lin = (pre > 0.0) && (av < ll[qq]);
                const bool cap = av >= ll[qq];
#pragma unroll
                for (int c = 0; c < kMaxCot; ++c) {
                    if (lin) {
                        pe[c][0] += W[it][c] * l;
                        pe[c][1] -= W[it][c];
                    }
                    if (cap) pe[c][2] += W[it][c];
                }
            }
            double *dst = P.part_elt + (cw * P.n_elt_slots + (a + qq)) * P.n_cot * 3;
#pragma unroll
            for (int c = 0; c < kMaxCot; ++c)
                if (c < P.n_cot) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const double v = wave_inclusive_sum(pe[c][m]);
                        if (lane == 63) dst[c * 3 + m] = v;
                    }
                }
        }
    }
}

// Partial slots written for layer j: those of the workgroups that had hot events.
__device__ __forceinline__ int grad_slots_used(const int32_t *hot_base, int n_sr, int j, int n_cw) {
    const int H = hot_base[static_cast<size_t>(j) * (n_sr + 1) + n_sr];
    return min(n_cw, ((H + kGradHot - 1) / kGradHot) * kGradWaves);
}

// (7) fixed-order sums into the outputs: one workgroup per output value,
// each thread a fixed stride of the (chunk, wavefront) partials, then a
// fixed-order tree.
__global__ __launch_bounds__(256) void k_bwd_final(const int32_t *__restrict__ elt_off, const int32_t *__restrict__ elt_ids,
                                                  int n_layers, int n_elts, int n_cot, int n_cw,
                                                  const int32_t *__restrict__ hot_base, int n_sr, int n_elt_slots,
                                                  int nwg_v, const double *__restrict__ part_elt,
                                                  const double *__restrict__ part_occ,
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
                const int used = grad_slots_used(hot_base, n_sr, j, n_cw);
                for (int cw = tid; cw < used; cw += blockDim.x)
                    v += part_elt[((static_cast<size_t>(cw) * n_elt_slots + q) * n_cot + c) * 3 + m];
            }
    } else {
        const int i = o - n_e;
        const int c = i / (n_layers * 4), j = (i / 4) % n_layers, m = i % 4;
        if (m < 2) {
            const int used = grad_slots_used(hot_base, n_sr, j, n_cw);
            for (int cw = tid; cw < used; cw += blockDim.x)
                v += part_occ[((static_cast<size_t>(j) * n_cw + cw) * n_cot + c) * 2 + m];
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
    int nwg_v, n_cw, cs;
    size_t bytes;
};

static int bwd_nwg_v(int64_t n) {   // about two trials per thread, at most 512 workgroups
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 2047) / 2048, 512)));
}

static int64_t dev_blocks(int64_t n) { return std::max<int64_t>(1, (n + kDevChunk - 1) / kDevChunk); }

static int bwd_cs(int n_cot) { return n_cot <= 1 ? 1 : (n_cot <= 2 ? 2 : 4); }

static BwdLayout bwd_layout(const ara_tables *tables, const ara_layers *layers, int n_cot, int64_t n) {
    BwdLayout B{};
    B.z = occ_sizes(tables->catalog, false);
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    B.nwg_v = bwd_nwg_v(n);
    B.n_cw = static_cast<int>((static_cast<int64_t>(tables->catalog) + kGradHot - 1) / kGradHot) * kGradWaves;
    B.cs = bwd_cs(n_cot);
    const size_t cat = static_cast<size_t>(tables->catalog);
    Carver c(nullptr);
    c.take<int32_t>(kWsHeaderBytes / 4);
    c.take<int32_t>(static_cast<size_t>(L + 1));
    c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    c.take<OccTables>(static_cast<size_t>(std::max(L, 1)));
    size_t b = c.bytes() + static_cast<size_t>(L) * B.z.per_layer;
    Carver d(nullptr);
    d.take<VScale>(static_cast<size_t>(std::max(L * n_cot, 1)));
    d.take<unsigned long long>(static_cast<size_t>(std::max(L, 1)));
    d.take<int64_t>(static_cast<size_t>(std::max(L, 1)) * kMaxCot);
    d.take<int32_t>(static_cast<size_t>(L) * std::max<int64_t>(n, 1));
    d.take<double>(static_cast<size_t>(L) * n_cot * B.nwg_v * 2);
    d.take<int64_t>(static_cast<size_t>(L) * std::max<int64_t>(n, 1) * B.cs);
    d.take<int32_t>(static_cast<size_t>(L) * cat);
    d.take<int32_t>(static_cast<size_t>(L) * (B.z.n_sr + 1));
    d.take<int64_t>(static_cast<size_t>(L) * n_cot * cat);
    d.take<double>(static_cast<size_t>(B.n_cw) * std::max(nJ, 1) * n_cot * 3);
    d.take<double>(static_cast<size_t>(L) * B.n_cw * n_cot * 2);
    B.bytes = b + d.bytes();
    return B;
}

static int32_t check_pair_b(const ara_tables *tables, const ara_yet *yet) {
    if (!tables || !yet) return fail(ARA_E_INVAL, "null tables or yet");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (yet->range_bits != kRangeBits || yet->groups != kGroups) return fail(ARA_E_INVAL, "YET not prepared by this library");
    if (yet->n_slices != kSlices || !yet->tr_off || (yet->nnz > 0 && !yet->tr_ent))
        return fail(ARA_E_INVAL, "the backward needs a YET prepared with ARA_PREP_TRANSPOSED");
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
    *bytes = bwd_layout(tables, layers, n_cot, yet->n_trials).bytes;
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
    const BwdLayout B = bwd_layout(tables, layers, n_cot, yet->n_trials);
    if (ws_bytes < B.bytes) return fail(ARA_E_NOSPACE, "backward workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L == 0 || n == 0) {
        ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
        ARA_HIP(hipMemsetAsync(grad_elt, 0, static_cast<size_t>(n_cot) * tables->n_elts * 3 * sizeof(double), st));
        if (L > 0) ARA_HIP(hipMemsetAsync(grad_layer, 0, static_cast<size_t>(n_cot) * L * 4 * sizeof(double), st));
        return ARA_OK;
    }
    // otherwise every output value is written by the final reduction

    const int nJ = layers->elt_off[L];
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / 4);
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    VScale *vs = c.take<VScale>(static_cast<size_t>(L * n_cot));
    unsigned long long *ndev = c.take<unsigned long long>(static_cast<size_t>(L));
    int64_t *common = c.take<int64_t>(static_cast<size_t>(L) * kMaxCot);
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, B.z, false);
    double *aggpart = c.take<double>(static_cast<size_t>(L) * n_cot * bwd_nwg_v(n) * 2);
    int64_t *vq = c.take<int64_t>(static_cast<size_t>(L) * n * B.cs);
    int32_t *hot_ev = c.take<int32_t>(static_cast<size_t>(L) * tables->catalog);
    int32_t *hot_base = c.take<int32_t>(static_cast<size_t>(L) * (B.z.n_sr + 1));
    int64_t *W = c.take<int64_t>(static_cast<size_t>(L) * n_cot * tables->catalog);
    double *part_elt = c.take<double>(static_cast<size_t>(B.n_cw) * std::max(nJ, 1) * n_cot * 3);
    double *part_occ = c.take<double>(static_cast<size_t>(L) * B.n_cw * n_cot * 2);
    int32_t *dev = c.take<int32_t>(static_cast<size_t>(L) * std::max<int64_t>(n, 1));
    HeadImage img(ws);   // clears the error header, the weight scales and the deviating-trial counts
    img.put(d_off, layers->elt_off, static_cast<size_t>(L + 1));
    img.put(d_ids, layers->elt_ids, static_cast<size_t>(nJ));
    img.put(d_tabs, tabs.data(), tabs.size());
    img.cover(ndev + L);
    if ((rc = img.send(st))) return rc;

    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, false, false, d_tabs, B.z.n_sr, d_err, st)))
            return rc;
    }
    const int nwg_v = bwd_nwg_v(n);
    {
        ProfScope prof(ARA_PROF_BWD_RED, st);
        k_bwd_vmax<<<dim3(nwg_v, L), kBwdThreads, 0, st>>>(grad_ylt, s_pre, layer_terms, n, L, n_cot, nwg_v, vs, aggpart);
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 2048));
        k_bwd_vq<<<dim3(gx, L), 256, 0, st>>>(grad_ylt, s_pre, layer_terms, n, L, n_cot, B.cs, yet->max_occ, vs, vq);
        k_bwd_hot<<<dim3(B.z.n_sr, L), 256, 0, st>>>(d_tabs, B.z.n_sr, n_cot, tables->catalog, hot_ev, hot_base, W);
        ARA_HIP(hipGetLastError());
    }
    BwdGather S{};
    S.tr_off = yet->tr_off;
    S.tr_ent = yet->tr_ent;
    S.catalog = tables->catalog;
    S.n_sr = B.z.n_sr;
    S.n_cot = n_cot;
    S.slice_trials = yet->slice_trials;
    S.t0 = trial_begin;
    S.t1 = trial_end;
    S.n = n;
    S.hot_ev = hot_ev;
    S.hot_base = hot_base;
    S.vq = vq;
    S.W = W;
    // the second form of step (5) needs the trial-major copy
    BwdSparse &Q = S.sp;
    // (the list of deviating trials holds call-relative int32 indices)
    S.use_sp = yet->t_off != nullptr && yet->t_ids != nullptr && yet->t_cnt != nullptr && n < (int64_t(1) << 31);
    Q.vq = vq;
    Q.n = n;
    Q.t0 = trial_begin;
    Q.n_trials = yet->n_trials;
    Q.cs = B.cs;
    Q.n_cot = n_cot;
    Q.catalog = tables->catalog;
    Q.n_sr = B.z.n_sr;
    Q.slice_trials = yet->slice_trials;
    Q.tr_off = yet->tr_off;
    Q.tr_ent = yet->tr_ent;
    Q.ndev = ndev;
    Q.common = common;
    Q.dev = dev;
    Q.t_cnt = yet->t_cnt;
    Q.t_off = yet->t_off;
    Q.t_ids = yet->t_ids;
    Q.tabs = d_tabs;
    Q.hot_ev = hot_ev;
    Q.hot_base = hot_base;
    Q.W = W;
    {
        ProfScope prof(ARA_PROF_BWD, st);
        // four 256-thread workgroups per CU, a multiple of the slice count
        const int cu = device_cu_count();
        const unsigned gx = static_cast<unsigned>(kSlices * std::max(1, (4 * cu) / kSlices));
        const dim3 grid(gx, L);
        // lanes per hot event: about a third of the mean list length, 4 or 16
        const double mean_list = static_cast<double>(yet->nnz) / (static_cast<double>(kSlices) * tables->catalog);
        const bool wide = mean_list >= 24.0;
        if (S.use_sp) {
            const unsigned gt = static_cast<unsigned>(dev_blocks(n));
            k_bwd_pick<<<L, kPickSamples, 0, st>>>(Q);
            k_bwd_dev<<<dim3(gt, L), 1024, 0, st>>>(Q);
            const unsigned gh = static_cast<unsigned>(std::min<int64_t>((tables->catalog + 255) / 256, 1024));
            k_bwd_winit<<<dim3(gh, L), 256, 0, st>>>(Q);
            // the slices the range cuts: at most its first and its last
            int cut[2], ncut = 0;
            for (int64_t t : {trial_begin, trial_end - 1}) {
                const int x = static_cast<int>(t / yet->slice_trials);
                const int64_t lo = static_cast<int64_t>(x) * yet->slice_trials;
                const int64_t hi = std::min(lo + yet->slice_trials, yet->n_trials);
                const bool inside = lo >= trial_begin && hi <= trial_end;
                if (n > 0 && !inside && (ncut == 0 || cut[0] != x)) cut[ncut++] = x;
            }
            if (ncut > 0) {
                const dim3 gc(static_cast<unsigned>(ncut * std::max(1, (4 * cu) / ncut)), L);
                const int2 cx = make_int2(cut[0], ncut > 1 ? cut[1] : cut[0]);
                if (wide) k_bwd_wcut<16><<<gc, 256, 0, st>>>(Q, cx, ncut);
                else k_bwd_wcut<4><<<gc, 256, 0, st>>>(Q, cx, ncut);
            }
            k_bwd_wsparse<<<dim3(2048, L), 256, 0, st>>>(Q);
        }
        if (wide) launch_bwd_w<16>(B.cs, grid, st, S);
        else launch_bwd_w<4>(B.cs, grid, st, S);
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
    Gp.W = W;
    Gp.hot_base = hot_base;
    Gp.n_sr = B.z.n_sr;
    Gp.n_cot = n_cot;
    Gp.n_cw = B.n_cw;
    Gp.hot_ev = hot_ev;
    Gp.n_elt_slots = std::max(nJ, 1);
    Gp.vs = vs;
    Gp.part_elt = part_elt;
    Gp.part_occ = part_occ;
    {
        ProfScope prof(ARA_PROF_BWD_RED, st);
        k_bwd_grad<<<dim3(B.n_cw / kGradWaves, L), kGradThreads, 0, st>>>(Gp);
        const int outs = n_cot * tables->n_elts * 3 + n_cot * L * 4;
        k_bwd_final<<<outs, 256, 0, st>>>(d_off, d_ids, L, tables->n_elts, n_cot, B.n_cw, hot_base, B.z.n_sr,
                                          std::max(nJ, 1), nwg_v, part_elt, part_occ, aggpart, grad_elt, grad_layer);
        ARA_HIP(hipGetLastError());
    }
    return ARA_OK;
}
