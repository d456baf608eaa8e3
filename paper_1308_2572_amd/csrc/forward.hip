// Forward: stream the prepared YET, gather each occurrence's O(e) from the
// occurrence table held in LDS, accumulate per trial, apply the aggregate
// terms (Algorithm 1, steps three and four).
//
// One workgroup per block of trials; wavefront g owns trial group g of the
// block.  The per-trial totals live in LDS for the whole pass over the
// catalogue (one super-range table at a time), so each trial's total is
// accumulated by a single wavefront in a fixed order: deterministic.
#include "occ.h"

#include <algorithm>
#include <string>

namespace ara {

constexpr int kUnroll = 16;
constexpr int kLdsBytes = 160 * 1024;

struct FwdParams {
    const uint32_t *ent;
    const int64_t *seg_base;
    const int32_t *seg_run;
    int64_t n_trials;
    int32_t tg, tb, n_ranges, n_sr;
    int32_t cap;               // values held in LDS per super-range
    const FwdItem *items;      // one (layer, block of trials) per workgroup
};

__device__ __forceinline__ uint32_t ld_stream(const uint32_t *p) { return __builtin_nontemporal_load(p); }

// LDS bytes before the values: per-trial totals (and hit counts) including
// the padding slot, then the super-range's bitmap words with ranks.
__host__ __device__ inline size_t fwd_fixed_lds(int tb, bool hits) {
    return align256(static_cast<size_t>(tb + 1) * 8 + (hits ? static_cast<size_t>(tb + 1) * 4 : 0)) +
           kSrWords * sizeof(uint2);
}

template <bool HITS>
__global__ __launch_bounds__(1024) void k_fwd(FwdParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tb = P.tb;
    double *acc = reinterpret_cast<double *>(smem);                                     // [tb + 1]
    int32_t *hacc = reinterpret_cast<int32_t *>(smem + static_cast<size_t>(tb + 1) * 8);   // [tb + 1]
    const size_t tbr_off = fwd_fixed_lds(tb, HITS) - kSrWords * sizeof(uint2);
    uint2 *tbr = reinterpret_cast<uint2 *>(smem + tbr_off);
    double *tvals = reinterpret_cast<double *>(smem + tbr_off + kSrWords * sizeof(uint2));
    uint8_t *tcnt = reinterpret_cast<uint8_t *>(tvals + P.cap);

    const FwdItem I = P.items[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b = I.block;
    const uint32_t pad = pad_entry(tb);
    const int64_t gt0 = b * tb + static_cast<int64_t>(w) * P.tg;
    const int64_t gt1 = min(gt0 + P.tg, P.n_trials);
    const bool active = gt0 < gt1 && gt1 > I.t0 && gt0 < I.t1;
    const int G = P.n_ranges;
    const size_t seg0 = static_cast<size_t>(b) * G * kGroups + w;

    for (int i = tid; i <= tb; i += blockDim.x) {   // slot tb collects the padding
        acc[i] = 0.0;
        if (HITS) hacc[i] = 0;
    }
    const OccTables T = *I.tab;

    // stream cursor over this wave's segments (range rr, step within it)
    int rr = active ? 0 : G, step = 0, R = 0;
    int64_t sb = 0;
    auto seek = [&]() {
        while (rr < G) {
            const size_t si = seg0 + static_cast<size_t>(rr) * kGroups;
            R = P.seg_run[si];
            sb = P.seg_base[si];
            if (R > 0) break;
            ++rr;
        }
    };
    uint32_t X[kUnroll];
    int chunk_rr = G;
    auto load = [&]() {
        chunk_rr = rr;
        if (rr < G) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                X[u] = (step + u < R) ? ld_stream(P.ent + sb + static_cast<int64_t>(step + u) * kWave + lane) : pad;
            step += kUnroll;
            if (step >= R) {
                ++rr;
                step = 0;
                seek();
            }
        }
    };
    seek();
    load();

    for (int s = 0; s < P.n_sr; ++s) {
        __syncthreads();
        const int cnt_s = T.count[s];
        const int inl = min(cnt_s, P.cap);
        const uint2 *gbr = T.br + static_cast<size_t>(s) * kSrWords;
        const double *gvals = T.vals + static_cast<size_t>(s) * kSr;
        const uint8_t *gcnt = HITS ? T.cnt + static_cast<size_t>(s) * kSr : nullptr;
        for (int i = tid; i < kSrWords; i += blockDim.x) tbr[i] = gbr[i];
        for (int i = tid; i < inl; i += blockDim.x) tvals[i] = gvals[i];
        if (HITS)
            for (int i = tid; i < inl; i += blockDim.x) tcnt[i] = gcnt[i];
        __syncthreads();
        const int rr_end = min(2 * s + 2, G);
        const bool all_lds = cnt_s <= P.cap;     // uniform over the workgroup
        while (chunk_rr < rr_end) {
            uint32_t Y[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) Y[u] = X[u];
            const uint32_t hb = static_cast<uint32_t>(chunk_rr & 1) << kRangeBits;
            load();   // prefetch the next chunk (possibly of the next super-range)
            // lookups first, without branches, so the LDS reads of all
            // entries are in flight together; then the masked accumulation
            uint2 q[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) q[u] = tbr[(hb | (Y[u] & (kRange - 1))) >> 5];
            uint32_t rank[kUnroll];
            bool hit[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t bit = Y[u] & 31;
                hit[u] = (q[u].x >> bit) & 1u;
                rank[u] = q[u].y + __popc(q[u].x & ((1u << bit) - 1u));
            }
            if (all_lds) {
                double v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) v[u] = tvals[hit[u] ? rank[u] : 0];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (hit[u]) {
                        atomicAdd(&acc[Y[u] >> kRangeBits], v[u]);
                        if (HITS) atomicAdd(&hacc[Y[u] >> kRangeBits], static_cast<int>(tcnt[rank[u]]));
                    }
            } else {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (hit[u]) {
                        const bool in = rank[u] < static_cast<uint32_t>(P.cap);
                        double v;
                        int c = 0;
                        if (in) {
                            v = tvals[rank[u]];
                            if (HITS) c = tcnt[rank[u]];
                        } else {
                            v = gvals[rank[u]];
                            if (HITS) c = gcnt[rank[u]];
                        }
                        atomicAdd(&acc[Y[u] >> kRangeBits], v);
                        if (HITS) atomicAdd(&hacc[Y[u] >> kRangeBits], c);
                    }
            }
        }
    }
    __syncthreads();
    if (active) {
        const double aggR = I.lterm[2], aggL = I.lterm[3];
        const int64_t lo = max(gt0, I.t0), hi = min(gt1, I.t1);
        for (int64_t t = lo + lane; t < hi; t += kWave) {
            const int i = static_cast<int>(t - b * tb);
            const double S = acc[i];
            const size_t o = static_cast<size_t>(t - I.t0);
            I.ylt[o] = xl(S, aggR, aggL);
            if (I.s_pre) I.s_pre[o] = S;
            if (HITS && I.hits) I.hits[o] = hacc[i];
        }
    }
}

int32_t launch_forward(const ara_yet *yet, int n_sr, bool hits, const FwdItem *d_items, int n_items, hipStream_t st) {
    if (n_items <= 0) return ARA_OK;
    FwdParams P{};
    P.ent = yet->ent;
    P.seg_base = yet->seg_base;
    P.seg_run = yet->seg_run;
    P.n_trials = yet->n_trials;
    P.tg = yet->trials_per_group;
    P.tb = yet->trials_per_block;
    P.n_ranges = yet->n_ranges;
    P.n_sr = n_sr;
    const size_t fixed = fwd_fixed_lds(P.tb, hits);
    P.cap = static_cast<int32_t>((kLdsBytes - fixed) / (hits ? 9 : 8));
    P.items = d_items;
    ProfScope prof(ARA_PROF_FWD, st);
    if (hits) {
        static bool attr = false;
        if (!attr) {
            ARA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd<true>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes));
            attr = true;
        }
        k_fwd<true><<<n_items, 1024, kLdsBytes, st>>>(P);
    } else {
        static bool attr = false;
        if (!attr) {
            ARA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fwd<false>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes));
            attr = true;
        }
        k_fwd<false><<<n_items, 1024, kLdsBytes, st>>>(P);
    }
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

static size_t fwd_workspace(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, bool hits) {
    const OccLayoutSizes z = occ_sizes(tables->catalog, hits);
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    size_t b = kWsHeaderBytes;
    b += align256(static_cast<size_t>(L + 1) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(nJ, 1)) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(L, 1)) * sizeof(OccTables));
    b += align256(static_cast<size_t>(std::max(L, 1)) * std::max(yet->n_blocks, 1) * sizeof(FwdItem));
    b += static_cast<size_t>(L) * z.per_layer;
    return b;
}

static int32_t check_pair(const ara_tables *tables, const ara_yet *yet) {
    if (!tables || !yet) return fail(ARA_E_INVAL, "null tables or yet");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (yet->range_bits != kRangeBits || yet->groups != kGroups) return fail(ARA_E_INVAL, "YET not prepared by this library");
    return ARA_OK;
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_ylt_workspace_bytes(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                           uint32_t flags, size_t *bytes) {
    if (!bytes) return fail(ARA_E_INVAL, "null output");
    int32_t rc = check_pair(tables, yet);
    if (rc) return rc;
    if ((rc = check_layers(layers, tables->n_elts))) return rc;
    if (flags & ~ARA_F_EMIT_HITS) return fail(ARA_E_INVAL, "unknown flag");
    *bytes = fwd_workspace(tables, yet, layers, (flags & ARA_F_EMIT_HITS) != 0);
    return ARA_OK;
}

extern "C" int32_t ara_ylt_forward(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                   const double *elt_terms, const double *layer_terms, int64_t trial_begin,
                                   int64_t trial_end, uint32_t flags, double *ylt, double *s_pre, int32_t *hits,
                                   void *ws, size_t ws_bytes, void *stream) {
    int32_t rc = check_pair(tables, yet);
    if (rc) return rc;
    if ((rc = check_layers(layers, tables->n_elts))) return rc;
    if (flags & ~ARA_F_EMIT_HITS) return fail(ARA_E_INVAL, "unknown flag");
    const bool want_hits = (flags & ARA_F_EMIT_HITS) != 0;
    if (hits && !want_hits) return fail(ARA_E_INVAL, "hits output requires ARA_F_EMIT_HITS");
    if (trial_begin < 0 || trial_end < trial_begin || trial_end > yet->n_trials)
        return fail(ARA_E_RANGE, "trial range outside the YET");
    if (!ws) return fail(ARA_E_INVAL, "null workspace");
    const int L = layers->n_layers;
    const int64_t n = trial_end - trial_begin;
    if (L > 0 && n > 0 && (!ylt || !elt_terms || !layer_terms)) return fail(ARA_E_INVAL, "null output or terms");
    if (ws_bytes < fwd_workspace(tables, yet, layers, want_hits)) return fail(ARA_E_NOSPACE, "forward workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
    if (L == 0 || n == 0) return ARA_OK;

    const OccLayoutSizes z = occ_sizes(tables->catalog, want_hits);
    const int nJ = layers->elt_off[L];
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / sizeof(int32_t));
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    const int64_t b_lo = trial_begin / yet->trials_per_block;
    const int64_t b_hi = (trial_end + yet->trials_per_block - 1) / yet->trials_per_block;
    const int nb = static_cast<int>(b_hi - b_lo);
    FwdItem *d_items = c.take<FwdItem>(static_cast<size_t>(L) * std::max(yet->n_blocks, 1));
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, z, want_hits);
    std::vector<FwdItem> items(static_cast<size_t>(L) * nb);
    for (int j = 0; j < L; ++j)
        for (int i = 0; i < nb; ++i) {
            FwdItem &it = items[static_cast<size_t>(j) * nb + i];
            it.tab = d_tabs + j;
            it.lterm = layer_terms + 4 * j;
            it.block = static_cast<int32_t>(b_lo + i);
            it.t0 = trial_begin;
            it.t1 = trial_end;
            it.ylt = ylt + static_cast<size_t>(j) * n;
            it.s_pre = s_pre ? s_pre + static_cast<size_t>(j) * n : nullptr;
            it.hits = hits ? hits + static_cast<size_t>(j) * n : nullptr;
        }
    ARA_HIP(hipMemcpyAsync(d_off, layers->elt_off, (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (nJ > 0) ARA_HIP(hipMemcpyAsync(d_ids, layers->elt_ids, nJ * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(d_tabs, tabs.data(), L * sizeof(OccTables), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(FwdItem), hipMemcpyHostToDevice, st));

    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, want_hits, d_tabs, z.n_sr, d_err, st)))
            return rc;
    }
    return launch_forward(yet, z.n_sr, want_hits, d_items, L * nb, st);
}
