// Forward: stream the prepared YET (16-bit codes), gather each occurrence's
// O(e) from the occurrence table held in LDS, accumulate per trial, apply
// the aggregate terms (Algorithm 1, steps three and four).
//
// One workgroup per block of trials; wavefront g owns trial group g of the
// block.  The per-trial totals live in LDS for the whole pass over the
// catalogue, so each trial's total is accumulated by a single wavefront in a
// fixed order: deterministic.  The catalogue is walked one range (2^15
// events) at a time; the range's slice of the occurrence table (bitmap words
// with ranks, then the values) is copied into LDS by LDS DMA
// (global_load_lds_dwordx4).  A workgroup takes 80 KB of LDS and at most 64
// registers per lane, so two workgroups share a CU (8 wavefronts per SIMD):
// while one waits for its next table slice the other streams.
#include "occ.h"

#include <algorithm>
#include <string>
#include <type_traits>

namespace ara {

constexpr int kUnroll = 8;
constexpr int kLdsBytes = 80 * 1024;
constexpr int kBrBytes = 1024 * static_cast<int>(sizeof(uint2));   // one range's bitmap words with ranks

struct FwdParams {
    const uint16_t *code;
    const uint16_t *pad;       // kPadCodes skip codes
    const int64_t *seg_base;
    const int32_t *seg_run;
    const uint8_t *lane_start;
    int64_t n_trials;
    int32_t tg, tb, n_ranges;
    int32_t capv;              // values per range buffer
    int32_t buf_bytes;         // bytes per range buffer
    const FwdItem *items;      // one (layer, block of trials) per workgroup, or null: then the
                               // workgroups take the regular set below (fwd_item)
    const OccTables *reg_tabs;
    const double *reg_lterm;
    double *reg_ylt, *reg_s_pre;
    int32_t *reg_hits;
    int64_t reg_t0, reg_t1;
    int32_t reg_b0, reg_nb;
    int32_t reg_nl;            // layers of the regular set
};

// Workgroup i's item: from the list, or formed from the regular set.  With
// one layer, workgroup i takes block reg_b0 + i.  With several, the layers
// of one block go to the same XCD one after another (workgroups are dealt to
// the eight XCDs round-robin by index): workgroup i = 8k + x is the k-th on
// XCD x and takes layer k % L of block 8 (k / L) + x, so the L workgroups
// that stream the same codes run together under one L2 and the codes come
// from HBM once.  Indexes past the last block give an empty item (block -1).
__device__ __forceinline__ FwdItem fwd_item(const FwdParams &P, int i) {
    if (P.items) return P.items[i];
    FwdItem it;
    int j = 0, bi = i;
    if (P.reg_nl > 1) {
        const int x = i & (kXcds - 1), k = i / kXcds;
        j = k % P.reg_nl;
        bi = (k / P.reg_nl) * kXcds + x;
    }
    const size_t n = static_cast<size_t>(P.reg_t1 - P.reg_t0);
    it.tab = P.reg_tabs + j;
    it.lterm = P.reg_lterm + 4 * j;
    it.block = bi < P.reg_nb ? P.reg_b0 + bi : -1;
    it.pad = 0;
    it.t0 = P.reg_t0;
    it.t1 = P.reg_t1;
    it.ylt = P.reg_ylt + static_cast<size_t>(j) * n;
    it.s_pre = P.reg_s_pre ? P.reg_s_pre + static_cast<size_t>(j) * n : nullptr;
    it.hits = P.reg_hits ? P.reg_hits + static_cast<size_t>(j) * n : nullptr;
    return it;
}

// Four consecutive codes of one lane: streamed past the cache when this
// workgroup is the only reader of its block's codes; kept in L2 when the
// workgroups of the block's other layers (or quotes) read them too.
template <bool SHARED>
__device__ __forceinline__ unsigned long long ld_codes(const uint16_t *p) {
    if (SHARED) return *reinterpret_cast<const unsigned long long *>(p);
    return __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
}

// 16 bytes per lane from global memory straight into LDS at lds_base + 16 *
// lane (lds_base uniform over the wavefront).  Issued as inline assembly so
// that the compiler does not make the next LDS reads wait for it: the
// kernel waits for these copies itself (vmcnt(0) before the barrier that
// publishes the buffer).  The wait counts the compiler computes for its own
// loads stay sufficient, since an extra outstanding load only makes them
// stricter.
__device__ __forceinline__ void lds_dma16(const void *src, uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_base)), "v"(src)
                 : "memory", "m0");
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// a + (bit POS of x << SH): two instructions.  Written out because the
// optimiser otherwise turns it into shift, mask and add, or re-derives every
// address of a chain from a running count (three instructions either way).
template <int POS, int SH>
__device__ __forceinline__ uint32_t add_bit(uint32_t a, uint32_t x) {
    uint32_t b, r;
    asm("v_bfe_u32 %0, %1, %2, 1" : "=v"(b) : "v"(x), "n"(POS));
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "n"(SH), "v"(a));
    return r;
}

// LDS bytes of the per-trial totals (binary64, or binary32 when
// accumulating in binary32) and hit counts, including the padding slot; the
// table counts of every range; each wavefront's window of 64 segment
// descriptors (run length, base) -- descriptors come from LDS so that moving
// to the next range never waits on the vector memory counter, which also
// counts the prefetched stream.
__host__ __device__ inline size_t fwd_acc_lds(int tb, bool hits, size_t vbytes) {
    return align256(static_cast<size_t>(tb + 1) * vbytes + (hits ? static_cast<size_t>(tb + 1) * 4 : 0));
}
__host__ __device__ inline size_t fwd_meta_lds(int n_ranges) {
    return align256(static_cast<size_t>(n_ranges) * 8) + align256(static_cast<size_t>(kGroups) * kWave * 12);
}

// Range r of the catalogue is half (r & 1) of occurrence-table super-range
// r >> 1; its set events have super-range ranks [base, base + cnt).
struct RangeInfo {
    uint32_t base, cnt;
};

// F32: occurrence values are binary32 in the table and trial totals are
// accumulated in binary32 (the aggregate terms are still applied in
// binary64); otherwise both are binary64.
// SHARED: several workgroups of the launch stream the same block's codes.
template <bool HITS, bool F32, bool SHARED>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_fwd(FwdParams P) {
    using V = typename std::conditional<F32, float, double>::type;
    // codes per lane and chunk: half as many with hit counts, whose extra
    // per-code state would not fit the registers of eight codes
    constexpr int kUn = HITS ? kUnroll / 2 : kUnroll;
    constexpr uint32_t kV = sizeof(V);             // bytes per value and per trial total
    constexpr int kVSh = F32 ? 2 : 3;              // log2(kV)
    constexpr uint32_t kVPer16 = 16 / kV;          // values per 16-byte copy
    // LDS: [range buffer][trial totals][hit counts][range table][segment windows].
    // A static array: its addresses are compile-time constants, which the LDS
    // instructions take as immediate offsets.
    __shared__ __align__(16) unsigned char smem[kLdsBytes];
    const int tb = P.tb;
    const uint32_t acc_off = static_cast<uint32_t>(P.buf_bytes);
    const uint32_t hacc_off = acc_off + static_cast<uint32_t>(tb + 1) * kV;
    V *acc = reinterpret_cast<V *>(smem + acc_off);                // [tb + 1]
    int32_t *hacc = reinterpret_cast<int32_t *>(smem + hacc_off);  // [tb + 1]
    const int G = P.n_ranges;
    unsigned char *meta = smem + acc_off + fwd_acc_lds(tb, HITS, kV);
    uint2 *rinfo = reinterpret_cast<uint2 *>(meta);                                             // [G] (base, cnt)
    unsigned char *meta2 = meta + align256(static_cast<size_t>(G) * 8);
    int64_t *wbase_all = reinterpret_cast<int64_t *>(meta2);                                    // [16][64]
    int32_t *wrun_all = reinterpret_cast<int32_t *>(meta2 + kGroups * kWave * 8);               // [16][64]
    unsigned char *bufs = smem;
    const uint32_t bufs_lds = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(bufs));

    const FwdItem I = fwd_item(P, blockIdx.x);
    if (I.block < 0) return;   // uniform over the workgroup, before any barrier
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b = I.block;
    const int64_t gt0 = b * tb + static_cast<int64_t>(w) * P.tg;
    const int64_t gt1 = min(gt0 + P.tg, P.n_trials);
    const bool active = gt0 < gt1 && gt1 > I.t0 && gt0 < I.t1;
    const size_t seg0 = static_cast<size_t>(b) * G * kGroups + w;

    for (int i = tid; i <= tb; i += blockDim.x) {   // slot tb collects the padding
        acc[i] = V(0);
        if (HITS) hacc[i] = 0;
    }
    const OccTables T = *I.tab;

    // copy range r's table slice into LDS, split over the wavefronts
    auto fetch = [&](int r, RangeInfo ri) {
        const uint32_t dst = bufs_lds;
        const size_t s = static_cast<size_t>(r >> 1);
        const unsigned char *gbr = reinterpret_cast<const unsigned char *>(T.br + s * kSrWords + (r & 1) * 1024);
        for (int c0 = w * kWave; c0 < kBrBytes / 16; c0 += kGroups * kWave)
            lds_dma16(gbr + static_cast<size_t>(c0 + lane) * 16, dst + c0 * 16);
        const uint32_t nv = min(ri.cnt + (ri.base & (kVPer16 - 1u)), static_cast<uint32_t>(P.capv));
        const int nvc = static_cast<int>((nv + kVPer16 - 1u) / kVPer16);
        const unsigned char *gv =
            reinterpret_cast<const unsigned char *>(reinterpret_cast<const V *>(T.vals) + s * kSr + (ri.base & ~(kVPer16 - 1u)));
        for (int c0 = w * kWave; c0 < nvc; c0 += kGroups * kWave)
            if (c0 + lane < nvc) lds_dma16(gv + static_cast<size_t>(c0 + lane) * 16, dst + kBrBytes + c0 * 16);
        if (HITS) {
            const uint32_t nb = min(ri.cnt + (ri.base & 15u), static_cast<uint32_t>(P.capv));
            const int nbc = static_cast<int>((nb + 15) / 16);
            const unsigned char *gc = T.cnt + s * kSr + (ri.base & ~15u);
            const uint32_t cdst = dst + kBrBytes + static_cast<uint32_t>(P.capv) * kV;
            for (int c0 = w * kWave; c0 < nbc; c0 += kGroups * kWave)
                if (c0 + lane < nbc) lds_dma16(gc + static_cast<size_t>(c0 + lane) * 16, cdst + c0 * 16);
        }
    };

    for (int r = tid; r < G; r += blockDim.x) {
        const size_t sr = static_cast<size_t>(r >> 1);
        const uint32_t mid = T.br[sr * kSrWords + 1024].y;
        const uint32_t tot = static_cast<uint32_t>(T.count[sr]);
        rinfo[r] = (r & 1) ? make_uint2(mid, tot - mid) : make_uint2(0u, mid);
    }
    auto range_info = [&](int r) {   // uniform
        const uint2 v = rinfo[r];
        RangeInfo ri;
        ri.base = __builtin_amdgcn_readfirstlane(v.x);
        ri.cnt = __builtin_amdgcn_readfirstlane(v.y);
        return ri;
    };

    // stream cursor over this wave's segments (range rr, step within it); the
    // descriptors of 64 consecutive ranges are staged in this wave's LDS window
    int64_t *wbase = wbase_all + w * kWave;
    int32_t *wrun = wrun_all + w * kWave;
    int seg_win = -kWave;
    uint64_t nonempty = 0;
    int rr = active ? 0 : G, step = 0, R = 0;
    int64_t sb = 0;
    auto seek = [&]() {   // first range >= rr in which this wave has entries
        while (rr < G) {
            if (rr >= seg_win + kWave) {
                seg_win = rr & ~(kWave - 1);
                const int r = seg_win + lane;
                int32_t run = 0;
                int64_t base = 0;
                if (r < G) {
                    const size_t si = seg0 + static_cast<size_t>(r) * kGroups;
                    run = P.seg_run[si];
                    base = P.seg_base[si];
                }
                wrun[lane] = run;
                wbase[lane] = base;
                nonempty = __ballot(run > 0);
            }
            const uint64_t m = nonempty & (~0ull << (rr - seg_win));
            if (m) {
                const int l = __builtin_ctzll(m);
                rr = seg_win + l;
                R = __builtin_amdgcn_readfirstlane(wrun[l]);
                const int64_t bv = wbase[l];
                sb = static_cast<int64_t>(
                    (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(bv) >> 32))) << 32) |
                    __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(bv)));
                return;
            }
            rr = seg_win + kWave;
        }
    };
    // a chunk is kUn codes per lane (8-byte loads of four); the first chunk of
    // a segment also brings the lane's starting trial.  Runs are multiples of
    // 4 codes, so only the second load of an eight-code chunk can lie past the
    // segment's end: it then reads skip codes from the block after the last
    // code.  Nothing
    // is selected on the loaded words, so the loads stay in flight while the
    // previous chunk is processed.
    unsigned long long X[kUn / 4];
    int X_start = 0;
    bool X_first = false;
    int chunk_rr = G;
    auto load = [&]() {
        chunk_rr = rr;
        if (rr < G) {
            X_first = step == 0;
            if (X_first) X_start = P.lane_start[(seg0 + static_cast<size_t>(rr) * kGroups) * kWave + lane];
#pragma unroll
            for (int q = 0; q < kUn / 4; ++q) {
                const uint16_t *src = step + 4 * q < R ? P.code + sb + static_cast<int64_t>((step >> 2) + q) * (4 * kWave)
                                                       : P.pad;   // uniform
                X[q] = ld_codes<SHARED>(src + 4 * lane);
            }
            step += kUn;
            if (step >= R) {
                ++rr;
                step = 0;
                seek();
            }
        }
    };

    // byte offset (from smem) of the lane's current trial total; a trial
    // advance moves it by one slot
    const uint32_t accw_off = acc_off + static_cast<uint32_t>(w * P.tg) * kV;
    uint32_t tofs = accw_off;
    __syncthreads();   // range table counts published
    RangeInfo cur = range_info(0);
    fetch(0, cur);
    seek();
    load();
    wait_dma();
    __syncthreads();

    for (int r = 0; r < G; ++r) {
        const uint2 *tbr = reinterpret_cast<const uint2 *>(smem);
        const V *tvals = reinterpret_cast<const V *>(smem + kBrBytes);
        const uint8_t *tcnt = smem + kBrBytes + static_cast<size_t>(P.capv) * kV;
        const size_t s = static_cast<size_t>(r >> 1);
        const V *gvals = reinterpret_cast<const V *>(T.vals) + s * kSr;
        const uint8_t *gcnt = HITS ? T.cnt + s * kSr : nullptr;
        const uint32_t vsh = cur.base & ~(kVPer16 - 1u), csh = cur.base & ~15u;
        // values with buffer index below vlim (and counts below clim) are in LDS
        const uint32_t vlim = static_cast<uint32_t>(P.capv), clim = static_cast<uint32_t>(P.capv);
        const bool all_lds = cur.cnt + (cur.base & 15u) <= static_cast<uint32_t>(P.capv);   // uniform
        // skip codes (0xFFFF) read the range's last bitmap bit: only when that
        // event is set do they have to be told apart from it
        const bool last_set = (__builtin_amdgcn_readfirstlane(tbr[1023].x) >> 31) != 0u;   // uniform
        RangeInfo nxt{0, 0};
        if (r + 1 < G) nxt = range_info(r + 1);
        // LDS byte offsets of value and count 0 of the super-range: unsigned
        // arithmetic, so the offsets wrap, while every address formed from
        // them lies in the buffer
        const uint32_t vbase = static_cast<uint32_t>(kBrBytes) - vsh * kV;
        const uint32_t cbase = static_cast<uint32_t>(kBrBytes) + static_cast<uint32_t>(P.capv) * kV - csh;
        auto chunk = [&](auto skip_tag) {
            constexpr bool kTellSkip = decltype(skip_tag)::value;
            if (X_first) tofs = accw_off + kV * static_cast<uint32_t>(X_start);
            // codes of this chunk, two per 32-bit word, low half first
            uint32_t wd[kUn / 2];
#pragma unroll
            for (int h = 0; h < kUn / 2; ++h) wd[h] = static_cast<uint32_t>(X[h >> 1] >> (32 * (h & 1)));
            load();   // prefetch the next chunk (possibly of a later range)
            // bitmap words of all codes first, without branches, so the LDS
            // reads are in flight together (offset bits 5..14 pick the word)
            uint32_t cw[kUn];
#pragma unroll
            for (int u = 0; u < kUn; ++u) cw[u] = (u & 1) ? (wd[u >> 1] >> 16) : wd[u >> 1];
            uint2 q[kUn];
#pragma unroll
            for (int u = 0; u < kUn; ++u) q[u] = tbr[__builtin_amdgcn_ubfe(cw[u], 5, 10)];
            // each code advances the lane's trial by its top bit
            uint32_t ta[kUn];
#pragma unroll
            for (int u = 0; u < kUn; ++u) {
                tofs = (u & 1) ? add_bit<31, kVSh>(tofs, wd[u >> 1]) : add_bit<15, kVSh>(tofs, wd[u >> 1]);
                ta[u] = tofs;
            }
            // bit and rank: the bit field instructions read only the low five
            // bits of their offset and width operands, which hold the bit
            bool on[kUn];
            uint32_t rank[kUn];
#pragma unroll
            for (int u = 0; u < kUn; ++u) {
                on[u] = __builtin_amdgcn_ubfe(q[u].x, cw[u], 1) != 0u;
                if (kTellSkip) on[u] = on[u] && (cw[u] & 0xFFFFu) != 0xFFFFu;
                rank[u] = __popc(__builtin_amdgcn_ubfe(q[u].x, 0, cw[u])) + q[u].y;
            }
            if (all_lds) {
                V v[kUn];
#pragma unroll
                for (int u = 0; u < kUn; ++u)
                    v[u] = *reinterpret_cast<const V *>(smem + ((on[u] ? rank[u] : vsh) * kV + vbase));
#pragma unroll
                for (int u = 0; u < kUn; ++u)
                    if (on[u]) {
                        atomicAdd(reinterpret_cast<V *>(smem + ta[u]), v[u]);
                        if (HITS)
                            atomicAdd(reinterpret_cast<int32_t *>(smem + hacc_off + ((ta[u] - acc_off) >> (kVSh - 2))),
                                      static_cast<int>(smem[rank[u] + cbase]));
                    }
            } else {
#pragma unroll
                for (int u = 0; u < kUn; ++u)
                    if (on[u]) {
                        // indexes relative to the buffer start, so that every
                        // address stays inside its array
                        V v;
                        int c = 0;
                        const uint32_t iv = rank[u] - vsh;
                        if (iv < vlim) v = tvals[iv];
                        else v = gvals[rank[u]];
                        if (HITS) {
                            const uint32_t ic = rank[u] - csh;
                            if (ic < clim) c = tcnt[ic];
                            else c = gcnt[rank[u]];
                        }
                        atomicAdd(reinterpret_cast<V *>(smem + ta[u]), v);
                        if (HITS) atomicAdd(reinterpret_cast<int32_t *>(smem + hacc_off + ((ta[u] - acc_off) >> (kVSh - 2))), c);
                    }
            }
        };
        if (last_set) {
            while (chunk_rr == r) chunk(std::true_type{});
        } else {
            while (chunk_rr == r) chunk(std::false_type{});
        }
        cur = nxt;
        __syncthreads();   // every wave is done with the table slice
        if (r + 1 < G) fetch(r + 1, nxt);
        wait_dma();
        __syncthreads();
    }
    if (active) {
        const double aggR = I.lterm[2], aggL = I.lterm[3];
        const int64_t lo = max(gt0, I.t0), hi = min(gt1, I.t1);
        for (int64_t t = lo + lane; t < hi; t += kWave) {
            const int i = static_cast<int>(t - b * tb);
            const double S = static_cast<double>(acc[i]);
            const size_t o = static_cast<size_t>(t - I.t0);
            I.ylt[o] = xl(S, aggR, aggL);
            if (I.s_pre) I.s_pre[o] = S;
            if (HITS && I.hits) I.hits[o] = hacc[i];
        }
    }
}

// LDS of one forward workgroup: the per-trial totals (and hit counts), the
// range table and segment windows, and what is left for one range's table
// slice: its 8 KB of bitmap words with ranks, then capv values (and capv
// ELT counts with hits; values and counts past capv are read from global
// memory).  Signed arithmetic: with the largest blocks, hit counts and the
// largest catalogue the fixed parts leave no room, which is a limit of this
// layout (ARA_E_LIMIT), not a wrap-around.
int32_t fwd_lds_plan(int tb, int n_ranges, bool hits, bool f32, int32_t *buf_bytes, int32_t *capv_out) {
    const int64_t vb = f32 ? 4 : 8;
    const int64_t fixed = static_cast<int64_t>(fwd_acc_lds(tb, hits, static_cast<size_t>(vb))) +
                          static_cast<int64_t>(fwd_meta_lds(n_ranges));
    const int64_t per_buf = (static_cast<int64_t>(kLdsBytes) - fixed) / 256 * 256;
    const int64_t room = per_buf - kBrBytes - (hits ? 16 : 0);
    int64_t capv = room > 0 ? (hits ? room / (vb + 1) : room / vb) : 0;
    capv = capv / 16 * 16;
    if (capv < 16)
        return fail(ARA_E_LIMIT, "forward: " + std::to_string(tb) + " trials per block and " + std::to_string(n_ranges) +
                                     " catalogue ranges leave no LDS for the table slice" +
                                     (hits ? " with hit counts" : ""));
    *buf_bytes = static_cast<int32_t>(per_buf);
    *capv_out = static_cast<int32_t>(capv);
    return ARA_OK;
}

int32_t launch_forward(const ara_yet *yet, int n_sr, bool hits, bool f32, const FwdItem *d_items, int n_items,
                       hipStream_t st, const FwdRegular *reg, bool shared) {
    (void)n_sr;
    if (n_items <= 0) return ARA_OK;
    FwdParams P{};
    P.code = yet->code;
    P.pad = yet->code + yet->n_codes;
    P.seg_base = yet->seg_base;
    P.seg_run = yet->seg_run;
    P.lane_start = yet->lane_start;
    P.n_trials = yet->n_trials;
    P.tg = yet->trials_per_group;
    P.tb = yet->trials_per_block;
    P.n_ranges = yet->n_ranges;
    // the range's table slice: [bitmap words with ranks][values][counts (hits mode)]
    int32_t rc = fwd_lds_plan(P.tb, P.n_ranges, hits, f32, &P.buf_bytes, &P.capv);
    if (rc) return rc;
    P.items = d_items;
    if (reg) {
        P.reg_tabs = reg->tabs;
        P.reg_lterm = reg->lterm;
        P.reg_ylt = reg->ylt;
        P.reg_s_pre = reg->s_pre;
        P.reg_hits = reg->hits;
        P.reg_t0 = reg->t0;
        P.reg_t1 = reg->t1;
        P.reg_b0 = reg->b0;
        P.reg_nb = reg->nb;
        P.reg_nl = reg->nl;
        shared = reg->nl > 1;
    }
    ProfScope prof(ARA_PROF_FWD, st);
#define ARA_FWD_LAUNCH(H, F)                                                   \
    do {                                                                     \
        if (shared) k_fwd<H, F, true><<<n_items, 1024, 0, st>>>(P);          \
        else k_fwd<H, F, false><<<n_items, 1024, 0, st>>>(P);                \
    } while (0)
    if (f32) {
        if (hits) ARA_FWD_LAUNCH(true, true);
        else ARA_FWD_LAUNCH(false, true);
    } else {
        if (hits) ARA_FWD_LAUNCH(true, false);
        else ARA_FWD_LAUNCH(false, false);
    }
#undef ARA_FWD_LAUNCH
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

// Layers are served in groups of four by the grouped forward (one
// workgroup streams a block's codes once for the group) when the call asks
// for neither hit counts nor binary32 accumulation and the workgroup holds
// four layers' totals; the layers after the last full group (and every layer
// otherwise) take the one-layer kernel.  Measured on the uneven workload's
// YET: a group of four costs 0.85 of four one-layer passes, two or three
// layers in one group no less than their one-layer passes.  Both kernels add
// a trial's values in the same order, so the split does not change a bit.
static int fwd_group_size(const ara_yet *yet, int n_layers, bool hits, bool f32) {
    if (n_layers < kGrpMax || hits || f32) return 0;
    return grp_max_members(yet->trials_per_block) >= kGrpMax ? kGrpMax : 0;
}

// Work items of a grouped launch: with one group, workgroup i takes block
// b0 + i; with several, the groups of one block run back to back on one XCD
// (workgroup 8k + x is the k-th on XCD x: group k % n_groups of block
// 8 (k / n_groups) + x), padded with empty items.
static int grp_items(int n_groups, int nb) {
    return n_groups <= 1 ? nb : n_groups * kXcds * ((nb + kXcds - 1) / kXcds);
}

struct GrpLayout {
    int gsize = 0, n_groups = 0, n_sr = 0;
    size_t gts, ubr, ucount, sbr, items;
};

static GrpLayout grp_layout(const ara_yet *yet, int n_sr, int n_layers, bool hits, bool f32) {
    GrpLayout g;
    g.gsize = fwd_group_size(yet, n_layers, hits, f32);
    if (!g.gsize) return g;
    g.n_groups = n_layers / g.gsize;   // full groups only
    g.n_sr = n_sr;
    g.gts = align256(static_cast<size_t>(g.n_groups) * sizeof(GrpTables));
    g.ubr = align256(static_cast<size_t>(g.n_groups) * n_sr * kSrWords * sizeof(uint2));
    g.ucount = align256(static_cast<size_t>(g.n_groups) * n_sr * sizeof(int32_t));
    g.sbr = align256(static_cast<size_t>(g.n_groups) * kGrpMax * n_sr * kSrWords * sizeof(uint2));
    g.items = align256(static_cast<size_t>(grp_items(g.n_groups, yet->n_blocks)) * sizeof(GrpItem));
    return g;
}

static size_t fwd_workspace(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, bool hits,
                            bool f32) {
    const OccLayoutSizes z = occ_sizes(tables->catalog, hits);
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    size_t b = kWsHeaderBytes;
    b += align256(static_cast<size_t>(L + 1) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(nJ, 1)) * sizeof(int32_t));
    b += align256(static_cast<size_t>(std::max(L, 1)) * sizeof(OccTables));
    b += static_cast<size_t>(L) * z.per_layer;
    const GrpLayout g = grp_layout(yet, z.n_sr, L, hits, f32);
    if (g.gsize) b += g.gts + g.ubr + g.ucount + g.sbr + g.items;
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
    if (flags & ~(ARA_F_EMIT_HITS | ARA_F_FP32_ACCUM)) return fail(ARA_E_INVAL, "unknown flag");
    int32_t bb = 0, cv = 0;
    if ((rc = fwd_lds_plan(yet->trials_per_block, yet->n_ranges, (flags & ARA_F_EMIT_HITS) != 0,
                           (flags & ARA_F_FP32_ACCUM) != 0, &bb, &cv)))
        return rc;
    *bytes = fwd_workspace(tables, yet, layers, (flags & ARA_F_EMIT_HITS) != 0, (flags & ARA_F_FP32_ACCUM) != 0);
    return ARA_OK;
}

namespace ara {

// Checks the arguments of a forward call; on success *need holds the
// workspace bytes it takes.
int32_t forward_args(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, const double *elt_terms,
                     const double *layer_terms, int64_t trial_begin, int64_t trial_end, uint32_t flags,
                     const double *ylt, const int32_t *hits, size_t *need) {
    int32_t rc = check_pair(tables, yet);
    if (rc) return rc;
    if ((rc = check_layers(layers, tables->n_elts))) return rc;
    if (flags & ~(ARA_F_EMIT_HITS | ARA_F_FP32_ACCUM)) return fail(ARA_E_INVAL, "unknown flag");
    const bool want_hits = (flags & ARA_F_EMIT_HITS) != 0;
    if (hits && !want_hits) return fail(ARA_E_INVAL, "hits output requires ARA_F_EMIT_HITS");
    if (trial_begin < 0 || trial_end < trial_begin || trial_end > yet->n_trials)
        return fail(ARA_E_RANGE, "trial range outside the YET");
    if (layers->n_layers > 0 && trial_end > trial_begin && (!ylt || !elt_terms || !layer_terms))
        return fail(ARA_E_INVAL, "null output or terms");
    int32_t bb = 0, cv = 0;
    if ((rc = fwd_lds_plan(yet->trials_per_block, yet->n_ranges, want_hits, (flags & ARA_F_FP32_ACCUM) != 0, &bb, &cv)))
        return rc;
    *need = fwd_workspace(tables, yet, layers, want_hits, (flags & ARA_F_FP32_ACCUM) != 0);
    return ARA_OK;
}

// The forward proper, once the arguments are checked, over a workspace of
// at least the bytes forward_args gave.
int32_t forward_run(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, const double *elt_terms,
                    const double *layer_terms, int64_t trial_begin, int64_t trial_end, uint32_t flags, double *ylt,
                    double *s_pre, int32_t *hits, void *ws, hipStream_t st) {
    int32_t rc = ARA_OK;
    const bool want_hits = (flags & ARA_F_EMIT_HITS) != 0;
    const bool f32 = (flags & ARA_F_FP32_ACCUM) != 0;
    const int L = layers->n_layers;
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
    const int64_t n = trial_end - trial_begin;
    const GrpLayout gl = grp_layout(yet, z.n_sr, L, want_hits, f32);
    GrpTables *d_gts = nullptr;
    GrpItem *d_gitems = nullptr;
    std::vector<GrpTables> gts;
    std::vector<GrpItem> gitems;
    // what the host sends (descriptors, layer lists, group descriptors and
    // work items) comes first, so that the one copy per call stays small
    if (gl.gsize) {
        d_gts = c.take<GrpTables>(static_cast<size_t>(gl.n_groups));
        d_gitems = c.take<GrpItem>(static_cast<size_t>(grp_items(gl.n_groups, nb)));
    }
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, z, want_hits);
    if (gl.gsize) {
        uint2 *ubr = c.take<uint2>(static_cast<size_t>(gl.n_groups) * z.n_sr * kSrWords);
        int32_t *ucount = c.take<int32_t>(static_cast<size_t>(gl.n_groups) * z.n_sr);
        uint2 *sbr = c.take<uint2>(static_cast<size_t>(gl.n_groups) * kGrpMax * z.n_sr * kSrWords);
        // layers [g G, (g + 1) G) form group g
        gts.resize(static_cast<size_t>(gl.n_groups));
        for (int g = 0; g < gl.n_groups; ++g) {
            GrpTables &t = gts[g];
            t = GrpTables{};
            t.ubr = ubr + static_cast<size_t>(g) * z.n_sr * kSrWords;
            t.ucount = ucount + static_cast<size_t>(g) * z.n_sr;
            t.sbr = sbr + static_cast<size_t>(g) * kGrpMax * z.n_sr * kSrWords;
            const int j0 = g * gl.gsize, j1 = j0 + gl.gsize;
            t.n = j1 - j0;
            for (int m = 0; m < t.n; ++m) t.mt[m] = d_tabs + j0 + m;
        }
        gitems.assign(static_cast<size_t>(grp_items(gl.n_groups, nb)), GrpItem{});
        for (size_t i = 0; i < gitems.size(); ++i) {
            GrpItem &it = gitems[i];
            it.block = -1;
            int g = 0, bi = static_cast<int>(i);
            if (gl.n_groups > 1) {
                const int x = static_cast<int>(i % kXcds), k = static_cast<int>(i / kXcds);
                g = k % gl.n_groups;
                bi = (k / gl.n_groups) * kXcds + x;
            }
            if (bi >= nb) continue;
            const int j0 = g * gl.gsize, j1 = j0 + gl.gsize;
            it.gt = d_gts + g;
            it.block = static_cast<int32_t>(b_lo) + bi;
            it.n = j1 - j0;
            it.mask = (1u << it.n) - 1u;
            for (int m = 0; m < it.n; ++m) {
                const int j = j0 + m;
                it.lterm[m] = layer_terms + 4 * j;
                it.t0[m] = trial_begin;
                it.t1[m] = trial_end;
                it.ylt[m] = ylt + static_cast<size_t>(j) * n;
                it.s_pre[m] = s_pre ? s_pre + static_cast<size_t>(j) * n : nullptr;
            }
        }
    }
    FwdRegular reg{};
    reg.tabs = d_tabs;
    reg.lterm = layer_terms;
    reg.ylt = ylt;
    reg.s_pre = s_pre;
    reg.hits = hits;
    reg.t0 = trial_begin;
    reg.t1 = trial_end;
    reg.b0 = static_cast<int32_t>(b_lo);
    reg.nb = nb;
    reg.nl = L;
    HeadImage img(ws);
    img.cover(d_err + kWsHeaderBytes / sizeof(int32_t));
    img.put(d_off, layers->elt_off, static_cast<size_t>(L + 1));
    img.put(d_ids, layers->elt_ids, static_cast<size_t>(nJ));
    img.put(d_tabs, tabs.data(), tabs.size());
    if (gl.gsize) {
        img.put(d_gts, gts.data(), gts.size());
        img.put(d_gitems, gitems.data(), gitems.size());
    }
    if ((rc = img.send(st))) return rc;

    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, want_hits, f32, d_tabs, z.n_sr, d_err,
                             st)))
            return rc;
    }
    int jg = 0;   // layers served by the grouped forward
    if (gl.gsize) {
        if ((rc = launch_grp_union(d_gts, gl.n_groups, z.n_sr, st))) return rc;
        if ((rc = launch_fwd_group(yet, d_gitems, static_cast<int>(gitems.size()), gl.gsize, st))) return rc;
        jg = gl.n_groups * gl.gsize;
    }
    if (jg == L) return ARA_OK;
    // the other layers [jg, L): the one-layer kernel
    reg.tabs = d_tabs + jg;
    reg.lterm = layer_terms + 4 * jg;
    reg.ylt = ylt + static_cast<size_t>(jg) * n;
    reg.s_pre = s_pre ? s_pre + static_cast<size_t>(jg) * n : nullptr;
    reg.hits = hits ? hits + static_cast<size_t>(jg) * n : nullptr;
    reg.nl = L - jg;
    return launch_forward(yet, z.n_sr, want_hits, f32, nullptr, fwd_regular_items(L - jg, nb), st, &reg);
}

}  // namespace ara

extern "C" int32_t ara_ylt_forward(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                   const double *elt_terms, const double *layer_terms, int64_t trial_begin,
                                   int64_t trial_end, uint32_t flags, double *ylt, double *s_pre, int32_t *hits,
                                   void *ws, size_t ws_bytes, void *stream) {
    size_t need = 0;
    int32_t rc = forward_args(tables, yet, layers, elt_terms, layer_terms, trial_begin, trial_end, flags, ylt, hits,
                              &need);
    if (rc) return rc;
    if (!ws) return fail(ARA_E_INVAL, "null workspace");
    if (ws_bytes < need) return fail(ARA_E_NOSPACE, "forward workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (layers->n_layers == 0 || trial_end == trial_begin) {
        ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
        return ARA_OK;
    }
    return forward_run(tables, yet, layers, elt_terms, layer_terms, trial_begin, trial_end, flags, ylt, s_pre, hits,
                       ws, st);
}
