// Grouped forward: the layers of one call (or the quotes of one server
// launch) that share a block of trials are served by ONE workgroup, which
// streams and decodes the block's codes once for all of them.
//
// Per group and super-range, a union table holds the events that are set
// (O != 0) in any member, with ranks, and per member a bitmap over the
// union's ranks marking the member's own set events (k_grp_union).  The
// streaming kernel walks the block's segments like the one-layer kernel,
// but probes the union table only: every occurrence of a union event is
// appended, as (trial, union rank), to a queue of its wavefront in LDS, and
// whenever 64 are queued each lane takes one and, for every member, tests
// the member's bitmap at that union rank and adds the member's O to the
// member's trial total.  So the decode and the table probe are paid once
// per code whatever the number of members, and the per-member work runs on
// full wavefronts of union hits instead of on every code.
//
// A member's additions to one trial happen in queue order (code order per
// lane, lane order per code position), which does not depend on the other
// members: a quote's totals are the same alone and in any mix.
//
// One workgroup per CU (160 KB of LDS): the totals of every member, the
// range's union words, each member's bitmap words and values for the range
// (or, when they do not fit, read from global memory), the queues and the
// segment windows.
#include "occ.h"

#include <algorithm>
#include <string>

namespace ara {

constexpr int kGrpLds = 160 * 1024;
constexpr int kGrpUn = 12;           // codes per lane and chunk (three 8-byte loads; 8 and 16 measured slower)
constexpr int kGrpQ = 128;           // queue entries per wavefront (a power of two)
constexpr int kRangeWin = 64;        // ranges whose counts are staged at once
constexpr uint32_t kNoLds = 0xFFFFFFFFu;

// counts of one range of the catalogue, staged in LDS
struct GrpRange {
    uint32_t ubase, ucnt;                      // union ranks [ubase, ubase + ucnt) of the super-range
    uint32_t mbase[kGrpMax], mcnt[kGrpMax];    // each member's ranks
};
static_assert(sizeof(GrpRange) == 40, "range record");

// where the current range's member tables are
struct GrpSlice {
    uint32_t sub_off;   // LDS byte offset of bitmap word sub_k0, or kNoLds (read from global memory)
    uint32_t sub_k0;
    uint32_t val_off;   // LDS byte offset of value rank val_r0, or kNoLds
    uint32_t val_r0;
};

// static LDS layout
constexpr uint32_t kOffUnion = 0;                                    // 1024 union words (8 KB)
constexpr uint32_t kOffWin = 8192;                                   // kRangeWin GrpRange
constexpr uint32_t kOffSlice = kOffWin + kRangeWin * 40;             // kGrpMax GrpSlice
constexpr uint32_t kOffSeg = kOffSlice + 256;                        // 16 x 64 (base, run) windows
constexpr uint32_t kOffQueue = kOffSeg + kGroups * kWave * 12;       // 16 x kGrpQ entries
constexpr uint32_t kOffAcc = kOffQueue + kGroups * kGrpQ * 4;        // members' totals
static_assert(kOffAcc % 256 == 0, "layout");

static uint32_t grp_acc_bytes(int tb, int gmax) {
    return static_cast<uint32_t>(align256(static_cast<size_t>(gmax) * (tb + 1) * sizeof(double)));
}

int grp_max_members(int tb) {
    for (int g = kGrpMax; g >= 1; --g)
        if (kOffAcc + grp_acc_bytes(tb, g) + 16 * 1024 <= static_cast<uint32_t>(kGrpLds)) return g;
    return 0;
}

// ---------------------------------------------------------------------------
// Union tables.

// The bits of m at the positions of u's set bits, packed from bit 0 up.
__device__ __forceinline__ uint32_t pext32(uint32_t m, uint32_t u) {
    uint32_t r = 0;
    int i = 0;
    while (u) {
        const uint32_t low = u & (0u - u);
        if (m & low) r |= 1u << i;
        ++i;
        u ^= low;
    }
    return r;
}

// Exclusive prefix sum of v over the 1024 threads; *total gets the sum.
// Every thread of the workgroup must call it.
__device__ uint32_t scan1024(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t incl = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t x = __shfl_up(incl, o);
        if (lane >= o) incl += x;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
        const uint32_t c = wsum[i];
        before += (i < w) ? c : 0u;
        tot += c;
    }
    *total = tot;
    __syncthreads();   // wsum is reused by the next call
    return before + incl - v;
}

// One workgroup per (super-range, group): the union words with ranks, then
// each member's bits over the union's ranks (gathered in LDS), then their
// ranks.  Thread t owns words 2t and 2t + 1.
__global__ __launch_bounds__(1024) void k_grp_union(const GrpTables *__restrict__ gts, int n_sr) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t sb[kGrpMax][kSrWords];
    const int s = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
    const GrpTables G = gts[g];
    const int n = G.n;
    const size_t w0 = static_cast<size_t>(s) * kSrWords;
    uint32_t mb[kGrpMax][2];
    uint32_t U[2] = {0u, 0u};
#pragma unroll
    for (int m = 0; m < kGrpMax; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            mb[m][h] = m < n ? G.mt[m]->br[w0 + 2 * tid + h].x : 0u;
            U[h] |= mb[m][h];
        }
    uint32_t total = 0;
    const uint32_t r0 = scan1024(__popc(U[0]) + __popc(U[1]), wsum, &total);
    const uint32_t r1 = r0 + __popc(U[0]);
    G.ubr[w0 + 2 * tid] = make_uint2(U[0], r0);
    G.ubr[w0 + 2 * tid + 1] = make_uint2(U[1], r1);
    if (tid == 0) G.ucount[s] = static_cast<int32_t>(total);
    for (int i = tid; i < kGrpMax * kSrWords; i += blockDim.x) sb[i / kSrWords][i % kSrWords] = 0u;
    __syncthreads();
    for (int m = 0; m < n; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t u = U[h];
            if (!u) continue;
            const uint32_t x = pext32(mb[m][h], u);
            const uint32_t p = h ? r1 : r0;
            const uint32_t sh = p & 31u;
            atomicOr(&sb[m][p >> 5], x << sh);
            // p + popc(u) <= 65536, so a second word exists whenever the bits spill into it
            if (sh && sh + static_cast<uint32_t>(__popc(u)) > 32u) atomicOr(&sb[m][(p >> 5) + 1], x >> (32u - sh));
        }
    __syncthreads();
    for (int m = 0; m < n; ++m) {   // uniform: scan1024 holds barriers
        const uint32_t a0 = sb[m][2 * tid], a1 = sb[m][2 * tid + 1];
        uint32_t tot = 0;
        const uint32_t q0 = scan1024(__popc(a0) + __popc(a1), wsum, &tot);
        uint2 *dst = G.sbr + (static_cast<size_t>(m) * n_sr + s) * kSrWords;
        dst[2 * tid] = make_uint2(a0, q0);
        dst[2 * tid + 1] = make_uint2(a1, q0 + __popc(a0));
    }
}

// ---------------------------------------------------------------------------
// Streaming.

struct GrpParams {
    const uint16_t *code;
    const uint16_t *pad;        // kPadCodes skip codes
    const int64_t *seg_base;
    const int32_t *seg_run;
    const uint8_t *lane_start;
    int64_t n_trials;
    int32_t tg, tb, n_ranges, n_sr;
    uint32_t slice_off, slice_end;   // LDS bytes for the members' range tables
    int32_t gmax;                    // members the totals region holds
    const GrpItem *items;
};

__device__ __forceinline__ unsigned long long ld_codes_l2(const uint16_t *p) {
    return *reinterpret_cast<const unsigned long long *>(p);
}

// 16 bytes per lane from global memory into LDS at lds_base + 16 * lane
// (lds_base uniform); the kernel waits for these copies itself (vmcnt(0)
// before the barrier that publishes them).
__device__ __forceinline__ void grp_dma16(const void *src, uint32_t lds_base) {
    asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_base)), "v"(src)
                 : "memory", "m0");
}

__device__ __forceinline__ void grp_wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__global__ __launch_bounds__(1024) void k_fwd_group(GrpParams P) {
    __shared__ __align__(16) unsigned char smem[kGrpLds];
    const GrpItem I = P.items[blockIdx.x];
    if (I.block < 0 || I.n <= 0) return;   // uniform over the workgroup, before any barrier
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tb = P.tb, NR = P.n_ranges;
    const int nm = min(I.n, P.gmax);   // the host never groups more
    const int64_t b = I.block;
    const GrpTables GT = *I.gt;
    const double *mvals[kGrpMax];
    for (int m = 0; m < kGrpMax; ++m) mvals[m] = m < nm ? GT.mt[m]->vals : nullptr;
    const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(smem));
    const uint32_t acc_stride = static_cast<uint32_t>(tb + 1) * 8u;

    // members whose trial range meets this block (uniform)
    const int64_t bt0 = b * tb, bt1 = min(bt0 + tb, P.n_trials);
    uint32_t act = 0;
#pragma unroll
    for (int m = 0; m < kGrpMax; ++m)
        if (m < nm && ((I.mask >> m) & 1u) && I.t0[m] < bt1 && I.t1[m] > bt0) act |= 1u << m;
    const int64_t gt0 = bt0 + static_cast<int64_t>(w) * P.tg;
    const int64_t gt1 = min(gt0 + P.tg, P.n_trials);
    const bool active = act != 0u && gt0 < gt1;
    const size_t seg0 = static_cast<size_t>(b) * NR * kGroups + w;

    double *acc = reinterpret_cast<double *>(smem + kOffAcc);
    for (int i = tid; i < nm * (tb + 1); i += blockDim.x) acc[i] = 0.0;

    GrpRange *win = reinterpret_cast<GrpRange *>(smem + kOffWin);
    GrpSlice *sl = reinterpret_cast<GrpSlice *>(smem + kOffSlice);
    // counts of ranges [r0, r0 + kRangeWin): thread i reads table i / kRangeWin
    // (0: the union, m + 1: member m) for range r0 + i % kRangeWin
    auto stage_window = [&](int r0) {
        for (int i = tid; i < kRangeWin * (1 + nm); i += blockDim.x) {
            const int rl = i % kRangeWin, which = i / kRangeWin, r = r0 + rl;
            if (r >= NR) continue;
            const size_t sr = static_cast<size_t>(r >> 1);
            uint32_t mid, tot;
            if (which == 0) {
                mid = GT.ubr[sr * kSrWords + 1024].y;
                tot = static_cast<uint32_t>(GT.ucount[sr]);
            } else {
                const OccTables *T = which == 1 ? GT.mt[0] : which == 2 ? GT.mt[1] : which == 3 ? GT.mt[2] : GT.mt[3];
                mid = T->br[sr * kSrWords + 1024].y;
                tot = static_cast<uint32_t>(T->count[sr]);
            }
            const uint32_t base = (r & 1) ? mid : 0u, cnt = (r & 1) ? tot - mid : mid;
            if (which == 0) {
                win[rl].ubase = base;
                win[rl].ucnt = cnt;
            } else {
                win[rl].mbase[which - 1] = base;
                win[rl].mcnt[which - 1] = cnt;
            }
        }
    };
    // thread 0: where range r's member tables go in LDS (first every member's
    // bitmap words, then their values, in member order, while they fit).
    // Every region planned holds at least 16 bytes, so that the reads of
    // lanes without an entry (at offset 0) stay inside it.
    auto plan = [&](int r) {
        const GrpRange &R = win[r % kRangeWin];
        uint32_t off = P.slice_off;
        const uint32_t k0 = (R.ubase >> 5) & ~1u, k1 = (R.ubase + R.ucnt + 31u) >> 5;
        const uint32_t sub_bytes = max(((k1 - k0) * 8u + 15u) & ~15u, 16u);
        for (int m = 0; m < nm; ++m) {
            sl[m].sub_k0 = k0;
            sl[m].sub_off = kNoLds;
            if (((act >> m) & 1u) && off + sub_bytes <= P.slice_end) {
                sl[m].sub_off = off;
                off += sub_bytes;
            }
        }
        for (int m = 0; m < nm; ++m) {
            const uint32_t v0 = R.mbase[m] & ~1u;
            const uint32_t vb = max(((R.mbase[m] + R.mcnt[m] - v0) * 8u + 15u) & ~15u, 16u);
            sl[m].val_r0 = v0;
            sl[m].val_off = kNoLds;
            if (((act >> m) & 1u) && off + vb <= P.slice_end) {
                sl[m].val_off = off;
                off += vb;
            }
        }
    };
    // copy range r's union words and the planned member tables into LDS
    auto fetch = [&](int r) {
        const size_t sr = static_cast<size_t>(r >> 1);
        const GrpRange &R = win[r % kRangeWin];
        const unsigned char *gu = reinterpret_cast<const unsigned char *>(GT.ubr + sr * kSrWords + (r & 1) * 1024);
        for (int c0 = w * kWave; c0 < 512; c0 += kGroups * kWave)
            grp_dma16(gu + static_cast<size_t>(c0 + lane) * 16, lds0 + kOffUnion + c0 * 16);
#pragma unroll
        for (int m = 0; m < kGrpMax; ++m) {
            if (m >= nm) break;
            const uint32_t so = uni(sl[m].sub_off), k0 = uni(sl[m].sub_k0);
            if (so != kNoLds) {
                const uint32_t k1 = (uni(R.ubase) + uni(R.ucnt) + 31u) >> 5;
                const int nc = static_cast<int>((k1 - k0 + 1u) / 2u);
                const unsigned char *src = reinterpret_cast<const unsigned char *>(
                    GT.sbr + (static_cast<size_t>(m) * P.n_sr + sr) * kSrWords + k0);
                for (int c0 = w * kWave; c0 < nc; c0 += kGroups * kWave)
                    if (c0 + lane < nc) grp_dma16(src + static_cast<size_t>(c0 + lane) * 16, lds0 + so + c0 * 16);
            }
            const uint32_t vo = uni(sl[m].val_off), v0 = uni(sl[m].val_r0);
            if (vo != kNoLds) {
                const uint32_t v1 = uni(R.mbase[m]) + uni(R.mcnt[m]);
                const int nc = static_cast<int>((v1 - v0 + 1u) / 2u);
                const unsigned char *src = reinterpret_cast<const unsigned char *>(mvals[m] + sr * kSr + v0);
                for (int c0 = w * kWave; c0 < nc; c0 += kGroups * kWave)
                    if (c0 + lane < nc) grp_dma16(src + static_cast<size_t>(c0 + lane) * 16, lds0 + vo + c0 * 16);
            }
        }
    };

    // stream cursor over this wave's segments, as in the one-layer kernel
    int64_t *wbase = reinterpret_cast<int64_t *>(smem + kOffSeg) + w * kWave;
    int32_t *wrun = reinterpret_cast<int32_t *>(smem + kOffSeg + kGroups * kWave * 8) + w * kWave;
    int seg_win = -kWave;
    uint64_t nonempty = 0;
    int rr = active ? 0 : NR, step = 0, R = 0;
    int64_t sb = 0;
    auto seek = [&]() {
        while (rr < NR) {
            if (rr >= seg_win + kWave) {
                seg_win = rr & ~(kWave - 1);
                const int r = seg_win + lane;
                int32_t run = 0;
                int64_t base = 0;
                if (r < NR) {
                    const size_t si = seg0 + static_cast<size_t>(r) * kGroups;
                    run = P.seg_run[si];
                    base = P.seg_base[si];
                }
                wrun[lane] = run;
                wbase[lane] = base;
                nonempty = __ballot(run > 0);
            }
            const uint64_t mk = nonempty & (~0ull << (rr - seg_win));
            if (mk) {
                const int l = __builtin_ctzll(mk);
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
    unsigned long long X[kGrpUn / 4];
    int X_start = 0;
    bool X_first = false;
    int chunk_rr = NR;
    auto load = [&]() {
        chunk_rr = rr;
        if (rr < NR) {
            X_first = step == 0;
            if (X_first) X_start = P.lane_start[(seg0 + static_cast<size_t>(rr) * kGroups) * kWave + lane];
#pragma unroll
            for (int q = 0; q < kGrpUn / 4; ++q) {
                const uint16_t *src = step + 4 * q < R ? P.code + sb + static_cast<int64_t>((step >> 2) + q) * (4 * kWave)
                                                       : P.pad;   // uniform
                X[q] = ld_codes_l2(src + 4 * lane);
            }
            step += kGrpUn;
            if (step >= R) {
                ++rr;
                step = 0;
                seek();
            }
        }
    };

    uint32_t *queue = reinterpret_cast<uint32_t *>(smem + kOffQueue) + w * kGrpQ;
    int qhead = 0, qlen = 0;          // uniform
    uint32_t tl = 0;                  // the lane's trial within the block

    stage_window(0);
    __syncthreads();
    if (tid == 0) plan(0);
    __syncthreads();
    fetch(0);
    seek();
    load();
    grp_wait_dma();
    __syncthreads();

    for (int r = 0; r < NR; ++r) {
        const size_t sr = static_cast<size_t>(r >> 1);
        const uint32_t ubase = uni(win[r % kRangeWin].ubase);
        GrpSlice S[kGrpMax];
        for (int m = 0; m < kGrpMax; ++m) {
            if (m < nm) {
                S[m].sub_off = uni(sl[m].sub_off);
                S[m].sub_k0 = uni(sl[m].sub_k0);
                S[m].val_off = uni(sl[m].val_off);
                S[m].val_r0 = uni(sl[m].val_r0);
            } else {
                S[m] = GrpSlice{kNoLds, 0u, kNoLds, 0u};
            }
        }
        const uint2 *ubr = reinterpret_cast<const uint2 *>(smem + kOffUnion);
        // per member, for 64 queued union occurrences at most: test the
        // member's bit at the union rank, rank it, add O to the trial total
        auto drain = [&](int n) {   // n uniform, 1..64
            const bool in = lane < n;
            uint32_t e = queue[(qhead + lane) & (kGrpQ - 1)];
            if (!in) e = ubase;   // a harmless in-range entry (trial 0, the range's first union rank)
            qhead = (qhead + n) & (kGrpQ - 1);
            qlen -= n;
            const uint32_t gu = e & 0xFFFFu, t = e >> 16, bit = gu & 31u;
#pragma unroll
            for (int m = 0; m < kGrpMax; ++m) {
                if (m >= nm || !((act >> m) & 1u)) continue;
                uint2 sw;
                if (S[m].sub_off != kNoLds)
                    sw = *reinterpret_cast<const uint2 *>(smem + S[m].sub_off + ((gu >> 5) - S[m].sub_k0) * 8u);
                else
                    sw = GT.sbr[(static_cast<size_t>(m) * P.n_sr + sr) * kSrWords + (gu >> 5)];
                const bool on = in && ((sw.x >> bit) & 1u);
                const uint32_t rk = __popc(sw.x & ((1u << bit) - 1u)) + sw.y;
                double v;
                if (S[m].val_off != kNoLds)
                    v = *reinterpret_cast<const double *>(smem + S[m].val_off + ((on ? rk : S[m].val_r0) - S[m].val_r0) * 8u);
                else
                    v = on ? mvals[m][sr * kSr + rk] : 0.0;
                if (on) atomicAdd(reinterpret_cast<double *>(smem + kOffAcc + m * acc_stride + t * 8u), v);
            }
        };
        while (chunk_rr == r) {
            if (X_first) tl = static_cast<uint32_t>(w * P.tg + X_start);
            uint32_t wd[kGrpUn / 2];
#pragma unroll
            for (int h = 0; h < kGrpUn / 2; ++h) wd[h] = static_cast<uint32_t>(X[h >> 1] >> (32 * (h & 1)));
            load();   // prefetch the next chunk (possibly of a later range)
            uint32_t cw[kGrpUn];
            uint2 q[kGrpUn];
#pragma unroll
            for (int u = 0; u < kGrpUn; ++u) {
                cw[u] = (u & 1) ? (wd[u >> 1] >> 16) : (wd[u >> 1] & 0xFFFFu);
                q[u] = ubr[__builtin_amdgcn_ubfe(cw[u], 5, 10)];
            }
#pragma unroll
            for (int u = 0; u < kGrpUn; ++u) {
                tl += cw[u] >> 15;
                // skip codes (0xFFFF) stand for no event
                const bool on = __builtin_amdgcn_ubfe(q[u].x, cw[u], 1) != 0u && cw[u] != 0xFFFFu;
                const uint32_t gu = __popc(__builtin_amdgcn_ubfe(q[u].x, 0, cw[u])) + q[u].y;
                const uint64_t mk = __ballot(on);
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mk >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mk), 0u));
                if (on) queue[(qhead + qlen + below) & (kGrpQ - 1)] = (tl << 16) | gu;
                qlen += __popcll(mk);
                if (qlen >= kWave) drain(kWave);
            }
        }
        while (qlen > 0) drain(min(qlen, kWave));
        __syncthreads();   // every wave is done with range r's tables
        if (r + 1 < NR) {
            if ((r + 1) % kRangeWin == 0) {
                stage_window(r + 1);
                __syncthreads();
            }
            if (tid == 0) plan(r + 1);
            __syncthreads();
            fetch(r + 1);
        }
        grp_wait_dma();
        __syncthreads();
    }
    // aggregate terms, per member over its trials in this block
#pragma unroll
    for (int m = 0; m < kGrpMax; ++m) {
        if (m >= nm || !((act >> m) & 1u)) continue;
        const double aggR = I.lterm[m][2], aggL = I.lterm[m][3];
        const int64_t lo = max(bt0, I.t0[m]), hi = min(bt1, I.t1[m]);
        for (int64_t t = lo + tid; t < hi; t += blockDim.x) {
            const double S = acc[m * (tb + 1) + static_cast<int>(t - bt0)];
            const size_t o = static_cast<size_t>(t - I.t0[m]);
            I.ylt[m][o] = xl(S, aggR, aggL);
            if (I.s_pre[m]) I.s_pre[m][o] = S;
        }
    }
}

int32_t launch_grp_union(const GrpTables *d_gts, int n_groups, int n_sr, hipStream_t st) {
    if (n_groups <= 0 || n_sr <= 0) return ARA_OK;
    k_grp_union<<<dim3(static_cast<unsigned>(n_sr), static_cast<unsigned>(n_groups)), 1024, 0, st>>>(d_gts, n_sr);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

int32_t launch_fwd_group(const ara_yet *yet, const GrpItem *d_items, int n_items, int gmax, hipStream_t st) {
    if (n_items <= 0) return ARA_OK;
    if (gmax < 1 || gmax > grp_max_members(yet->trials_per_block))
        return fail(ARA_E_LIMIT, "grouped forward: more members than the LDS of one workgroup holds");
    GrpParams P{};
    P.code = yet->code;
    P.pad = yet->code + yet->n_codes;
    P.seg_base = yet->seg_base;
    P.seg_run = yet->seg_run;
    P.lane_start = yet->lane_start;
    P.n_trials = yet->n_trials;
    P.tg = yet->trials_per_group;
    P.tb = yet->trials_per_block;
    P.n_ranges = yet->n_ranges;
    P.n_sr = (yet->catalog + kSr - 1) / kSr;
    P.slice_off = kOffAcc + grp_acc_bytes(P.tb, gmax);
    P.slice_end = kGrpLds;
    P.gmax = gmax;
    P.items = d_items;
    ProfScope prof(ARA_PROF_FWD, st);
    k_fwd_group<<<n_items, 1024, 0, st>>>(P);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

}  // namespace ara
