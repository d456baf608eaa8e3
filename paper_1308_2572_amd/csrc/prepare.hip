// YET preparation: validate the trials and lay them out by (block of trials,
// catalogue range, trial group) so that the forward kernel can keep one
// range's occurrence table in LDS while streaming, in 16-bit codes; and, on
// request, the event-major copy that the backward reads.
//
// Code stream of one segment (block b, range r, group g): the occurrences of
// the group's trials whose event lies in range r, in trial order (storage
// order inside a trial), one 16-bit code each:
//     bit 15      advance to the next trial of the group before this code
//     bits 0..14  the event's offset in the range
// 0xFFFF means "advance, no event": it stands for each trial of the group
// with no event in the range between two that have some, for the advance of
// an event at offset 0x7FFF that opens a trial (which then follows as plain
// 0x7FFF), and for padding.  The padded stream is dealt to the 64 lanes as
// runs of `run` consecutive codes (run a multiple of 4), lane j starting from
// trial lane_start[j] of the group; code s of lane j sits at
//     base + (s / 4) * 256 + 4 * j + s % 4,
// so a wavefront reads four steps of all its lanes as one 512-byte block.
//
// With positions, a second array of the same shape holds, at each code's
// slot, the occurrence's position in its trial (its index less the trial's
// first index; 0xFFFF for gap codes and padding), so that a walk of the code
// stream can name each occurrence by its trial-major index.  Trials then hold
// at most 65536 occurrences.
#include "ara_internal.h"

#include <algorithm>
#include <vector>

namespace ara {

constexpr uint16_t kAdvance = 0x8000;
constexpr uint16_t kSkip = 0xFFFF;
constexpr int kRangeWindow = 1024;   // ranges tracked at once in a wavefront's LDS state

struct Geometry {
    int tg, tb, n_blocks, n_ranges, gbits;
    int slice_blocks;   // blocks per trial slice of the event-major copy
    size_t nseg;
};

static Geometry geometry(int64_t n_trials, int32_t catalog) {
    Geometry g{};
    const int64_t cu = device_cu_count();
    // two blocks per CU: the forward runs two workgroups on every CU
    int64_t tg = (n_trials + 2 * kGroups * cu - 1) / (2 * kGroups * cu);
    tg = std::max<int64_t>(1, std::min<int64_t>(tg, kMaxTrialsPerGroup));
    g.tg = static_cast<int>(tg);
    g.tb = kGroups * g.tg;
    g.n_blocks = static_cast<int>((n_trials + g.tb - 1) / g.tb);
    g.n_ranges = (catalog + kRange - 1) / kRange;
    g.gbits = 0;
    while ((1 << g.gbits) < g.n_ranges) ++g.gbits;
    g.nseg = static_cast<size_t>(g.n_blocks) * g.n_ranges * kGroups;
    g.slice_blocks = std::max(1, (g.n_blocks + kSlices - 1) / kSlices);
    return g;
}

// Upper bound of the codes: a segment holds its events, at most tg - 1 gap
// codes, at most tg - 1 advances for events at offset 0x7FFF, and fewer than
// 4 * 64 padding codes.
static int64_t max_codes(const Geometry &g, int64_t nnz) {
    return nnz + static_cast<int64_t>(g.nseg) * (2 * g.tg + 4 * kWave);
}

static size_t prepare_bytes(const Geometry &g, int64_t n_trials, int64_t nnz, int32_t catalog, uint32_t flags) {
    Carver c(nullptr);
    c.take<uint16_t>(static_cast<size_t>(max_codes(g, nnz)) + kPadCodes);
    c.take<int64_t>(g.nseg);
    c.take<int32_t>(g.nseg);
    c.take<uint8_t>(g.nseg * kWave);
    c.take<int64_t>(32);
    if (flags & ARA_PREP_TRANSPOSED) {
        c.take<int64_t>(static_cast<size_t>(kSlices) * catalog + 1);
        c.take<uint32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        c.take<int64_t>(static_cast<size_t>(kSlices) * g.n_ranges);
    }
    if (flags & ARA_PREP_TRIAL_MAJOR) {
        c.take<int64_t>(static_cast<size_t>(n_trials) + 1);
        c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        c.take<int32_t>(static_cast<size_t>(catalog));
    }
    if (flags & ARA_PREP_POSITIONS) {
        c.take<uint16_t>(static_cast<size_t>(max_codes(g, nnz)) + kPadCodes);
        if (!(flags & ARA_PREP_TRIAL_MAJOR)) c.take<int64_t>(static_cast<size_t>(n_trials) + 1);
    }
    return c.bytes();
}

__device__ __forceinline__ int64_t code_slot(int64_t base, int s, int lane) {
    return base + static_cast<int64_t>(s >> 2) * (4 * kWave) + 4 * lane + (s & 3);
}

// One pass over a wavefront's trial group, in trial order, per window of
// ranges.  Pass one (SCATTER = false) counts each segment's codes and the
// events, validating IDs and offsets; pass two writes the codes and the
// lanes' starting trials.  Within a 64-ID chunk of a trial, the lanes of one
// range are its occurrences in storage order (a stable multi-split by
// ballots); the first of them settles what precedes them in the segment: gap
// codes for skipped trials and the advance flag.  With `pos`, pass two also
// writes each occurrence's position in its trial beside its code, and with
// `long_trial`, pass one flags a trial of more than kMaxPositions occurrences.
template <bool SCATTER>
__global__ __launch_bounds__(1024) void k_prep_codes(const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ ids, int64_t n_trials,
                                                     int32_t catalog, int tg, int tb, int n_ranges, int gbits,
                                                     int32_t *__restrict__ seg_codes,
                                                     const int64_t *__restrict__ seg_base,
                                                     const int32_t *__restrict__ seg_run,
                                                     uint16_t *__restrict__ code, uint8_t *__restrict__ lane_start,
                                                     uint16_t *__restrict__ pos, int32_t *__restrict__ err,
                                                     int32_t *__restrict__ long_trial,
                                                     unsigned long long *__restrict__ events) {
    __shared__ int32_t cur_all[kGroups * kRangeWindow];   // codes so far per range
    __shared__ int16_t last_all[kGroups * kRangeWindow];  // last trial seen per range, -1 none
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t *cur = cur_all + w * kRangeWindow;
    int16_t *last = last_all + w * kRangeWindow;
    const int64_t b = blockIdx.x;
    const int64_t t0 = b * tb + static_cast<int64_t>(w) * tg;
    const int64_t t1 = std::min<int64_t>(t0 + tg, n_trials);
    auto seg_of = [&](int r) { return (static_cast<size_t>(b) * n_ranges + r) * kGroups + w; };
    // position p of range r's segment gets code c (and, for an occurrence,
    // its position `at` in the trial); the state before it is trial `start`
    auto put = [&](int r, int64_t p, uint16_t c, int start, uint16_t at) {
        const size_t si = seg_of(r);
        const int run = seg_run[si];
        const int lj = static_cast<int>(p / run);
        const int s = static_cast<int>(p - static_cast<int64_t>(lj) * run);
        const int64_t slot = code_slot(seg_base[si], s, lj);
        code[slot] = c;
        if (pos) pos[slot] = at;
        if (s == 0) lane_start[si * kWave + lj] = static_cast<uint8_t>(start);
    };
    unsigned long long ev = 0;
    for (int w0 = 0; w0 < n_ranges; w0 += kRangeWindow) {
        const int wn = min(kRangeWindow, n_ranges - w0);
        for (int r = lane; r < wn; r += kWave) {
            cur[r] = 0;
            last[r] = -1;
        }
        __builtin_amdgcn_wave_barrier();
        for (int64_t t = t0; t < t1; ++t) {
            const int i = static_cast<int>(t - t0);
            const int64_t o0 = off[t], o1 = off[t + 1];
            if (o1 < o0 || o0 < 0) {
                if (!SCATTER && lane == 0 && w0 == 0) atomicCAS(err, 0, ARA_E_RANGE);
                continue;
            }
            if (!SCATTER && long_trial && lane == 0 && w0 == 0 && o1 - o0 > kMaxPositions) atomicOr(long_trial, 1);
            for (int64_t base = o0; base < o1; base += kWave) {
                const int64_t k = base + lane;
                const bool in = k < o1;
                const int32_t id = in ? ids[k] : 0;
                const bool bad = in && (id < 0 || id >= catalog);
                if (!SCATTER && bad && w0 == 0) atomicCAS(err, 0, ARA_E_RANGE);
                const int r = (in && !bad) ? (id >> kRangeBits) : -1;
                const bool active = r >= w0 && r < w0 + wn;
                uint64_t peers = __ballot(active);
                for (int bit = 0; bit < gbits; ++bit) {
                    const bool on = (r >> bit) & 1;
                    const uint64_t m = __ballot(active && on);
                    peers &= on ? m : ~m;
                }
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(peers >> 32),
                                                                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(peers), 0u));
                const int tot = __popcll(peers);
                const int leader = active ? __builtin_ctzll(peers) : lane;
                const uint16_t local = static_cast<uint16_t>(id & (kRange - 1));
                int p_open = 0, adv_open = 0;
                if (active && rank == 0) {
                    const int rl = r - w0;
                    const int L = last[rl];
                    int gap = 0;
                    bool adv = false;
                    if (L >= 0 && L != i) {       // opens trial i after trial L in this segment
                        gap = i - L - 1;
                        adv = true;
                        if (local == (kRange - 1)) {   // offset 0x7FFF cannot carry the flag
                            ++gap;
                            adv = false;
                        }
                    }
                    const int p0 = cur[rl];
                    if (SCATTER)
                        for (int q = 0; q < gap; ++q) put(r, p0 + q, kSkip, L + q, kSkip);   // each advances one trial
                    cur[rl] = p0 + gap + tot;
                    last[rl] = static_cast<int16_t>(i);
                    p_open = p0 + gap;
                    adv_open = adv ? 1 : 0;
                }
                if (!SCATTER) ev += active ? 1u : 0u;
                p_open = __shfl(p_open, leader);
                adv_open = __shfl(adv_open, leader);
                if (SCATTER && active) {
                    const int a = (rank == 0) ? adv_open : 0;
                    put(r, p_open + static_cast<int>(rank), static_cast<uint16_t>((a ? kAdvance : 0) | local), i - a,
                        static_cast<uint16_t>(k - o0));
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (!SCATTER)
            for (int r = lane; r < wn; r += kWave) seg_codes[seg_of(w0 + r)] = cur[r];
        __builtin_amdgcn_wave_barrier();
    }
    if (!SCATTER) {
        for (int o = 32; o > 0; o >>= 1) ev += __shfl_down(ev, o);
        if (lane == 0 && ev) atomicAdd(events, ev);
    }
}

// Largest number of occurrences of any single event (bounds the backward's
// fixed-point accumulators), and on request every event's count (ev_count,
// [catalog]).  0xFFFF never encodes an occurrence, so the counts are exact.
__global__ __launch_bounds__(1024) void k_prep_max_occ(const uint16_t *__restrict__ code,
                                                       const int64_t *__restrict__ seg_base,
                                                       const int32_t *__restrict__ seg_run, int n_blocks,
                                                       int n_ranges, int32_t *__restrict__ max_occ,
                                                       int32_t catalog, int32_t *__restrict__ ev_count) {
    __shared__ uint32_t hist[kRange];
    __shared__ uint32_t red[16];
    for (int i = threadIdx.x; i < kRange; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int r = blockIdx.x;
    for (int b = 0; b < n_blocks; ++b) {
        for (int g = 0; g < kGroups; ++g) {
            const size_t sidx = (static_cast<size_t>(b) * n_ranges + r) * kGroups + g;
            const int64_t sb = seg_base[sidx];
            const int64_t n = static_cast<int64_t>(seg_run[sidx]) * kWave;
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
                const uint16_t c = code[sb + i];
                if (c != kSkip) atomicAdd(&hist[c & (kRange - 1)], 1u);
            }
        }
    }
    __syncthreads();
    if (ev_count)
        for (int i = threadIdx.x; i < kRange; i += blockDim.x) {
            const int64_t e = static_cast<int64_t>(r) * kRange + i;
            if (e < catalog) ev_count[e] = static_cast<int32_t>(hist[i]);
        }
    uint32_t m = 0;
    for (int i = threadIdx.x; i < kRange; i += blockDim.x) m = std::max(m, hist[i]);
    for (int o = 32; o > 0; o >>= 1) m = std::max(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), o)));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t mm = 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) mm = std::max(mm, red[i]);
        atomicMax(max_occ, static_cast<int32_t>(mm));
    }
}

// Event-major copy, pass 1: per (catalogue range r, trial slice x) count the
// occurrences of each event of the range in the slice's blocks; counts go to
// tr_off[x*catalog + e] and the region's total to rtot[x*n_ranges + r].
__global__ __launch_bounds__(1024) void k_tr_count(const uint16_t *__restrict__ code,
                                                   const int64_t *__restrict__ seg_base,
                                                   const int32_t *__restrict__ seg_run, int n_blocks, int n_ranges,
                                                   int slice_blocks, int32_t catalog, int64_t *__restrict__ tr_off,
                                                   int64_t *__restrict__ rtot) {
    __shared__ uint32_t hist[kRange];
    __shared__ unsigned long long red[16];
    const int r = blockIdx.x, x = blockIdx.y, tid = threadIdx.x;
    for (int i = tid; i < kRange; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int b0 = x * slice_blocks, b1 = min(n_blocks, b0 + slice_blocks);
    for (int b = b0; b < b1; ++b)
        for (int g = 0; g < kGroups; ++g) {
            const size_t sidx = (static_cast<size_t>(b) * n_ranges + r) * kGroups + g;
            const int64_t sb = seg_base[sidx];
            const int64_t n = static_cast<int64_t>(seg_run[sidx]) * kWave;
            for (int64_t i = tid; i < n; i += blockDim.x) {
                const uint16_t c = code[sb + i];
                if (c != kSkip) atomicAdd(&hist[c & (kRange - 1)], 1u);
            }
        }
    __syncthreads();
    const int64_t e0 = static_cast<int64_t>(r) * kRange;
    const int nloc = static_cast<int>(min<int64_t>(kRange, catalog - e0));
    unsigned long long sum = 0;
    for (int l = tid; l < nloc; l += blockDim.x) {
        tr_off[static_cast<int64_t>(x) * catalog + e0 + l] = hist[l];
        sum += hist[l];
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
    if ((tid & 63) == 0) red[tid >> 6] = sum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += red[i];
        rtot[static_cast<size_t>(x) * n_ranges + r] = static_cast<int64_t>(t);
    }
}

// Event-major copy, pass 2: turn the region's counts into list starts (the
// region begins at rbase[x*n_ranges + r]) and scatter each occurrence's
// slice-local trial index into its event's list.  Wavefront g decodes the
// segments of trial group g, each lane its own run.
__global__ __launch_bounds__(1024) void k_tr_scatter(const uint16_t *__restrict__ code,
                                                     const int64_t *__restrict__ seg_base,
                                                     const int32_t *__restrict__ seg_run,
                                                     const uint8_t *__restrict__ lane_start, int n_blocks,
                                                     int n_ranges, int tg, int tb, int slice_blocks, int32_t catalog,
                                                     const int64_t *__restrict__ rbase, int64_t *__restrict__ tr_off,
                                                     uint32_t *__restrict__ tr_ent) {
    constexpr int kPer = kRange / 1024;
    __shared__ uint32_t cur[kRange];
    __shared__ uint32_t wsum[16];
    const int r = blockIdx.x, x = blockIdx.y, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t e0 = static_cast<int64_t>(r) * kRange;
    const int nloc = static_cast<int>(min<int64_t>(kRange, catalog - e0));
    const int64_t rb = rbase[static_cast<size_t>(x) * n_ranges + r];
    int64_t *off = tr_off + static_cast<int64_t>(x) * catalog + e0;
    uint32_t c[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int l = tid * kPer + k;
        c[k] = l < nloc ? static_cast<uint32_t>(off[l]) : 0u;
        s += c[k];
    }
    // exclusive scan of the per-thread sums over the workgroup
    uint32_t inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int i = 0; i < w; ++i) pre += wsum[i];
    uint32_t ex = pre + inc - s;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int l = tid * kPer + k;
        cur[l] = ex;
        if (l < nloc) off[l] = rb + ex;
        ex += c[k];
    }
    __syncthreads();
    const int b0 = x * slice_blocks, b1 = min(n_blocks, b0 + slice_blocks);
    for (int b = b0; b < b1; ++b) {
        const size_t sidx = (static_cast<size_t>(b) * n_ranges + r) * kGroups + w;
        const int64_t sb = seg_base[sidx];
        const int run = seg_run[sidx];
        const uint32_t tbase = static_cast<uint32_t>(b - b0) * static_cast<uint32_t>(tb) +
                               static_cast<uint32_t>(w) * static_cast<uint32_t>(tg);
        int t = lane_start[sidx * kWave + lane];
        for (int s4 = 0; s4 < run; s4 += 4) {
            const uint2 q = *reinterpret_cast<const uint2 *>(code + code_slot(sb, s4, lane));
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t cd = ((h < 2 ? q.x : q.y) >> (16 * (h & 1))) & 0xFFFFu;
                t += static_cast<int>(cd >> 15);
                if (cd != kSkip) {
                    const uint32_t pos = atomicAdd(&cur[cd & (kRange - 1)], 1u);
                    tr_ent[rb + pos] = tbase + static_cast<uint32_t>(t);
                }
            }
        }
    }
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_yet_prepare_bytes(int64_t n_trials, int64_t nnz, int32_t catalog, uint32_t flags,
                                         size_t *bytes) {
    if (!bytes) return fail(ARA_E_INVAL, "ara_yet_prepare_bytes: null output");
    if (n_trials < 0 || nnz < 0 || catalog <= 0) return fail(ARA_E_INVAL, "ara_yet_prepare_bytes: negative size");
    if (catalog > ARA_MAX_CATALOG) return fail(ARA_E_LIMIT, "catalog exceeds ARA_MAX_CATALOG");
    if (flags & ~kPrepFlags) return fail(ARA_E_INVAL, "ara_yet_prepare_bytes: unknown flag");
    *bytes = prepare_bytes(geometry(n_trials, catalog), n_trials, nnz, catalog, flags);
    return ARA_OK;
}

extern "C" int32_t ara_yet_prepare(const int64_t *offsets, const int32_t *ids, int64_t n_trials, int32_t catalog,
                                   uint32_t flags, void *buf, size_t buf_bytes, void *stream, ara_yet *out) {
    if (!offsets || !buf || !out) return fail(ARA_E_INVAL, "ara_yet_prepare: null pointer");
    if (n_trials < 0 || catalog <= 0) return fail(ARA_E_INVAL, "ara_yet_prepare: bad size");
    if (catalog > ARA_MAX_CATALOG) return fail(ARA_E_LIMIT, "catalog exceeds ARA_MAX_CATALOG");
    if (flags & ~kPrepFlags) return fail(ARA_E_INVAL, "ara_yet_prepare: unknown flag");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Geometry g = geometry(n_trials, catalog);
    int64_t ends[2] = {0, 0};
    ARA_HIP(hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipMemcpyAsync(&ends[1], offsets + n_trials, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] < 0) return fail(ARA_E_RANGE, "offsets[0] must be 0 and offsets[n] >= 0");
    const int64_t nnz = ends[1];
    if (nnz > 0 && !ids) return fail(ARA_E_INVAL, "ara_yet_prepare: null ids");
    if (buf_bytes < prepare_bytes(g, n_trials, nnz, catalog, flags)) return fail(ARA_E_NOSPACE, "ara_yet_prepare: buffer too small");

    Carver c(buf);
    uint16_t *code = c.take<uint16_t>(static_cast<size_t>(max_codes(g, nnz)) + kPadCodes);
    int64_t *seg_base = c.take<int64_t>(g.nseg);
    int32_t *seg_run = c.take<int32_t>(g.nseg);
    uint8_t *lane_start = c.take<uint8_t>(g.nseg * kWave);
    int64_t *misc = c.take<int64_t>(32);   // [0] error (int32), [1] max occurrences (int32), [2] events
    int32_t *err = reinterpret_cast<int32_t *>(misc);
    int32_t *max_occ = reinterpret_cast<int32_t *>(misc + 1);
    unsigned long long *events = reinterpret_cast<unsigned long long *>(misc + 2);
    const bool transposed = (flags & ARA_PREP_TRANSPOSED) != 0;
    int64_t *tr_off = nullptr, *rtot = nullptr;
    uint32_t *tr_ent = nullptr;
    if (transposed) {
        tr_off = c.take<int64_t>(static_cast<size_t>(kSlices) * catalog + 1);
        tr_ent = c.take<uint32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        rtot = c.take<int64_t>(static_cast<size_t>(kSlices) * g.n_ranges);
    }
    int64_t *t_off = nullptr;
    int32_t *t_ids = nullptr, *t_cnt = nullptr;
    if (flags & ARA_PREP_TRIAL_MAJOR) {
        t_off = c.take<int64_t>(static_cast<size_t>(n_trials) + 1);
        t_ids = c.take<int32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        t_cnt = c.take<int32_t>(static_cast<size_t>(catalog));
        ARA_HIP(hipMemsetAsync(t_cnt, 0, static_cast<size_t>(catalog) * sizeof(int32_t), st));
        if (nnz > 0)
            ARA_HIP(hipMemcpyAsync(t_ids, ids, static_cast<size_t>(nnz) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
    const bool positions = (flags & ARA_PREP_POSITIONS) != 0;
    uint16_t *pos = nullptr;
    if (positions) {
        pos = c.take<uint16_t>(static_cast<size_t>(max_codes(g, nnz)) + kPadCodes);
        if (!t_off) t_off = c.take<int64_t>(static_cast<size_t>(n_trials) + 1);
    }
    if (t_off)
        ARA_HIP(hipMemcpyAsync(t_off, offsets, (static_cast<size_t>(n_trials) + 1) * sizeof(int64_t),
                               hipMemcpyDeviceToDevice, st));
    ARA_HIP(hipMemsetAsync(misc, 0, 32 * sizeof(int64_t), st));
    int32_t *long_trial = positions ? reinterpret_cast<int32_t *>(misc + 3) : nullptr;

    ara_yet y{};
    y.n_trials = n_trials;
    y.nnz = nnz;
    y.catalog = catalog;
    y.range_bits = kRangeBits;
    y.n_ranges = g.n_ranges;
    y.groups = kGroups;
    y.trials_per_group = g.tg;
    y.trials_per_block = g.tb;
    y.n_blocks = g.n_blocks;
    y.code = code;
    y.seg_base = seg_base;
    y.seg_run = seg_run;
    y.lane_start = lane_start;
    y.t_off = t_off;
    y.t_ids = t_ids;
    y.t_cnt = t_cnt;
    y.pos = pos;
    if (transposed) {
        y.n_slices = kSlices;
        y.slice_trials = static_cast<int64_t>(g.slice_blocks) * g.tb;
        y.tr_off = tr_off;
        y.tr_ent = tr_ent;
        // every list is empty until the counting pass has run
        ARA_HIP(hipMemsetAsync(tr_off, 0, (static_cast<size_t>(kSlices) * catalog + 1) * sizeof(int64_t), st));
    }
    if (g.n_blocks == 0) {
        ARA_HIP(hipStreamSynchronize(st));
        *out = y;
        return ARA_OK;
    }
    // pass 1: codes per segment (into seg_run for now)
    k_prep_codes<false><<<g.n_blocks, 1024, 0, st>>>(offsets, ids, n_trials, catalog, g.tg, g.tb, g.n_ranges,
                                                     g.gbits, seg_run, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                     err, long_trial, events);
    ARA_HIP(hipGetLastError());
    std::vector<int32_t> cnt(g.nseg);
    int64_t head[4] = {0, 0, 0, 0};
    ARA_HIP(hipMemcpyAsync(head, misc, sizeof(head), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipMemcpyAsync(cnt.data(), seg_run, g.nseg * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    const int32_t err_h = static_cast<int32_t>(head[0] & 0xffffffff);
    if (err_h) return fail(err_h, "ara_yet_prepare: an event ID lies outside [0, catalog) or offsets decrease");
    if (head[2] != nnz) return fail(ARA_E_RANGE, "ara_yet_prepare: offsets do not cover the IDs consistently");
    if (head[3] != 0) return fail(ARA_E_LIMIT, "ara_yet_prepare: a trial holds more than 65536 occurrences (positions)");

    std::vector<int64_t> base(g.nseg);
    std::vector<int32_t> run(g.nseg);
    int64_t total = 0;
    for (size_t i = 0; i < g.nseg; ++i) {
        run[i] = ((cnt[i] + kWave - 1) / kWave + 3) & ~3;   // codes per lane, a multiple of 4
        base[i] = total;
        total += static_cast<int64_t>(run[i]) * kWave;
    }
    if (total > max_codes(g, nnz)) return fail(ARA_E_LIMIT, "ara_yet_prepare: code bound exceeded");
    ARA_HIP(hipMemcpyAsync(seg_base, base.data(), g.nseg * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(seg_run, run.data(), g.nseg * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // padding, and the block of skip codes after the last code
    ARA_HIP(hipMemsetAsync(code, 0xFF, static_cast<size_t>(total + kPadCodes) * sizeof(uint16_t), st));
    if (pos) ARA_HIP(hipMemsetAsync(pos, 0xFF, static_cast<size_t>(total + kPadCodes) * sizeof(uint16_t), st));
    ARA_HIP(hipMemsetAsync(lane_start, 0, g.nseg * kWave, st));
    // pass 2: the codes themselves
    k_prep_codes<true><<<g.n_blocks, 1024, 0, st>>>(offsets, ids, n_trials, catalog, g.tg, g.tb, g.n_ranges,
                                                    g.gbits, nullptr, seg_base, seg_run, code, lane_start, pos, err,
                                                    nullptr, nullptr);
    ARA_HIP(hipGetLastError());
    ARA_HIP(hipStreamSynchronize(st));   // the host copies of base and run live in this scope
    k_prep_max_occ<<<g.n_ranges, 1024, 0, st>>>(code, seg_base, seg_run, g.n_blocks, g.n_ranges, max_occ, catalog,
                                                t_cnt);
    ARA_HIP(hipGetLastError());
    if (transposed) {
        const dim3 grid(static_cast<unsigned>(g.n_ranges), kSlices);
        k_tr_count<<<grid, 1024, 0, st>>>(code, seg_base, seg_run, g.n_blocks, g.n_ranges, g.slice_blocks, catalog,
                                          tr_off, rtot);
        ARA_HIP(hipGetLastError());
        const size_t nreg = static_cast<size_t>(kSlices) * g.n_ranges;
        std::vector<int64_t> tot(nreg);
        ARA_HIP(hipMemcpyAsync(tot.data(), rtot, nreg * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        ARA_HIP(hipStreamSynchronize(st));
        int64_t acc = 0;
        for (size_t i = 0; i < nreg; ++i) {   // regions in (slice, range) order = list order
            if (tot[i] >= (int64_t(1) << 32))
                return fail(ARA_E_LIMIT, "ara_yet_prepare: 2^32 or more occurrences in one (slice, range)");
            const int64_t t = tot[i];
            tot[i] = acc;
            acc += t;
        }
        if (acc != nnz) return fail(ARA_E_RANGE, "ara_yet_prepare: event-major copy lost occurrences");
        ARA_HIP(hipMemcpyAsync(rtot, tot.data(), nreg * sizeof(int64_t), hipMemcpyHostToDevice, st));
        ARA_HIP(hipMemcpyAsync(tr_off + static_cast<size_t>(kSlices) * catalog, &acc, sizeof(int64_t),
                               hipMemcpyHostToDevice, st));
        ARA_HIP(hipStreamSynchronize(st));   // the host sources live in this scope
        k_tr_scatter<<<grid, 1024, 0, st>>>(code, seg_base, seg_run, lane_start, g.n_blocks, g.n_ranges, g.tg, g.tb,
                                            g.slice_blocks, catalog, rtot, tr_off, tr_ent);
        ARA_HIP(hipGetLastError());
    }
    int32_t mo = 0;
    ARA_HIP(hipMemcpyAsync(&mo, max_occ, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    y.max_occ = mo;
    y.n_codes = total;
    *out = y;
    return ARA_OK;
}
