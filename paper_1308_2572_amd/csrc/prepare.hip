// YET preparation: validate the trials and lay them out by (block of trials,
// catalogue range, trial group) so that the forward and backward kernels can
// keep one range's occurrence table in LDS while streaming.
#include "ara_internal.h"

#include <algorithm>
#include <vector>

namespace ara {

struct Geometry {
    int tg, tb, n_blocks, n_ranges, gbits;
    int slice_blocks;   // blocks per trial slice of the event-major copy
    size_t nseg;
};

static Geometry geometry(int64_t n_trials, int32_t catalog) {
    Geometry g{};
    const int64_t cu = device_cu_count();
    int64_t tg = (n_trials + kGroups * cu - 1) / (kGroups * cu);
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

static size_t prepare_bytes(const Geometry &g, int64_t nnz, int32_t catalog, uint32_t flags) {
    Carver c(nullptr);
    c.take<uint32_t>(static_cast<size_t>(nnz) + g.nseg * (kWave - 1));
    c.take<int64_t>(g.nseg);
    c.take<int32_t>(g.nseg);
    c.take<int32_t>(64);
    if (flags & ARA_PREP_TRANSPOSED) {
        c.take<int64_t>(static_cast<size_t>(kSlices) * catalog + 1);
        c.take<uint32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        c.take<int64_t>(static_cast<size_t>(kSlices) * g.n_ranges);
    }
    return c.bytes();
}

// Count, per (block, range, group), the occurrences whose event lies in the
// range; validate IDs and offsets.
__global__ __launch_bounds__(1024) void k_prep_count(const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ ids, int64_t n_trials,
                                                     int32_t catalog, int tg, int tb, int n_ranges,
                                                     int32_t *__restrict__ cnt, int32_t *__restrict__ err) {
    __shared__ int32_t hist[kGroups * 2048];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kGroups * n_ranges; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int64_t b = blockIdx.x;
    const int64_t t0 = b * tb + static_cast<int64_t>(w) * tg;
    const int64_t t1 = std::min<int64_t>(t0 + tg, n_trials);
    int32_t *h = hist + w * n_ranges;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t o0 = off[t], o1 = off[t + 1];
        if (o1 < o0 || o0 < 0) {
            if (lane == 0) atomicCAS(err, 0, ARA_E_RANGE);
            continue;
        }
        for (int64_t i = o0 + lane; i < o1; i += kWave) {
            const int32_t id = ids[i];
            if (id < 0 || id >= catalog) {
                atomicCAS(err, 0, ARA_E_RANGE);
            } else {
                atomicAdd(&h[id >> kRangeBits], 1);
            }
        }
    }
    // each wave publishes its own row; no other wave touches it
    for (int r = lane; r < n_ranges; r += kWave)
        cnt[(static_cast<size_t>(b) * n_ranges + r) * kGroups + w] = h[r];
}

// Scatter every occurrence into its segment, keeping trial order (and the
// order inside a trial) within each segment.
__global__ __launch_bounds__(1024) void k_prep_scatter(const int64_t *__restrict__ off,
                                                       const int32_t *__restrict__ ids, int64_t n_trials,
                                                       int tg, int tb, int n_ranges, int gbits,
                                                       const int64_t *__restrict__ seg_base,
                                                       const int32_t *__restrict__ seg_run,
                                                       uint32_t *__restrict__ ent) {
    __shared__ int32_t cursor[kGroups * 2048];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int32_t *cur = cursor + w * n_ranges;
    for (int r = lane; r < n_ranges; r += kWave) cur[r] = 0;
    const int64_t b = blockIdx.x;
    const int64_t t0 = b * tb + static_cast<int64_t>(w) * tg;
    const int64_t t1 = std::min<int64_t>(t0 + tg, n_trials);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t o0 = off[t], o1 = off[t + 1];
        const uint32_t tl = static_cast<uint32_t>(t - b * tb);
        for (int64_t base = o0; base < o1; base += kWave) {
            const int64_t i = base + lane;
            const bool active = i < o1;
            const int32_t id = active ? ids[i] : 0;
            const int r = id >> kRangeBits;
            // lanes holding the same range, in lane order (stable multi-split)
            uint64_t peers = __ballot(active);
            for (int bit = 0; bit < gbits; ++bit) {
                const bool on = (r >> bit) & 1;
                const uint64_t m = __ballot(active && on);
                peers &= on ? m : ~m;
            }
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(peers >> 32),
                                                            __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(peers), 0u));
            const int tot = __popcll(peers);
            int32_t c0 = 0;
            if (active) c0 = cur[r];
            __builtin_amdgcn_wave_barrier();
            if (active && rank == 0) cur[r] = c0 + tot;
            if (active) {
                const size_t sidx = (static_cast<size_t>(b) * n_ranges + r) * kGroups + w;
                const int32_t R = seg_run[sidx];
                const int64_t sb = seg_base[sidx];
                const int32_t pos = c0 + static_cast<int32_t>(rank);
                const int32_t lj = pos / R;
                const int32_t step = pos - lj * R;
                ent[sb + static_cast<int64_t>(step) * kWave + lj] =
                    (tl << kRangeBits) | static_cast<uint32_t>(id & (kRange - 1));
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Largest number of occurrences of any single event (bounds the backward's
// fixed-point accumulators).
__global__ __launch_bounds__(1024) void k_prep_max_occ(const uint32_t *__restrict__ ent,
                                                       const int64_t *__restrict__ seg_base,
                                                       const int32_t *__restrict__ seg_run, int n_blocks,
                                                       int n_ranges, int tb, int32_t *__restrict__ max_occ) {
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
                const uint32_t e = ent[sb + i];
                if ((e >> kRangeBits) < static_cast<uint32_t>(tb)) atomicAdd(&hist[e & (kRange - 1)], 1u);
            }
        }
    }
    __syncthreads();
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
__global__ __launch_bounds__(1024) void k_tr_count(const uint32_t *__restrict__ ent,
                                                   const int64_t *__restrict__ seg_base,
                                                   const int32_t *__restrict__ seg_run, int n_blocks, int n_ranges,
                                                   int tb, int slice_blocks, int32_t catalog,
                                                   int64_t *__restrict__ tr_off, int64_t *__restrict__ rtot) {
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
                const uint32_t e = ent[sb + i];
                if ((e >> kRangeBits) < static_cast<uint32_t>(tb)) atomicAdd(&hist[e & (kRange - 1)], 1u);
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
// slice-local trial index into its event's list.
__global__ __launch_bounds__(1024) void k_tr_scatter(const uint32_t *__restrict__ ent,
                                                     const int64_t *__restrict__ seg_base,
                                                     const int32_t *__restrict__ seg_run, int n_blocks, int n_ranges,
                                                     int tb, int slice_blocks, int32_t catalog,
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
    for (int b = b0; b < b1; ++b)
        for (int g = 0; g < kGroups; ++g) {
            const size_t sidx = (static_cast<size_t>(b) * n_ranges + r) * kGroups + g;
            const int64_t sb = seg_base[sidx];
            const int64_t n = static_cast<int64_t>(seg_run[sidx]) * kWave;
            for (int64_t i = tid; i < n; i += blockDim.x) {
                const uint32_t e = ent[sb + i];
                const uint32_t tl = e >> kRangeBits;
                if (tl < static_cast<uint32_t>(tb)) {
                    const uint32_t pos = atomicAdd(&cur[e & (kRange - 1)], 1u);
                    tr_ent[rb + pos] = static_cast<uint32_t>(b - b0) * static_cast<uint32_t>(tb) + tl;
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
    if (flags & ~ARA_PREP_TRANSPOSED) return fail(ARA_E_INVAL, "ara_yet_prepare_bytes: unknown flag");
    *bytes = prepare_bytes(geometry(n_trials, catalog), nnz, catalog, flags);
    return ARA_OK;
}

extern "C" int32_t ara_yet_prepare(const int64_t *offsets, const int32_t *ids, int64_t n_trials, int32_t catalog,
                                   uint32_t flags, void *buf, size_t buf_bytes, void *stream, ara_yet *out) {
    if (!offsets || !buf || !out) return fail(ARA_E_INVAL, "ara_yet_prepare: null pointer");
    if (n_trials < 0 || catalog <= 0) return fail(ARA_E_INVAL, "ara_yet_prepare: bad size");
    if (catalog > ARA_MAX_CATALOG) return fail(ARA_E_LIMIT, "catalog exceeds ARA_MAX_CATALOG");
    if (flags & ~ARA_PREP_TRANSPOSED) return fail(ARA_E_INVAL, "ara_yet_prepare: unknown flag");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Geometry g = geometry(n_trials, catalog);
    int64_t ends[2] = {0, 0};
    ARA_HIP(hipMemcpyAsync(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipMemcpyAsync(&ends[1], offsets + n_trials, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    if (ends[0] != 0 || ends[1] < 0) return fail(ARA_E_RANGE, "offsets[0] must be 0 and offsets[n] >= 0");
    const int64_t nnz = ends[1];
    if (nnz > 0 && !ids) return fail(ARA_E_INVAL, "ara_yet_prepare: null ids");
    if (buf_bytes < prepare_bytes(g, nnz, catalog, flags)) return fail(ARA_E_NOSPACE, "ara_yet_prepare: buffer too small");

    Carver c(buf);
    uint32_t *ent = c.take<uint32_t>(static_cast<size_t>(nnz) + g.nseg * (kWave - 1));
    int64_t *seg_base = c.take<int64_t>(g.nseg);
    int32_t *seg_run = c.take<int32_t>(g.nseg);
    int32_t *misc = c.take<int32_t>(64);   // [0] error, [1] max occurrences
    const bool transposed = (flags & ARA_PREP_TRANSPOSED) != 0;
    int64_t *tr_off = nullptr, *rtot = nullptr;
    uint32_t *tr_ent = nullptr;
    if (transposed) {
        tr_off = c.take<int64_t>(static_cast<size_t>(kSlices) * catalog + 1);
        tr_ent = c.take<uint32_t>(static_cast<size_t>(std::max<int64_t>(nnz, 1)));
        rtot = c.take<int64_t>(static_cast<size_t>(kSlices) * g.n_ranges);
    }
    ARA_HIP(hipMemsetAsync(misc, 0, 64 * sizeof(int32_t), st));

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
    y.ent = ent;
    y.seg_base = seg_base;
    y.seg_run = seg_run;
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
    k_prep_count<<<g.n_blocks, 1024, 0, st>>>(offsets, ids, n_trials, catalog, g.tg, g.tb, g.n_ranges, seg_run, misc);
    ARA_HIP(hipGetLastError());
    std::vector<int32_t> cnt(g.nseg);
    int32_t err = 0;
    ARA_HIP(hipMemcpyAsync(&err, misc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipMemcpyAsync(cnt.data(), seg_run, g.nseg * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    if (err) return fail(err, "ara_yet_prepare: an event ID lies outside [0, catalog) or offsets decrease");

    std::vector<int64_t> base(g.nseg);
    std::vector<int32_t> run(g.nseg);
    int64_t total = 0, counted = 0;
    for (size_t i = 0; i < g.nseg; ++i) {
        run[i] = (cnt[i] + kWave - 1) / kWave;
        base[i] = total;
        total += static_cast<int64_t>(run[i]) * kWave;
        counted += cnt[i];
    }
    if (counted != nnz) return fail(ARA_E_RANGE, "ara_yet_prepare: offsets do not cover the IDs consistently");
    ARA_HIP(hipMemcpyAsync(seg_base, base.data(), g.nseg * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ARA_HIP(hipMemcpyAsync(seg_run, run.data(), g.nseg * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // padding entries name trial slot `tb` (one past the block) and event 0 of
    // their range: harmless to every consumer, so no sentinel test is needed
    if (total > 0)
        ARA_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(ent), static_cast<int>(pad_entry(g.tb)),
                                  static_cast<size_t>(total), st));
    k_prep_scatter<<<g.n_blocks, 1024, 0, st>>>(offsets, ids, n_trials, g.tg, g.tb, g.n_ranges, g.gbits, seg_base,
                                                seg_run, ent);
    ARA_HIP(hipGetLastError());
    k_prep_max_occ<<<g.n_ranges, 1024, 0, st>>>(ent, seg_base, seg_run, g.n_blocks, g.n_ranges, g.tb, misc + 1);
    ARA_HIP(hipGetLastError());
    if (transposed) {
        const dim3 grid(static_cast<unsigned>(g.n_ranges), kSlices);
        k_tr_count<<<grid, 1024, 0, st>>>(ent, seg_base, seg_run, g.n_blocks, g.n_ranges, g.tb, g.slice_blocks,
                                          catalog, tr_off, rtot);
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
        k_tr_scatter<<<grid, 1024, 0, st>>>(ent, seg_base, seg_run, g.n_blocks, g.n_ranges, g.tb, g.slice_blocks,
                                            catalog, rtot, tr_off, tr_ent);
        ARA_HIP(hipGetLastError());
    }
    int32_t mo = 0;
    ARA_HIP(hipMemcpyAsync(&mo, misc + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    y.max_occ = mo;
    y.n_entries = total;
    *out = y;
    return ARA_OK;
}
