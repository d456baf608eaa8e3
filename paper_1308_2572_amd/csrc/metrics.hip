// Tail metrics of the YLT: mean annual loss, PML_p (the r-th largest year
// loss) and TVaR_p (mean of the r largest), r = N - floor(p*N + 1e-9).
//
// Selection is a radix select on the binary64 bit patterns (year losses are
// >= 0, so the unsigned order of the bits is the numeric order), with digits
// of 11 bits from the top.  Two grid passes histogram the exponent and the
// leading mantissa digit; a third gathers every value sharing that 23-bit
// prefix, and the workgroup that finishes it last selects among them (in LDS
// when they fit, from the gathered copy otherwise, at once when they are all
// equal).  The same pass sums and counts the values above that bin, and its
// last workgroup adds the gathered values above the PML value exactly (as
// integers: they share one exponent) and writes the metrics.  Each pass ends
// in the workgroup that finishes last (a counter per layer), so a call is
// three kernels whatever the ties.  Sums use a fixed partition of the trials,
// fixed-order trees and exact integer sums, so every result is deterministic.
//
// A launch serves several rows (blockIdx.y): the layers of one call, rows of
// one length in one workspace, or a list of rows each with its own length,
// rank and workspace (the quote server's quotes finishing together).
#include "ara_internal.h"
#include "wave.h"

#include <algorithm>
#include <cmath>

namespace ara {

constexpr int kMetThreads = 1024;
constexpr int kMetUnroll = 8;                          // values per thread per sweep (loads in flight together)
constexpr int kMetSweep = kMetThreads * kMetUnroll;
constexpr int kBins = 2048;
constexpr int kDigits = 6;
constexpr int kCandCap = 16384;     // gathered values selected inside LDS
// digit d covers bits [kShift[d], kShift[d] + kWidth[d]) of the key; bit 63
// (the sign) is 0 for every year loss
__constant__ int kShift[kDigits] = {52, 41, 30, 19, 8, 0};
__constant__ int kWidth[kDigits] = {11, 11, 11, 11, 11, 8};

struct MetState {
    uint64_t prefix[3];        // bits fixed before digit d = 0, 1, 2 (prefix[d] = key >> (kShift[d-1]))
    int64_t need[3];           // rank (1-based from the top) to find among values with prefix[d]
    unsigned long long cand_n; // values gathered
    unsigned long long kmax;   // largest gathered key
    unsigned long long kminc;  // complement of the smallest gathered key
    double thr;                // the PML value
    int64_t cnt_gt, cnt_eq;
    int64_t r;
    uint32_t tick[3];          // workgroups finished, per pass
};

struct MetPart {
    double sum, sum_gt;
    int64_t cnt_gt;
    uint64_t kmax;     // the largest gathered key of the workgroup
    int64_t n_kmax;    // how many of its gathered keys equal it
};

// The rows of a launch: `rows` lists rows of their own (MetRow, declared with
// the internal interface), or, when it is null, n_rows rows of length n laid
// out one after another in one workspace.
struct MetCall {
    const MetRow *rows;
    const double *ylt;
    double *out, *w;
    int64_t n, r;
    int32_t nwg, n_rows;
    uint32_t *hist;
    MetState *st;
    MetPart *part;
    uint64_t *cand;
};

__device__ __forceinline__ MetRow met_row(const MetCall &c, int l) {
    if (c.rows) return c.rows[l];
    MetRow m;
    m.ylt = c.ylt + static_cast<size_t>(l) * c.n;
    m.out = c.out + 3 * l;
    m.w = c.w ? c.w + static_cast<size_t>(l) * c.n : nullptr;
    m.wstride = static_cast<int64_t>(c.n_rows) * c.n;
    m.n = c.n;
    m.r = c.r;
    m.nwg = c.nwg;
    m.pad = 0;
    m.hist = c.hist + static_cast<size_t>(l) * 2 * kBins;
    m.st = reinterpret_cast<char *>(c.st + l);
    m.part = reinterpret_cast<char *>(c.part + static_cast<size_t>(l) * c.nwg);
    m.cand = c.cand + static_cast<size_t>(l) * c.n;
    return m;
}

__device__ __forceinline__ uint64_t key_of(double y) {
    return (y == 0.0) ? 0ull : static_cast<uint64_t>(__double_as_longlong(y));
}

__device__ __forceinline__ void chunk_of(int64_t n, int nwg, int wg, int64_t &lo, int64_t &hi) {
    const int64_t c = (n + nwg - 1) / nwg;
    lo = std::min<int64_t>(n, static_cast<int64_t>(wg) * c);
    hi = std::min<int64_t>(n, lo + c);
}

// Workgroup sums of K binary64 values per thread (counts below 2^53 are
// exact as binary64), each in a fixed order: a DPP prefix sum within every
// wavefront, then one over the 16 wavefront totals, which every wavefront
// forms for itself.  All threads return the sums.  red: [K][16].
template <int K>
__device__ void block_sums(double (&v)[K], double (*red)[16]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_inclusive_sum(v[k]);
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = lane63(wave_inclusive_sum(lane < kMetThreads / 64 ? red[k][lane] : 0.0));
    __syncthreads();   // red may be reused
}

// Values one workgroup hands to the one that finishes last go through
// device-scope atomic stores and loads, which need no cache write-back or
// invalidation.
template <class T>
__device__ __forceinline__ void put(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T get(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in the workgroup that finishes pass k of layer l last.  Every wave
// waits for its own stores and atomics to complete before the workgroup
// counts itself done, and the last one reads only after its count returned,
// so it sees all the values handed over.
__device__ bool finished_last(MetState &S, int k, int nwg, int *flag) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) *flag = atomicAdd(&S.tick[k], 1u) == static_cast<uint32_t>(nwg - 1);
    __syncthreads();
    return *flag != 0;
}

struct FindShared {
    double wtot[16];
    int digit;
    int64_t need;
};

// Locate the bin holding the need-th largest value (counting from the top) in
// histogram h[0..bins); every thread of the block takes part (1024 threads,
// two bins each).  Result in fs.digit / fs.need (the rank inside that bin).
// Counts are summed as binary64, exact below 2^53.
__device__ void find_digit(const uint32_t *h, int bins, int64_t need, FindShared &fs) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) {   // defaults (never used when the histogram holds `need` values)
        fs.digit = 0;
        fs.need = 1;
    }
    const int64_t c_lo = (2 * t < bins) ? h[2 * t] : 0;
    const int64_t c_hi = (2 * t + 1 < bins) ? h[2 * t + 1] : 0;
    const int64_t v = c_lo + c_hi;
    const double incl = wave_inclusive_sum(static_cast<double>(v));   // lanes <= this one
    const double wsum = lane63(incl);
    if (lane == 63) fs.wtot[w] = incl;
    __syncthreads();
    // totals of the wavefronts after this one
    const double wp = wave_inclusive_sum(lane < kMetThreads / 64 ? fs.wtot[lane] : 0.0);
    const double all = lane63(wp);
    const double upto = __shfl(wp, w);   // wavefronts 0..w
    const int64_t above = static_cast<int64_t>((all - upto) + (wsum - incl));   // values in bins above 2t+1
    if (above < need && need <= above + c_hi) {
        fs.digit = 2 * t + 1;
        fs.need = need - above;
    } else if (above + c_hi < need && need <= above + v) {
        fs.digit = 2 * t;
        fs.need = need - above - c_hi;
    }
    __syncthreads();
}

// Digit pass d (0 or 1) over the whole YLT row: histogram of digit d among
// the values whose higher bits equal the prefix selected so far.  Pass 0 also
// forms the fixed-partition partial sums for the mean.  The last workgroup
// selects the digit for the next pass.
__global__ __launch_bounds__(kMetThreads) void k_met_hist(MetCall call, int d) {
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    __shared__ double red[1][16];
    __shared__ int flag;
    const int wg = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const MetRow R = met_row(call, blockIdx.y);
    if (wg >= R.nwg) return;   // uniform over the workgroup, before any barrier
    const int64_t n = R.n, r = R.r;
    const int nwg = R.nwg;
    MetState &S = *reinterpret_cast<MetState *>(R.st);
    const uint64_t prefix = d ? S.prefix[1] : 0ull;
    for (int i = tid; i < kBins; i += kMetThreads) h[i] = 0;
    __syncthreads();
    const int sh = kShift[d], hb = kShift[d] + kWidth[d];
    const uint32_t mask = (1u << kWidth[d]) - 1u;
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = R.ylt;
    double s = 0.0;
    for (int64_t i0 = lo; i0 < hi; i0 += kMetSweep) {   // uniform trip count: every lane reaches the ballots
        double v[kMetUnroll];
#pragma unroll
        for (int u = 0; u < kMetUnroll; ++u) {
            const int64_t i = i0 + u * kMetThreads + tid;
            v[u] = (i < hi) ? y[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMetUnroll; ++u) {
            const int64_t i = i0 + u * kMetThreads + tid;
            const uint64_t k = key_of(v[u]);
            if (d == 0) s += v[u];
            const bool want = i < hi && (k >> hb) == prefix;
            const uint32_t dg = static_cast<uint32_t>((k >> sh) & mask);
            // year losses of one row crowd into few digits (the exponent above
            // all): the first lane's digit is counted for all the lanes that
            // share it with one LDS atomic, the rest count themselves
            const uint64_t act = __ballot(want);
            if (act) {
                const int leader = __builtin_ctzll(act);
                const uint32_t ld = __builtin_amdgcn_readlane(dg, leader);
                const uint64_t same = __ballot(want && dg == ld);
                if (lane == leader) atomicAdd(&h[ld], static_cast<uint32_t>(__popcll(same)));
                if (want && dg != ld) atomicAdd(&h[dg], 1u);
            }
        }
    }
    if (d == 0) {
        double t[1] = {s};
        block_sums(t, red);
        if (tid == 0) reinterpret_cast<MetPart *>(R.part)[wg].sum = t[0];
    }
    __syncthreads();
    uint32_t *hd = R.hist + static_cast<size_t>(d) * kBins;
    for (int i = tid; i < kBins; i += kMetThreads)
        if (h[i]) atomicAdd(&hd[i], h[i]);
    if (!finished_last(S, d, nwg, &flag)) return;
    for (int i = tid; i < kBins; i += kMetThreads) h[i] = get(&hd[i]);
    __syncthreads();
    find_digit(h, 1 << kWidth[d], d ? S.need[1] : r, fs);
    if (tid == 0) {
        S.prefix[d + 1] = (prefix << kWidth[d]) | static_cast<uint64_t>(fs.digit);
        S.need[d + 1] = fs.need;
        if (d == 0) S.r = r;
    }
}

// Visits the gathered keys [0, cn) of one workgroup's walk, from LDS or from
// the global copy, kMetUnroll per thread and sweep so that the global reads
// are in flight together; f(valid, key) runs on every lane (uniform trip
// count, so f may hold ballots).
template <class F>
__device__ __forceinline__ void each_cand(bool in_lds, const uint64_t *cs, const uint64_t *c, int64_t cn, F f) {
    for (int64_t i0 = 0; i0 < cn; i0 += kMetSweep) {
        uint64_t u[kMetUnroll];
#pragma unroll
        for (int q = 0; q < kMetUnroll; ++q) {
            const int64_t i = i0 + q * kMetThreads + threadIdx.x;
            u[q] = i < cn ? (in_lds ? cs[i] : get(&c[i])) : 0ull;
        }
#pragma unroll
        for (int q = 0; q < kMetUnroll; ++q) f(i0 + q * kMetThreads + threadIdx.x < cn, u[q]);
    }
}

// Gathers every value whose 23-bit prefix is the selected one (a wavefront
// reserves its slots with one atomic), with their smallest and largest key.
// The last workgroup finishes digits 2..5 on them.
__global__ __launch_bounds__(kMetThreads) void k_met_collect(MetCall call) {
    __shared__ uint64_t cs[kCandCap];
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    __shared__ double red[4][16];
    __shared__ unsigned long long ired[4][16];
    __shared__ unsigned long long wkm[kMetThreads / 64];
    __shared__ long long wkn[kMetThreads / 64];
    __shared__ int flag;
    const int wg = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const MetRow R = met_row(call, blockIdx.y);
    if (wg >= R.nwg) return;   // uniform over the workgroup, before any barrier
    const int64_t n = R.n;
    const int nwg = R.nwg;
    MetState &S = *reinterpret_cast<MetState *>(R.st);
    MetPart *const part = reinterpret_cast<MetPart *>(R.part);
    const uint64_t prefix = S.prefix[2];
    double s_above = 0.0;   // values above the bin (all above the PML value)
    int64_t n_above = 0;
    const int hb = kShift[1];
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = R.ylt;
    uint64_t *c = R.cand;
    uint64_t kmin = ~0ull, kmax = 0ull;
    int64_t nkmax = 0;   // this lane's gathered keys equal to its kmax
    for (int64_t i0 = lo; i0 < hi; i0 += kMetSweep) {
        uint64_t k[kMetUnroll], m[kMetUnroll];
        int64_t mine = 0;
#pragma unroll
        for (int u = 0; u < kMetUnroll; ++u) {
            const int64_t i = i0 + u * kMetThreads + tid;
            k[u] = (i < hi) ? key_of(y[i]) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kMetUnroll; ++u) {
            const int64_t i = i0 + u * kMetThreads + tid;
            const bool is = i < hi && (k[u] >> hb) == prefix;
            if (i < hi && (k[u] >> hb) > prefix) {
                s_above += __longlong_as_double(static_cast<long long>(k[u]));
                ++n_above;
            }
            m[u] = __ballot(is);
            mine += __popcll(m[u]);
            if (is) {
                kmin = std::min(kmin, k[u]);
                if (nkmax == 0 || k[u] > kmax) {
                    kmax = k[u];
                    nkmax = 1;
                } else if (k[u] == kmax) {
                    ++nkmax;
                }
            }
        }
        if (mine) {   // uniform: the wavefront reserves its slots itself
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&S.cand_n, static_cast<unsigned long long>(mine));
            int64_t off = static_cast<int64_t>(__shfl(base, 0));
#pragma unroll
            for (int u = 0; u < kMetUnroll; ++u) {
                if ((m[u] >> lane) & 1ull) {
                    const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m[u] >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m[u]), 0u));
                    put(&c[off + pos], k[u]);
                }
                off += __popcll(m[u]);
            }
        }
    }
    unsigned long long wk = 0ull;   // the wavefront's largest gathered key and its count
    long long wn = 0;
    if (__ballot(nkmax > 0)) {   // uniform: this wavefront gathered something
        const uint64_t my_kmax = kmax;
        for (int o = 32; o > 0; o >>= 1) {
            kmin = std::min(kmin, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(kmin), o)));
            kmax = std::max(kmax, static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(kmax), o)));
        }
        wk = kmax;
        wn = (nkmax > 0 && my_kmax == kmax) ? nkmax : 0;
        for (int o = 32; o > 0; o >>= 1) wn += __shfl_xor(wn, o);
        if (lane == 0) {
            atomicMax(&S.kmax, static_cast<unsigned long long>(kmax));
            atomicMax(&S.kminc, static_cast<unsigned long long>(~kmin));
        }
    }
    if (lane == 0) {
        wkm[tid >> 6] = wk;
        wkn[tid >> 6] = wn;
    }
    {
        double t2[2] = {s_above, static_cast<double>(n_above)};
        block_sums(t2, red);   // also publishes wkm and wkn
        if (tid == 0) {
            MetPart *pw = part + wg;
            put(&pw->sum_gt, t2[0]);
            put(&pw->cnt_gt, static_cast<int64_t>(t2[1]));
            unsigned long long km = 0ull;
            long long kn = 0;
            for (int i = 0; i < kMetThreads / 64; ++i) km = wkm[i] > km ? wkm[i] : km;
            for (int i = 0; i < kMetThreads / 64; ++i) kn += wkm[i] == km ? wkn[i] : 0;
            put(&pw->kmax, static_cast<uint64_t>(km));
            put(&pw->n_kmax, static_cast<int64_t>(kn));
        }
    }
    if (!finished_last(S, 2, nwg, &flag)) return;
    const int64_t cn = static_cast<int64_t>(get(&S.cand_n));
    const uint64_t lo_key = ~static_cast<uint64_t>(get(&S.kminc)), hi_key = static_cast<uint64_t>(get(&S.kmax));
    uint64_t bits = hi_key;
    // how many gathered keys equal the largest: when they reach the rank
    // sought inside the bin (values capped at one limit crowd the top), that
    // key is the PML and no pass over the gathered copy is needed (asked only
    // when the keys do not fit in LDS, where the passes are cheap)
    int64_t n_top = 0;
    if (lo_key != hi_key && cn > kCandCap) {   // uniform
        long long v = 0;
        const MetPart *pl = part;
        for (int i = tid; i < nwg; i += kMetThreads)
            if (get(&pl[i].kmax) == hi_key) v += get(&pl[i].n_kmax);
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wkn[tid >> 6] = v;
        __syncthreads();
        for (int i = 0; i < kMetThreads / 64; ++i) n_top += wkn[i];
        __syncthreads();
    }
    const bool top_tied = lo_key != hi_key && n_top >= S.need[2];   // uniform
    if (lo_key != hi_key && !top_tied) {
        // the values differ: radix select on the gathered copy
        const bool in_lds = cn <= kCandCap;   // uniform
        if (in_lds)
            for (int64_t i = tid; i < cn; i += kMetThreads) cs[i] = get(&c[i]);
        uint64_t pre = prefix;
        int64_t need = S.need[2];
        for (int d = 2; d < kDigits; ++d) {
            for (int i = tid; i < kBins; i += kMetThreads) h[i] = 0;
            __syncthreads();
            const int sh = kShift[d], hbd = kShift[d] + kWidth[d];
            const uint32_t mask = (1u << kWidth[d]) - 1u;
            if (in_lds) {
                for (int64_t i = tid; i < cn; i += kMetThreads) {
                    const uint64_t u = cs[i];
                    if ((u >> hbd) == pre) atomicAdd(&h[(u >> sh) & mask], 1u);
                }
            } else each_cand(false, cs, c, cn, [&](bool valid, uint64_t u) {
                const bool want = valid && (u >> hbd) == pre;
                const uint32_t dg = static_cast<uint32_t>((u >> sh) & mask);
                // tied keys crowd one digit: the first lane's digit is counted
                // for all the lanes that share it with one LDS atomic
                const uint64_t act = __ballot(want);
                if (act) {
                    const int leader = __builtin_ctzll(act);
                    const uint32_t ld = __builtin_amdgcn_readlane(dg, leader);
                    const uint64_t same = __ballot(want && dg == ld);
                    if (lane == leader) atomicAdd(&h[ld], static_cast<uint32_t>(__popcll(same)));
                    if (want && dg != ld) atomicAdd(&h[dg], 1u);
                }
            });
            __syncthreads();
            find_digit(h, 1 << kWidth[d], need, fs);
            pre = (pre << kWidth[d]) | static_cast<uint64_t>(fs.digit);
            need = fs.need;
        }
        bits = pre;
    }
    const double thr = __longlong_as_double(static_cast<long long>(bits));
    // the gathered values above the PML value, summed exactly: they share one
    // exponent, so their 53-bit significands add as integers (in halves of 27
    // and 26 bits, any order), and those equal to it, counted
    unsigned long long sig_hi = 0, sig_lo = 0, c_gt = 0, c_eq = 0;
    if (lo_key == hi_key) {
        if (tid == 0) c_eq = static_cast<unsigned long long>(cn);
    } else if (top_tied) {
        if (tid == 0) c_eq = static_cast<unsigned long long>(n_top);   // none above it in the bin
    } else {
        const bool in_lds = cn <= kCandCap;   // uniform; the copy in LDS is still there
        auto add = [&](bool valid, uint64_t u) {
            if (!valid) return;
            if (u > bits) {
                const uint64_t e = (u >> 52) & 0x7FFull;
                const uint64_t sig = (u & ((1ull << 52) - 1ull)) | (e ? (1ull << 52) : 0ull);
                sig_hi += sig >> 26;
                sig_lo += sig & ((1ull << 26) - 1ull);
                ++c_gt;
            } else if (u == bits) {
                ++c_eq;
            }
        };
        if (in_lds) {
            for (int64_t i = tid; i < cn; i += kMetThreads) add(true, cs[i]);
        } else {
            each_cand(false, cs, c, cn, add);
        }
    }
    {   // integer sums: any order gives the same totals
        unsigned long long v[4] = {sig_hi, sig_lo, c_gt, c_eq};
        const int w = tid >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
            if (lane == 0) ired[q][w] = v[q];
        }
        __syncthreads();
        if (tid == 0) {
            sig_hi = sig_lo = c_gt = c_eq = 0;
            for (int i = 0; i < kMetThreads / 64; ++i) {
                sig_hi += ired[0][i];
                sig_lo += ired[1][i];
                c_gt += ired[2][i];
                c_eq += ired[3][i];
            }
        }
        __syncthreads();
    }
    // the sums over the workgroups, in a fixed order
    MetPart *pl = part;
    double t4[3] = {0.0, 0.0, 0.0};
    for (int i = tid; i < nwg; i += kMetThreads) {
        t4[0] += pl[i].sum;   // written by an earlier kernel
        t4[1] += get(&pl[i].sum_gt);
        t4[2] += static_cast<double>(get(&pl[i].cnt_gt));
    }
    block_sums(t4, red);
    if (tid == 0) {
        const int e = static_cast<int>((prefix >> 11) & 0x7FFu);   // the bin's exponent field
        const double scale = ldexp(1.0, (e ? e : 1) - 1075);        // value of one significand unit
        const double cand_sum = (ldexp(static_cast<double>(sig_hi), 26) + static_cast<double>(sig_lo)) * scale;
        const int64_t r = S.r;
        const int64_t tgt = static_cast<int64_t>(t4[2]) + static_cast<int64_t>(c_gt);
        const double tsg = t4[1] + cand_sum;
        S.thr = thr;
        S.cnt_gt = tgt;
        S.cnt_eq = static_cast<int64_t>(c_eq);
        R.out[0] = t4[0] / static_cast<double>(n);
        R.out[1] = thr;
        R.out[2] = (tsg + static_cast<double>(r - tgt) * thr) / static_cast<double>(r);
    }
}

__global__ void k_met_weights(MetCall call) {
    const MetRow R = met_row(call, blockIdx.y);
    if (!R.w) return;
    const MetState &S = *reinterpret_cast<const MetState *>(R.st);
    const int64_t n = R.n;
    const double thr = S.thr;
    const int64_t r = S.r, gt = S.cnt_gt, eq = S.cnt_eq;
    const double inv_n = 1.0 / static_cast<double>(n);
    const double w_pml = 1.0 / static_cast<double>(eq);
    const double w_gt = 1.0 / static_cast<double>(r);
    const double w_eq = static_cast<double>(r - gt) / (static_cast<double>(r) * static_cast<double>(eq));
    const double *y = R.ylt;
    double *wa = R.w, *wp = R.w + R.wstride, *wt = R.w + 2 * R.wstride;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double v = y[i];
        wa[i] = inv_n;
        wp[i] = (v == thr) ? w_pml : 0.0;
        wt[i] = (v > thr) ? w_gt : ((v == thr) ? w_eq : 0.0);
    }
}

__global__ void k_met_vjp(const double *__restrict__ w, int64_t n, int n_layers, const double *__restrict__ g,
                          double *__restrict__ out) {
    const int l = blockIdx.y;
    const double g0 = g[3 * l + 0], g1 = g[3 * l + 1], g2 = g[3 * l + 2];
    const double *wa = w + (static_cast<size_t>(0) * n_layers + l) * n;
    const double *wp = w + (static_cast<size_t>(1) * n_layers + l) * n;
    const double *wt = w + (static_cast<size_t>(2) * n_layers + l) * n;
    double *o = out + static_cast<size_t>(l) * n;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        o[i] = (g0 * wa[i] + g1 * wp[i]) + g2 * wt[i];
}

static int met_nwg(int64_t n) {
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + kMetSweep - 1) / kMetSweep, 1024)));
}

static int64_t met_rank(int64_t n, double p) {
    const int64_t r = n - static_cast<int64_t>(std::floor(p * static_cast<double>(n) + 1e-9));
    return std::max<int64_t>(1, std::min<int64_t>(n, r));
}

// Clears each listed row's histograms and selection state.
__global__ __launch_bounds__(256) void k_met_clear(MetCall call) {
    const MetRow R = met_row(call, blockIdx.y);
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) R.hist[i] = 0;
    uint32_t *sw = reinterpret_cast<uint32_t *>(R.st);
    for (int i = threadIdx.x; i < static_cast<int>(sizeof(MetState) / 4); i += blockDim.x) sw[i] = 0;
}

static void met_launch(const MetCall &call, int max_nwg, int64_t max_n, bool weights, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>(max_nwg), static_cast<unsigned>(call.n_rows));
    k_met_hist<<<grid, kMetThreads, 0, st>>>(call, 0);
    k_met_hist<<<grid, kMetThreads, 0, st>>>(call, 1);
    k_met_collect<<<grid, kMetThreads, 0, st>>>(call);
    if (weights) {
        const unsigned gx = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((max_n + 255) / 256, 4096)));
        k_met_weights<<<dim3(gx, static_cast<unsigned>(call.n_rows)), 256, 0, st>>>(call);
    }
}

static size_t met_bytes(int32_t L, int64_t n) {
    const int nwg = met_nwg(n);
    Carver c(nullptr);
    c.take<int32_t>(kWsHeaderBytes / 4);
    c.take<uint32_t>(static_cast<size_t>(2) * L * kBins);
    c.take<MetState>(static_cast<size_t>(L));
    c.take<MetPart>(static_cast<size_t>(L) * nwg);
    c.take<uint64_t>(static_cast<size_t>(L) * n);   // gathered keys: up to the whole row
    return c.bytes();
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_metrics_workspace_bytes(int32_t n_layers, int64_t n, size_t *bytes) {
    if (!bytes || n_layers < 0 || n < 0) return fail(ARA_E_INVAL, "ara_metrics_workspace_bytes: bad argument");
    *bytes = met_bytes(n_layers, n);
    return ARA_OK;
}

extern "C" int32_t ara_metrics(const double *ylt, int32_t n_layers, int64_t n, double p, double *out, double *weights,
                               void *ws, size_t ws_bytes, void *stream) {
    if (n_layers < 0 || n <= 0) return fail(ARA_E_INVAL, "ara_metrics: need n > 0 trials");
    if (n_layers > ARA_MAX_LAYERS) return fail(ARA_E_LIMIT, "ara_metrics: more than ARA_MAX_LAYERS rows");
    if (!(p > 0.0 && p < 1.0)) return fail(ARA_E_INVAL, "ara_metrics: p must lie in (0, 1)");
    if (!ws || (n_layers > 0 && (!ylt || !out))) return fail(ARA_E_INVAL, "ara_metrics: null pointer");
    if (ws_bytes < met_bytes(n_layers, n)) return fail(ARA_E_NOSPACE, "ara_metrics: workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nwg = met_nwg(n);
    Carver c(ws);
    int32_t *hdr = c.take<int32_t>(kWsHeaderBytes / 4);
    uint32_t *hist = c.take<uint32_t>(static_cast<size_t>(2) * n_layers * kBins);
    MetState *state = c.take<MetState>(static_cast<size_t>(n_layers));
    MetPart *part = c.take<MetPart>(static_cast<size_t>(n_layers) * nwg);
    uint64_t *cand = c.take<uint64_t>(static_cast<size_t>(n_layers) * n);
    // header, histograms and states are contiguous: clear them at once
    const size_t clear = reinterpret_cast<char *>(part) - reinterpret_cast<char *>(hdr);
    ARA_HIP(hipMemsetAsync(hdr, 0, clear, st));
    if (n_layers == 0) return ARA_OK;
    MetCall call{};
    call.ylt = ylt;
    call.out = out;
    call.w = weights;
    call.n = n;
    call.r = met_rank(n, p);
    call.nwg = nwg;
    call.n_rows = n_layers;
    call.hist = hist;
    call.st = state;
    call.part = part;
    call.cand = cand;
    ProfScope prof(ARA_PROF_METRICS, st);
    met_launch(call, nwg, n, weights != nullptr, st);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

namespace ara {

MetRow metrics_row(void *ws, const double *ylt, int64_t n, double p, double *out, double *w) {
    const int nwg = met_nwg(n);
    Carver c(ws);   // the layout of a one-row ara_metrics workspace
    c.take<int32_t>(kWsHeaderBytes / 4);
    MetRow m{};
    m.hist = c.take<uint32_t>(static_cast<size_t>(2) * kBins);
    m.st = c.take<MetState>(1);
    m.part = c.take<MetPart>(static_cast<size_t>(nwg));
    m.cand = c.take<uint64_t>(static_cast<size_t>(n));
    m.ylt = ylt;
    m.out = out;
    m.w = w;
    m.wstride = n;
    m.n = n;
    m.r = met_rank(n, p);
    m.nwg = nwg;
    return m;
}

int32_t metrics_rows(const MetRow *d_rows, int n_rows, int max_nwg, int64_t max_n, bool any_weights, hipStream_t st) {
    if (n_rows <= 0) return ARA_OK;
    MetCall call{};
    call.rows = d_rows;
    call.n_rows = n_rows;
    ProfScope prof(ARA_PROF_METRICS, st);
    k_met_clear<<<dim3(1, static_cast<unsigned>(n_rows)), 256, 0, st>>>(call);
    met_launch(call, max_nwg, max_n, any_weights, st);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

}  // namespace ara

extern "C" int32_t ara_metrics_vjp(const double *weights, int32_t n_layers, int64_t n, const double *grad_out,
                                   double *grad_ylt, void *stream) {
    if (n_layers < 0 || n < 0) return fail(ARA_E_INVAL, "ara_metrics_vjp: bad size");
    if (n_layers > ARA_MAX_LAYERS) return fail(ARA_E_LIMIT, "ara_metrics_vjp: more than ARA_MAX_LAYERS rows");
    if (n_layers == 0 || n == 0) return ARA_OK;
    if (!weights || !grad_out || !grad_ylt) return fail(ARA_E_INVAL, "ara_metrics_vjp: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
    k_met_vjp<<<dim3(gx, static_cast<unsigned>(n_layers)), 256, 0, st>>>(weights, n, n_layers, grad_out, grad_ylt);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}
