// Tail metrics of the YLT: mean annual loss, PML_p (the r-th largest year
// loss) and TVaR_p (mean of the r largest), r = N - floor(p*N + 1e-9).
//
// Selection is a radix select on the binary64 bit patterns (year losses are
// >= 0, so the unsigned order of the bits is the numeric order), with digits
// of 11 bits from the top.  Two grid passes fix the exponent and the leading
// mantissa digit; if few values share that 23-bit prefix they are gathered
// and one workgroup finishes in LDS, otherwise (heavy ties) four more grid
// passes finish (they exit at once when the small path already finished).
// Sums use a fixed partition of the trials and fixed-order trees, so every
// result is deterministic.
#include "ara_internal.h"

#include <algorithm>
#include <cmath>

namespace ara {

constexpr int kMetThreads = 1024;
constexpr int kBins = 2048;
constexpr int kPassesMet = 6;
constexpr int kCandCap = 16384;     // candidates finished inside one workgroup's LDS
// digit d covers bits [kShift[d], kShift[d] + kWidth[d]) of the key; bit 63
// (the sign) is 0 for every year loss
__constant__ int kShift[kPassesMet] = {52, 41, 30, 19, 8, 0};
__constant__ int kWidth[kPassesMet] = {11, 11, 11, 11, 11, 8};

struct MetState {
    uint64_t prefix[kPassesMet + 1];   // bits fixed before digit d (prefix[d] has 64 - kShift[d] - kWidth[d] bits)
    int64_t need[kPassesMet + 1];      // rank (1-based from the top) to find among values with prefix[d]
    int64_t cand_n;
    int32_t small, done;
    double thr;
    int64_t cnt_gt, cnt_eq;
    int64_t r;
};

struct MetPart {
    double sum, sum_gt;
    int64_t cnt_gt, cnt_eq;
};

__device__ __forceinline__ uint64_t key_of(double y) {
    return (y == 0.0) ? 0ull : static_cast<uint64_t>(__double_as_longlong(y));
}

__device__ __forceinline__ void chunk_of(int64_t n, int nwg, int wg, int64_t &lo, int64_t &hi) {
    const int64_t c = (n + nwg - 1) / nwg;
    lo = std::min<int64_t>(n, static_cast<int64_t>(wg) * c);
    hi = std::min<int64_t>(n, lo + c);
}

// Fixed-order block reductions (value valid in thread 0).
__device__ double block_sum(double v, double *red) {
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

__device__ int64_t block_count(int64_t v, int64_t *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[w] = v;
    __syncthreads();
    int64_t t = 0;
    if (tid == 0)
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;
}

struct FindShared {
    int64_t wtot[16];
    int digit;
    int64_t need;
};

// Locate the bin holding the need-th largest value (counting from the top) in
// histogram h[0..bins); every thread of the block takes part (1024 threads,
// two bins each).  Result in fs.digit / fs.need (the rank inside that bin).
__device__ void find_digit(const uint32_t *h, int bins, int64_t need, FindShared &fs) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) {   // defaults (never used when the histogram holds `need` values)
        fs.digit = 0;
        fs.need = 1;
    }
    const int64_t c_lo = (2 * t < bins) ? h[2 * t] : 0;
    const int64_t c_hi = (2 * t + 1 < bins) ? h[2 * t + 1] : 0;
    const int64_t v = c_lo + c_hi;
    // inclusive suffix sum over threads t' >= t
    int64_t suf = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t x = __shfl_down(suf, o);
        if (lane + o < 64) suf += x;
    }
    if (lane == 0) fs.wtot[w] = suf;
    __syncthreads();
    int64_t higher = 0;
    for (int i = w + 1; i < static_cast<int>(blockDim.x >> 6); ++i) higher += fs.wtot[i];
    const int64_t above = suf - v + higher;   // values in bins above 2t+1
    if (above < need && need <= above + c_hi) {
        fs.digit = 2 * t + 1;
        fs.need = need - above;
    } else if (above + c_hi < need && need <= above + v) {
        fs.digit = 2 * t;
        fs.need = need - above - c_hi;
    }
    __syncthreads();
}

// Digit pass d over the whole YLT row: histogram of digit d among the values
// whose higher bits equal the prefix selected so far.  Pass 0 also forms the
// fixed-partition partial sums for the mean.
__global__ __launch_bounds__(kMetThreads) void k_met_pass(const double *__restrict__ ylt, int64_t n, int nwg, int d,
                                                         uint32_t *__restrict__ hist, MetState *__restrict__ st,
                                                         MetPart *__restrict__ part, int64_t r) {
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    __shared__ double red[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    MetState &S = st[l];
    uint64_t prefix = 0;
    int64_t need = r;
    if (d > 0) {
        if (S.done) return;
        const uint32_t *hp = hist + (static_cast<size_t>(d - 1) * gridDim.y + l) * kBins;
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hp[i];
        __syncthreads();
        find_digit(h, 1 << kWidth[d - 1], S.need[d - 1], fs);
        prefix = (S.prefix[d - 1] << kWidth[d - 1]) | static_cast<uint64_t>(fs.digit);
        need = fs.need;
    }
    if (wg == 0 && threadIdx.x == 0) {
        S.prefix[d] = prefix;
        S.need[d] = need;
        if (d == 0) S.r = r;
    }
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int sh = kShift[d], hb = kShift[d] + kWidth[d];
    const uint32_t mask = (1u << kWidth[d]) - 1u;
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = ylt + static_cast<size_t>(l) * n;
    double s = 0.0;
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = lo; i0 < hi; i0 += blockDim.x) {   // uniform trip count: every lane reaches the ballots
        const int64_t i = i0 + threadIdx.x;
        const double v = (i < hi) ? y[i] : 0.0;
        const uint64_t u = key_of(v);
        if (d == 0) s += v;
        const bool want = i < hi && (hb >= 64 || (u >> hb) == prefix);
        const uint32_t dg = static_cast<uint32_t>((u >> sh) & mask);
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
    if (d == 0) {
        const double tot = block_sum(s, red);
        if (threadIdx.x == 0) part[static_cast<size_t>(l) * nwg + wg].sum = tot;
    }
    __syncthreads();
    uint32_t *hd = hist + (static_cast<size_t>(d) * gridDim.y + l) * kBins;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hd[i], h[i]);
}

// After pass 1: if at most kCandCap values share the 23-bit prefix, gather
// them (one reservation per workgroup) so a single workgroup can finish.
__global__ __launch_bounds__(kMetThreads) void k_met_collect(const double *__restrict__ ylt, int64_t n, int nwg,
                                                            const uint32_t *__restrict__ hist, MetState *__restrict__ st,
                                                            uint64_t *__restrict__ cand) {
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    __shared__ int64_t wcnt[16], wbase[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    MetState &S = st[l];
    const uint32_t *hp = hist + (static_cast<size_t>(1) * gridDim.y + l) * kBins;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hp[i];
    __syncthreads();
    find_digit(h, 1 << kWidth[1], S.need[1], fs);
    const uint64_t prefix = (S.prefix[1] << kWidth[1]) | static_cast<uint64_t>(fs.digit);
    const int64_t in_bin = h[fs.digit];
    const bool small = in_bin <= kCandCap;
    if (wg == 0 && threadIdx.x == 0) S.small = small ? 1 : 0;
    if (!small) return;
    const int hb = kShift[1];
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = ylt + static_cast<size_t>(l) * n;
    uint64_t *c = cand + static_cast<size_t>(l) * kCandCap;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t mine = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) mine += ((key_of(y[i]) >> hb) == prefix);
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o);
    if (lane == 0) wcnt[w] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) tot += wcnt[i];
        int64_t base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(&S.cand_n),
                                                           static_cast<unsigned long long>(tot)))
                           : 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) {
            wbase[i] = base;
            base += wcnt[i];
        }
    }
    __syncthreads();
    int64_t off = wbase[w];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint64_t u = key_of(y[i]);
        const bool is = (u >> hb) == prefix;
        const uint64_t m = __ballot(is);
        if (is) {
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
            c[off + pos] = u;
        }
        off += __popcll(m);
    }
}

// One workgroup per layer finishes digits 2..5 on the collected candidates.
__global__ __launch_bounds__(kMetThreads) void k_met_small(const uint32_t *__restrict__ hist, MetState *__restrict__ st,
                                                          const uint64_t *__restrict__ cand) {
    __shared__ uint64_t cs[kCandCap];
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    const int l = blockIdx.x;
    MetState &S = st[l];
    if (!S.small) return;
    const int64_t cn = S.cand_n;
    for (int64_t i = threadIdx.x; i < cn; i += blockDim.x) cs[i] = cand[static_cast<size_t>(l) * kCandCap + i];
    const uint32_t *hp = hist + (static_cast<size_t>(1) * gridDim.x + l) * kBins;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hp[i];
    __syncthreads();
    find_digit(h, 1 << kWidth[1], S.need[1], fs);
    uint64_t prefix = (S.prefix[1] << kWidth[1]) | static_cast<uint64_t>(fs.digit);
    int64_t need = fs.need;
    for (int d = 2; d < kPassesMet; ++d) {
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
        __syncthreads();
        const int sh = kShift[d], hb = kShift[d] + kWidth[d];
        const uint32_t mask = (1u << kWidth[d]) - 1u;
        for (int64_t i = threadIdx.x; i < cn; i += blockDim.x) {
            const uint64_t u = cs[i];
            if ((u >> hb) == prefix) atomicAdd(&h[(u >> sh) & mask], 1u);
        }
        __syncthreads();
        find_digit(h, 1 << kWidth[d], need, fs);
        prefix = (prefix << kWidth[d]) | static_cast<uint64_t>(fs.digit);
        need = fs.need;
    }
    if (threadIdx.x == 0) {
        S.thr = __longlong_as_double(static_cast<long long>(prefix));
        S.done = 1;
    }
}

// Counts and sum above the PML value (fixed partition, fixed-order trees).
__global__ __launch_bounds__(kMetThreads) void k_met_tail(const double *__restrict__ ylt, int64_t n, int nwg,
                                                         const uint32_t *__restrict__ hist, MetState *__restrict__ st,
                                                         MetPart *__restrict__ part) {
    __shared__ uint32_t h[kBins];
    __shared__ FindShared fs;
    __shared__ double red[16];
    __shared__ int64_t redi[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    MetState &S = st[l];
    double thr;
    if (S.done) {
        thr = S.thr;
    } else {
        const int d = kPassesMet - 1;
        const uint32_t *hp = hist + (static_cast<size_t>(d) * gridDim.y + l) * kBins;
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hp[i];
        __syncthreads();
        find_digit(h, 1 << kWidth[d], S.need[d], fs);
        const uint64_t bits = (S.prefix[d] << kWidth[d]) | static_cast<uint64_t>(fs.digit);
        thr = __longlong_as_double(static_cast<long long>(bits));
        if (wg == 0 && threadIdx.x == 0) S.thr = thr;
    }
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = ylt + static_cast<size_t>(l) * n;
    double s = 0.0;
    int64_t gt = 0, eq = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double v = y[i];
        if (v > thr) {
            s += v;
            ++gt;
        } else if (v == thr) {
            ++eq;
        }
    }
    const double ts = block_sum(s, red);
    const int64_t tg = block_count(gt, redi);
    const int64_t te = block_count(eq, redi);
    if (threadIdx.x == 0) {
        MetPart &p = part[static_cast<size_t>(l) * nwg + wg];
        p.sum_gt = ts;
        p.cnt_gt = tg;
        p.cnt_eq = te;
    }
}

__global__ __launch_bounds__(kMetThreads) void k_met_final(int64_t n, int nwg, const MetPart *__restrict__ part,
                                                          MetState *__restrict__ st, double *__restrict__ out) {
    __shared__ double red[16];
    __shared__ int64_t redi[16];
    const int l = blockIdx.x;
    double s = 0.0, sg = 0.0;
    int64_t gt = 0, eq = 0;
    for (int i = threadIdx.x; i < nwg; i += blockDim.x) {
        const MetPart &p = part[static_cast<size_t>(l) * nwg + i];
        s += p.sum;
        sg += p.sum_gt;
        gt += p.cnt_gt;
        eq += p.cnt_eq;
    }
    const double ts = block_sum(s, red);
    const double tsg = block_sum(sg, red);
    const int64_t tgt = block_count(gt, redi);
    const int64_t teq = block_count(eq, redi);
    if (threadIdx.x == 0) {
        const int64_t r = st[l].r;
        const double thr = st[l].thr;
        st[l].cnt_gt = tgt;
        st[l].cnt_eq = teq;
        out[3 * l + 0] = ts / static_cast<double>(n);
        out[3 * l + 1] = thr;
        out[3 * l + 2] = (tsg + static_cast<double>(r - tgt) * thr) / static_cast<double>(r);
    }
}

__global__ void k_met_weights(const double *__restrict__ ylt, int64_t n, int n_layers, const MetState *__restrict__ st,
                              double *__restrict__ w) {
    const int l = blockIdx.y;
    const double thr = st[l].thr;
    const int64_t r = st[l].r, gt = st[l].cnt_gt, eq = st[l].cnt_eq;
    const double inv_n = 1.0 / static_cast<double>(n);
    const double w_pml = 1.0 / static_cast<double>(eq);
    const double w_gt = 1.0 / static_cast<double>(r);
    const double w_eq = static_cast<double>(r - gt) / (static_cast<double>(r) * static_cast<double>(eq));
    const double *y = ylt + static_cast<size_t>(l) * n;
    double *wa = w + (static_cast<size_t>(0) * n_layers + l) * n;
    double *wp = w + (static_cast<size_t>(1) * n_layers + l) * n;
    double *wt = w + (static_cast<size_t>(2) * n_layers + l) * n;
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
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 8191) / 8192, 1024)));
}

static size_t met_bytes(int32_t L, int64_t n) {
    const int nwg = met_nwg(n);
    Carver c(nullptr);
    c.take<int32_t>(kWsHeaderBytes / 4);
    c.take<uint32_t>(static_cast<size_t>(kPassesMet) * L * kBins);
    c.take<MetState>(static_cast<size_t>(L));
    c.take<MetPart>(static_cast<size_t>(L) * nwg);
    c.take<uint64_t>(static_cast<size_t>(L) * kCandCap);
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
    if (!(p > 0.0 && p < 1.0)) return fail(ARA_E_INVAL, "ara_metrics: p must lie in (0, 1)");
    if (!ws || (n_layers > 0 && (!ylt || !out))) return fail(ARA_E_INVAL, "ara_metrics: null pointer");
    if (ws_bytes < met_bytes(n_layers, n)) return fail(ARA_E_NOSPACE, "ara_metrics: workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nwg = met_nwg(n);
    Carver c(ws);
    int32_t *hdr = c.take<int32_t>(kWsHeaderBytes / 4);
    uint32_t *hist = c.take<uint32_t>(static_cast<size_t>(kPassesMet) * n_layers * kBins);
    MetState *state = c.take<MetState>(static_cast<size_t>(n_layers));
    MetPart *part = c.take<MetPart>(static_cast<size_t>(n_layers) * nwg);
    uint64_t *cand = c.take<uint64_t>(static_cast<size_t>(n_layers) * kCandCap);
    // header, histograms and states are contiguous: clear them at once
    const size_t clear = reinterpret_cast<char *>(part) - reinterpret_cast<char *>(hdr);
    ARA_HIP(hipMemsetAsync(hdr, 0, clear, st));
    if (n_layers == 0) return ARA_OK;
    int64_t r = n - static_cast<int64_t>(std::floor(p * static_cast<double>(n) + 1e-9));
    r = std::max<int64_t>(1, std::min<int64_t>(n, r));
    dim3 grid(static_cast<unsigned>(nwg), static_cast<unsigned>(n_layers));
    ProfScope prof(ARA_PROF_METRICS, st);
    k_met_pass<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, 0, hist, state, part, r);
    k_met_pass<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, 1, hist, state, part, r);
    k_met_collect<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, hist, state, cand);
    k_met_small<<<n_layers, kMetThreads, 0, st>>>(hist, state, cand);
    for (int d = 2; d < kPassesMet; ++d) k_met_pass<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, d, hist, state, part, r);
    k_met_tail<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, hist, state, part);
    k_met_final<<<n_layers, kMetThreads, 0, st>>>(n, nwg, part, state, out);
    if (weights) {
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
        k_met_weights<<<dim3(gx, static_cast<unsigned>(n_layers)), 256, 0, st>>>(ylt, n, n_layers, state, weights);
    }
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}

extern "C" int32_t ara_metrics_vjp(const double *weights, int32_t n_layers, int64_t n, const double *grad_out,
                                   double *grad_ylt, void *stream) {
    if (n_layers < 0 || n < 0) return fail(ARA_E_INVAL, "ara_metrics_vjp: bad size");
    if (n_layers == 0 || n == 0) return ARA_OK;
    if (!weights || !grad_out || !grad_ylt) return fail(ARA_E_INVAL, "ara_metrics_vjp: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
    k_met_vjp<<<dim3(gx, static_cast<unsigned>(n_layers)), 256, 0, st>>>(weights, n, n_layers, grad_out, grad_ylt);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}
