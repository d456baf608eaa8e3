// Tail metrics of the YLT: mean annual loss, PML_p (the r-th largest year
// loss) and TVaR_p (mean of the r largest), r = N - floor(p*N + 1e-9).
//
// Selection is a radix select on the binary64 bit patterns (year losses are
// >= 0, so the unsigned order of the bits is the numeric order): 11-bit
// digits from the top, one grid pass for the first digit, one grid pass that
// also collects the candidates sharing it, then a single workgroup per layer
// finishes on the candidates.  Sums use a fixed partition of the trials and
// fixed-order trees, so every result is deterministic.
#include "ara_internal.h"

#include <algorithm>
#include <cmath>

namespace ara {

constexpr int kDigit = 11;
constexpr int kBins = 1 << kDigit;
constexpr int kMetThreads = 1024;

struct MetState {
    uint64_t prefix;       // selected high bits so far
    int64_t need;          // rank (1-based from the top) still to find below the prefix
    int64_t cand_n;        // candidates collected
    uint64_t thr_bits;
    int64_t cnt_gt, cnt_eq;
    double thr;
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

// Fixed-order block sum of one double per thread.
__device__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (tid == 0)
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;   // valid in thread 0
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

// Scan bins from the top until `need` is reached: returns the digit, and the
// rank still needed inside that bin.  Runs in thread 0.
__device__ void pick_digit(const uint32_t *h, int bins, int64_t need, int &digit, int64_t &need_in) {
    int64_t acc = 0;
    digit = 0;
    need_in = need;
    for (int d = bins - 1; d >= 0; --d) {
        const int64_t c = h[d];
        if (acc + c >= need) {
            digit = d;
            need_in = need - acc;
            return;
        }
        acc += c;
    }
}

__global__ __launch_bounds__(kMetThreads) void k_met_hist1(const double *__restrict__ ylt, int64_t n, int nwg,
                                                          uint32_t *__restrict__ hist1, MetPart *__restrict__ part) {
    __shared__ uint32_t h[kBins];
    __shared__ double red[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = ylt + static_cast<size_t>(l) * n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double v = y[i];
        s += v;
        atomicAdd(&h[key_of(v) >> (64 - kDigit)], 1u);
    }
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) part[static_cast<size_t>(l) * nwg + wg].sum = tot;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist1[static_cast<size_t>(l) * kBins + i], h[i]);
}

__global__ __launch_bounds__(kMetThreads) void k_met_cand(const double *__restrict__ ylt, int64_t n, int nwg,
                                                         const uint32_t *__restrict__ hist1, uint32_t *__restrict__ hist2,
                                                         uint64_t *__restrict__ cand, MetState *__restrict__ st,
                                                         int64_t r) {
    __shared__ uint32_t h[kBins];
    __shared__ int sd;
    __shared__ int64_t sneed;
    __shared__ int64_t wcnt[16], wbase[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hist1[static_cast<size_t>(l) * kBins + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        int d;
        int64_t need_in;
        pick_digit(h, kBins, r, d, need_in);
        sd = d;
        sneed = need_in;
        if (wg == 0) {
            st[l].prefix = static_cast<uint64_t>(d);
            st[l].need = need_in;
            st[l].r = r;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t d1 = static_cast<uint64_t>(sd);
    int64_t lo, hi;
    chunk_of(n, nwg, wg, lo, hi);
    const double *y = ylt + static_cast<size_t>(l) * n;
    uint64_t *c = cand + static_cast<size_t>(l) * n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // pass 1: candidates per wavefront; one global reservation per workgroup
    int64_t mine = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) mine += ((key_of(y[i]) >> (64 - kDigit)) == d1);
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o);
    if (lane == 0) wcnt[w] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) tot += wcnt[i];
        int64_t base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(&st[l].cand_n),
                                                           static_cast<unsigned long long>(tot)))
                           : 0;
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) {
            wbase[i] = base;
            base += wcnt[i];
        }
    }
    __syncthreads();
    // pass 2: write them, each wavefront from its own base, in index order
    int64_t off = wbase[w];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint64_t u = key_of(y[i]);
        const bool is = (u >> (64 - kDigit)) == d1;
        const uint64_t m = __ballot(is);
        if (is) {
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
            c[off + pos] = u;
            atomicAdd(&h[(u >> (64 - 2 * kDigit)) & (kBins - 1)], 1u);
        }
        off += __popcll(m);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i]) atomicAdd(&hist2[static_cast<size_t>(l) * kBins + i], h[i]);
}

// One workgroup per layer: second digit from hist2, remaining digits over the
// candidate list.
__global__ __launch_bounds__(kMetThreads) void k_met_select(int64_t n, const uint32_t *__restrict__ hist2,
                                                           const uint64_t *__restrict__ cand, MetState *__restrict__ st) {
    __shared__ uint32_t h[kBins];
    __shared__ uint64_t sprefix;
    __shared__ int64_t sneed;
    const int l = blockIdx.x;
    const uint64_t *c = cand + static_cast<size_t>(l) * n;
    const int64_t cn = st[l].cand_n;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = hist2[static_cast<size_t>(l) * kBins + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        int d;
        int64_t need_in;
        pick_digit(h, kBins, st[l].need, d, need_in);
        sprefix = (st[l].prefix << kDigit) | static_cast<uint64_t>(d);
        sneed = need_in;
    }
    __syncthreads();
    int known = 2 * kDigit;   // high bits fixed so far
    while (known < 64) {
        const int width = std::min(kDigit, 64 - known);
        const int shift = 64 - known - width;
        const uint64_t prefix = sprefix;
        for (int i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < cn; i += blockDim.x) {
            const uint64_t u = c[i];
            if ((u >> (64 - known)) == prefix) atomicAdd(&h[(u >> shift) & ((1u << width) - 1u)], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int d;
            int64_t need_in;
            pick_digit(h, 1 << width, sneed, d, need_in);
            sprefix = (prefix << width) | static_cast<uint64_t>(d);
            sneed = need_in;
        }
        __syncthreads();
        known += width;
    }
    if (threadIdx.x == 0) {
        st[l].thr_bits = sprefix;
        st[l].thr = __longlong_as_double(static_cast<long long>(sprefix));
    }
}

__global__ __launch_bounds__(kMetThreads) void k_met_tail(const double *__restrict__ ylt, int64_t n, int nwg,
                                                         const MetState *__restrict__ st, MetPart *__restrict__ part) {
    __shared__ double red[16];
    __shared__ int64_t redi[16];
    const int l = blockIdx.y, wg = blockIdx.x;
    const double thr = st[l].thr;
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
    c.take<uint32_t>(static_cast<size_t>(L) * kBins);
    c.take<uint32_t>(static_cast<size_t>(L) * kBins);
    c.take<MetState>(static_cast<size_t>(L));
    c.take<MetPart>(static_cast<size_t>(L) * nwg);
    c.take<uint64_t>(static_cast<size_t>(L) * n);
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
    uint32_t *hist1 = c.take<uint32_t>(static_cast<size_t>(n_layers) * kBins);
    uint32_t *hist2 = c.take<uint32_t>(static_cast<size_t>(n_layers) * kBins);
    MetState *state = c.take<MetState>(static_cast<size_t>(n_layers));
    MetPart *part = c.take<MetPart>(static_cast<size_t>(n_layers) * nwg);
    uint64_t *cand = c.take<uint64_t>(static_cast<size_t>(n_layers) * n);
    // header, both histograms and the states are contiguous: clear them at once
    const size_t clear = reinterpret_cast<char *>(part) - reinterpret_cast<char *>(hdr);
    ARA_HIP(hipMemsetAsync(hdr, 0, clear, st));
    if (n_layers == 0) return ARA_OK;
    int64_t r = n - static_cast<int64_t>(std::floor(p * static_cast<double>(n) + 1e-9));
    r = std::max<int64_t>(1, std::min<int64_t>(n, r));
    dim3 grid(static_cast<unsigned>(nwg), static_cast<unsigned>(n_layers));
    ProfScope prof(ARA_PROF_METRICS, st);
    k_met_hist1<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, hist1, part);
    k_met_cand<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, hist1, hist2, cand, state, r);
    k_met_select<<<n_layers, kMetThreads, 0, st>>>(n, hist2, cand, state);
    k_met_tail<<<grid, kMetThreads, 0, st>>>(ylt, n, nwg, state, part);
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
