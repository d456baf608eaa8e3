// Secondary uncertainty (named as future work in Section VI): Algorithm 1 with
// the table lookup of step one replaced by a draw per (occurrence, ELT) from
// the lognormal distribution with the record's mean and standard deviation.
//
// Per call and layer:
//   * the occurrence table in union mode gives the layer's union of ELT
//     events as a bitmap with ranks, and the number of the layer's ELTs
//     holding each union event;
//   * a scan of those counts and a fill pass lay out, per union event and in
//     the layer's listed ELT order, one entry per ELT holding it: the
//     lognormal's parameters (m, s), the mean, the ELT's position and index;
//   * the streaming kernel walks the trial-major YET (the occurrence index
//     keys the draws, so storage order matters): one wavefront per trial, a
//     1-Mbit LDS filter of the union, a queue of union occurrences drawn 64
//     at a time: the draws of each one's entries, the ELT terms (step two)
//     summed in listed order, the occurrence terms (step three); the trial's
//     occurrence losses meet in a DPP wavefront sum and the aggregate terms
//     give the year loss (step four, telescoped).
// The draw: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) block of
// counter words (occurrence low, high, ELT index, 0) under key words (seed
// low, high); two uniforms from the top 52 bits of the word pairs (w1 w0)
// and (w3 w2), Box-Muller, x = exp(m + s z), with the logarithm, cosine and
// exponential of su_math.h.
#include "occ.h"
#include "su_math.h"
#include "wave.h"

#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <vector>

namespace ara {

constexpr int kSuThreads = 1024;
constexpr int kSuMaxJ = ARA_MAX_ELTS_PER_LAYER;
constexpr int kSuScanPer = kSr / kSuThreads;   // 64 ranks per thread in the count scan

// One (union event, ELT of the layer) pair; 32 bytes.  The first ELT (in
// listed order) holding a union event has its entry at the event's union
// rank; the others follow at `next`, contiguous.
struct SuEntry {
    double m, s;       // lognormal parameters of the draw
    float mu;          // the record's mean loss
    int32_t k;         // the ELT's index (keys the draw)
    uint32_t next;     // first of the event's further entries (first entry only)
    uint16_t q;        // the ELT's position in the layer's list
    uint8_t exact;     // sigma = 0: the draw is mu itself
    uint8_t more;      // number of further entries (first entry only)
};
static_assert(sizeof(SuEntry) == 32 && offsetof(SuEntry, mu) == 16 && offsetof(SuEntry, next) == 24 &&
                  offsetof(SuEntry, q) == 28 && offsetof(SuEntry, exact) == 30 && offsetof(SuEntry, more) == 31,
              "entry layout (read as two 16-byte words)");

// ---------------------------------------------------------------------------
// Standard-deviation tables.

// Records already checked on the host.
__global__ void k_sigma_scatter(const int64_t *__restrict__ rec_off, const int32_t *__restrict__ rec_ids,
                                const float *__restrict__ rec_sigma, int32_t catalog, float *__restrict__ sigma) {
    const int k = blockIdx.y;
    const int64_t a = rec_off[k], b = rec_off[k + 1];
    for (int64_t i = a + blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < b;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        sigma[static_cast<size_t>(k) * catalog + rec_ids[i]] = rec_sigma[i];
}

// ---------------------------------------------------------------------------
// Entry layout.

// Per (super-range, layer): exclusive scan, in rank order, of the number of
// further entries of each union event (its ELT count less one) -> ooff
// (relative to the super-range), total -> otot.
__global__ __launch_bounds__(kSuThreads) void k_su_scan(const OccTables *__restrict__ tabs, int n_sr,
                                                        uint32_t *__restrict__ ooff, uint32_t *__restrict__ otot) {
    __shared__ uint32_t wsum[kSuThreads / kWave];
    const int s = blockIdx.x, j = blockIdx.y, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const OccTables T = tabs[j];
    const int cnt_s = T.count[s];
    const uint8_t *c = T.cnt + static_cast<size_t>(s) * kSr;
    uint32_t *oo = ooff + (static_cast<size_t>(j) * n_sr + s) * kSr;
    const int r0 = tid * kSuScanPer;
    uint32_t mine = 0;
    for (int r = r0; r < min(r0 + kSuScanPer, cnt_s); ++r) mine += c[r] - 1u;
    uint32_t incl = mine;
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = incl - mine;
    for (int i = 0; i < w; ++i) before += wsum[i];
    for (int r = r0; r < min(r0 + kSuScanPer, cnt_s); ++r) {
        oo[r] = before;
        before += c[r] - 1u;
    }
    if (tid == kSuThreads - 1) otot[static_cast<size_t>(j) * n_sr + s] = before;
}

// Exclusive scan of n values of one workgroup (n up to a few thousand).
template <class T>
__device__ T block_exclusive_scan(const T *in, T *out, int n, T *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int per = (n + kSuThreads - 1) / kSuThreads;
    const int s0 = tid * per;
    T mine = 0;
    for (int s = s0; s < min(s0 + per, n); ++s) mine += in[s];
    T incl = mine;
    for (int o = 1; o < kWave; o <<= 1) {
        const T v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    T before = incl - mine;
    for (int i = 0; i < w; ++i) before += wsum[i];
    for (int s = s0; s < min(s0 + per, n); ++s) {
        out[s] = before;
        before += in[s];
    }
    __syncthreads();
    T total = 0;
    for (int i = 0; i < kSuThreads / kWave; ++i) total += wsum[i];
    __syncthreads();
    return total;
}

// Per layer: union-rank bases of the super-ranges (ubase, from the
// occurrence table's counts) and bases of their further entries (obase,
// after all first entries); every entry must fit the layer's capacity.
__global__ __launch_bounds__(kSuThreads) void k_su_base(const OccTables *__restrict__ tabs, const uint32_t *__restrict__ otot,
                                                        int n_sr, const uint64_t *__restrict__ ecap,
                                                        uint32_t *__restrict__ ubase, uint32_t *__restrict__ obase,
                                                        uint64_t *__restrict__ eused, int32_t *__restrict__ err) {
    __shared__ uint32_t wsum[kSuThreads / kWave];
    const int j = blockIdx.x;
    const OccTables T = tabs[j];
    uint32_t *ub = ubase + static_cast<size_t>(j) * (n_sr + 1);
    uint32_t *ob = obase + static_cast<size_t>(j) * n_sr;
    const uint32_t n_union = block_exclusive_scan<uint32_t>(reinterpret_cast<const uint32_t *>(T.count), ub, n_sr, wsum);
    const uint32_t n_more = block_exclusive_scan<uint32_t>(otot + static_cast<size_t>(j) * n_sr, ob, n_sr, wsum);
    for (int s = threadIdx.x; s < n_sr; s += blockDim.x) ob[s] += n_union;
    if (threadIdx.x == 0) {
        ub[n_sr] = n_union;
        eused[j] = static_cast<uint64_t>(n_union) + n_more;
        if (eused[j] > ecap[j]) atomicCAS(err, 0, ARA_E_LIMIT);
    }
}

// Per (1024-event chunk, layer): the entries of every union event, in the
// layer's listed ELT order; one event per thread, so that the chains of
// dependent loads (bitmap word, rank, counts; presence; losses) of many
// events are in flight at once.
constexpr int kSuFillWords = kSuThreads / 32;      // 1024 events per workgroup
constexpr int kSuFillChunks = kSrWords / kSuFillWords;
constexpr int kSuFillBatch = 8;                    // ELTs whose loads are in flight together

__global__ __launch_bounds__(kSuThreads) void k_su_fill(const float *__restrict__ loss, const float *__restrict__ sigma,
                                                        const uint32_t *__restrict__ present, int32_t catalog,
                                                        int32_t words, const int32_t *__restrict__ elt_off,
                                                        const int32_t *__restrict__ elt_ids,
                                                        const OccTables *__restrict__ tabs, int n_sr,
                                                        const uint32_t *__restrict__ ooff,
                                                        const uint32_t *__restrict__ ubase,
                                                        const uint32_t *__restrict__ obase,
                                                        const uint64_t *__restrict__ ecap,
                                                        const uint64_t *__restrict__ eregion,
                                                        SuEntry *__restrict__ ent) {
    __shared__ int32_t lk[kSuMaxJ];
    const int s = blockIdx.x / kSuFillChunks, p = blockIdx.x % kSuFillChunks, j = blockIdx.y;
    const int tid = threadIdx.x;
    const int a = elt_off[j], J = elt_off[j + 1] - a;
    for (int q = tid; q < J; q += blockDim.x) lk[q] = elt_ids[a + q];
    __syncthreads();
    const OccTables T = tabs[j];
    const uint64_t cap = ecap[j];
    const uint32_t ub = ubase[static_cast<size_t>(j) * (n_sr + 1) + s];
    const uint32_t n_union = ubase[static_cast<size_t>(j) * (n_sr + 1) + n_sr];
    const uint32_t ob = obase[static_cast<size_t>(j) * n_sr + s];
    if (n_union > cap) return;   // flagged by k_su_base
    SuEntry *E = ent + eregion[j];
    const uint32_t *oo = ooff + (static_cast<size_t>(j) * n_sr + s) * kSr;
    {
        const int local = p * (kSuFillWords * 32) + tid;   // event within the super-range
        const int64_t ev = static_cast<int64_t>(s) * kSr + local;
        if (ev >= catalog) return;
        const uint2 q2 = T.br[static_cast<size_t>(s) * kSrWords + (local >> 5)];
        const int bit = local & 31;
        if (!((q2.x >> bit) & 1u)) return;
        const uint32_t r = q2.y + __popc(q2.x & ((1u << bit) - 1u));
        const uint32_t nb = T.cnt[static_cast<size_t>(s) * kSr + r];
        const uint64_t first = static_cast<uint64_t>(ub) + r;
        const uint64_t next = static_cast<uint64_t>(ob) + oo[r];
        uint64_t o = first;
        int h = 0;
        // eight ELTs at a time: their presence words loaded together, then
        // the losses and deviations of the present ones, then the entries in
        // listed order
        for (int q0 = 0; q0 < J; q0 += kSuFillBatch) {
            bool on[kSuFillBatch];
            float mu8[kSuFillBatch], sg8[kSuFillBatch];
#pragma unroll
            for (int i = 0; i < kSuFillBatch; ++i) {
                const int k = lk[min(q0 + i, J - 1)];
                on[i] = q0 + i < J && ((present[static_cast<size_t>(k) * words + (ev >> 5)] >> (ev & 31)) & 1u);
            }
#pragma unroll
            for (int i = 0; i < kSuFillBatch; ++i) {
                mu8[i] = sg8[i] = 0.0f;
                if (on[i]) {
                    const int k = lk[q0 + i];
                    mu8[i] = loss[static_cast<size_t>(k) * catalog + ev];
                    sg8[i] = sigma[static_cast<size_t>(k) * catalog + ev];
                }
            }
#pragma unroll
            for (int i = 0; i < kSuFillBatch; ++i) {
                // entries past the capacity are not written (flagged by k_su_base)
                if (!on[i] || o >= cap) continue;
                const float mu = mu8[i], sg = sg8[i];
                SuEntry e;
                e.mu = mu;
                e.k = lk[q0 + i];
                e.q = static_cast<uint16_t>(q0 + i);
                e.exact = (sg == 0.0f) ? 1 : 0;
                e.next = h == 0 ? static_cast<uint32_t>(next) : 0u;
                e.more = h == 0 ? static_cast<uint8_t>(nb - 1) : 0;
                e.m = 0.0;
                e.s = static_cast<double>(sg);   // k_su_params turns (mu, sigma) into (m, s)
                E[o] = e;
                o = (h == 0) ? next : o + 1;
                ++h;
            }
        }
    }
}

// Per layer: each entry's lognormal parameters from its mean and deviation,
// s^2 = ln(1 + sigma^2/mu^2), m = ln mu - s^2/2 (0, 0 for an exact entry), one
// thread per entry so that the binary64 logarithms run on full wavefronts.
__global__ __launch_bounds__(256) void k_su_params(const uint64_t *__restrict__ eregion,
                                                   const uint64_t *__restrict__ ecap,
                                                   const uint64_t *__restrict__ eused, SuEntry *__restrict__ ent) {
    const int j = blockIdx.y;
    const uint64_t cap = ecap[j], used = eused[j];
    if (used > cap) return;   // nothing laid out (flagged by k_su_base)
    SuEntry *E = ent + eregion[j];
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < used;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        SuEntry &e = E[i];
        if (e.exact) continue;
        const double mu = static_cast<double>(e.mu);
        const double rr = e.s / mu;
        const double s2 = log1p(rr * rr);
        e.m = log(mu) - 0.5 * s2;
        e.s = sqrt(s2);
    }
}

// ---------------------------------------------------------------------------
// The draw.

// One round of Philox4x32 (Salmon et al., SC'11): the two 32 x 32-bit
// products A x.x and B x.z, each formed by one 64-bit multiply, their high
// halves mixed with the other two words and the round key.
__device__ __forceinline__ uint4 philox_round(uint4 x, uint32_t k0, uint32_t k1) {
    const uint64_t a = static_cast<uint64_t>(x.x) * 0xD2511F53u;
    const uint64_t b = static_cast<uint64_t>(x.z) * 0xCD9E8D57u;
    return make_uint4(static_cast<uint32_t>(b >> 32) ^ x.y ^ k0, static_cast<uint32_t>(b),
                      static_cast<uint32_t>(a >> 32) ^ x.w ^ k1, static_cast<uint32_t>(a));
}

// Ten rounds; round r's key is the key plus r times the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (uint32_t r = 0; r < 10; ++r) ctr = philox_round(ctr, k0 + r * 0x9E3779B9u, k1 + r * 0xBB67AE85u);
    return ctr;
}

// One entry as two 16-byte loads issued together.
__device__ __forceinline__ SuEntry su_entry(const SuEntry *p) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    const uint4 a = q[0], b = q[1];
    SuEntry e;
    e.m = __hiloint2double(static_cast<int>(a.y), static_cast<int>(a.x));
    e.s = __hiloint2double(static_cast<int>(a.w), static_cast<int>(a.z));
    e.mu = __uint_as_float(b.x);
    e.k = static_cast<int32_t>(b.y);
    e.next = b.z;
    e.q = static_cast<uint16_t>(b.w & 0xFFFFu);
    e.exact = static_cast<uint8_t>((b.w >> 16) & 0xFFu);
    e.more = static_cast<uint8_t>(b.w >> 24);
    return e;
}

// Without a branch on sigma = 0 (such a pair draws mu itself): the lanes of
// a round draw together either way, and a branch would let the compiler
// split the entry's loads around it.
__device__ __forceinline__ double su_draw(const SuEntry &e, uint64_t seed, int64_t occ) {
    const uint64_t o = static_cast<uint64_t>(occ);
    const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(o), static_cast<uint32_t>(o >> 32),
                                             static_cast<uint32_t>(e.k), 0u),
                                  static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const uint64_t b1 = (static_cast<uint64_t>(w.y) << 32) | w.x, b2 = (static_cast<uint64_t>(w.w) << 32) | w.z;
    const double u1 = (static_cast<double>(b1 >> 12) + 0.5) * 0x1p-52;
    const double u2 = (static_cast<double>(b2 >> 12) + 0.5) * 0x1p-52;
    const double z = sqrt(-2.0 * su_log(u1)) * su_cos_2pi(u2);
    const double x = su_exp(e.m + e.s * z);
    return e.exact ? static_cast<double>(e.mu) : x;
}

// ---------------------------------------------------------------------------
// Streaming kernel: the prepared YET walked by catalogue range.
//
// One workgroup per (block of trials, layer); wavefront g owns trial group g
// of the block, as in the forward.  The catalogue is walked one range (2^15
// events) at a time with the range's bitmap words (union ranks) in LDS.  All
// workgroups walk the ranges in the same order, so the entries of the few
// ranges in use at any time stay in L2, and the codes and positions stream
// past it.  Each lane decodes its run of codes (trial advances, event
// offsets); an occurrence whose event is in the union is appended, with its
// trial in the block and its position in the trial, to the wavefront's LDS
// queue, and whenever 64 are queued they are drawn in rounds of one draw per
// lane: a lane takes the next queued occurrence, draws its first ELT and,
// when further ELTs hold the event, keeps the occurrence and draws one of
// them per round while the other lanes take new ones.  A finished
// occurrence's loss after the occurrence terms (steps two and three) is added
// to its trial's total in LDS.  The queue carries over from range to range;
// what is left is drawn after the last range, and the totals then meet the
// aggregate terms (step four, telescoped).
//
// A trial's total is accumulated by one wavefront in an order fixed by the
// block's code layout (same-address LDS additions of one instruction apply in
// lane order), so the results depend neither on the trial window nor on the
// other layers of the call.

constexpr int kSuChunk = 4;                                 // codes per lane and step (runs are multiples of 4)
constexpr int kSuQCap = 512;                                // a ring: fewer than 64 waiting + one step's codes
static_assert(kSuQCap >= (kWave - 1) + kSuChunk * kWave && (kSuQCap & (kSuQCap - 1)) == 0, "queue ring");
static_assert(kSuThreads == kSrWords / 2, "one bitmap word of a range per thread");

struct SuParams {
    const uint16_t *code, *pos;
    const int64_t *seg_base;
    const int32_t *seg_run;
    const uint8_t *lane_start;
    const int64_t *t_off;        // the YET's offsets
    int64_t n_trials;
    int32_t tg, tb, n_ranges, n_sr;
    int32_t b0, nb, n_layers, pad;
    int64_t t0, t1;
    const OccTables *tabs;
    const uint32_t *ubase;       // [n_layers][n_sr + 1] union-rank bases of the super-ranges
    const uint64_t *eregion;     // [n_layers]
    const uint64_t *ecap;        // [n_layers] entries allocated
    const uint64_t *eused;       // [n_layers] entries the layer needs
    const SuEntry *ent;
    const int32_t *elt_off, *elt_ids;
    const double *elt_terms, *layer_terms;
    uint64_t seed;
    double *ylt, *s_pre;
};

// Workgroup i's block (relative to b0) and layer: with one layer, block i;
// with several, the layers of one block run back to back on one XCD
// (workgroups are dealt to the XCDs round-robin; workgroup 8k + x is the
// k-th on XCD x and takes layer k % L of block 8 (k / L) + x), so that they
// read the block's codes from HBM once.  -1 past the last block.
__device__ __forceinline__ int su_item(const SuParams &P, int i, int &layer) {
    if (P.n_layers == 1) {
        layer = 0;
        return i < P.nb ? i : -1;
    }
    const int x = i % kXcds, k = i / kXcds;
    layer = k % P.n_layers;
    const int bi = (k / P.n_layers) * kXcds + x;
    return bi < P.nb ? bi : -1;
}

// SHARED: the workgroups of several layers read the same block's codes, so
// they are kept in L2; otherwise they stream past it.
template <bool SHARED>
__device__ __forceinline__ unsigned long long su_ld4(const uint16_t *p) {
    if (SHARED) return *reinterpret_cast<const unsigned long long *>(p);
    return __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
}

template <bool SHARED>
__global__ __launch_bounds__(kSuThreads) void k_su_fwd(SuParams P) {
    __shared__ uint2 tbr[kSrWords / 2];                  // the range's bitmap words with super-range ranks
    __shared__ double acc[kMaxTrialsPerBlock + 1];       // per-trial totals (one slot past the trials)
    __shared__ uint32_t offl[kMaxTrialsPerBlock];        // each trial's first occurrence less the block's
    __shared__ uint2 q_es[kGroups][kSuQCap];             // queued occurrence: (its event's union index,
                                                         //   its trial in the block << 16 | position in the trial)
    __shared__ double ls[kSuMaxJ], lr[kSuMaxJ], ll[kSuMaxJ];
    int j = 0;
    const int bi = su_item(P, blockIdx.x, j);
    if (bi < 0) return;   // uniform over the workgroup, before any barrier
    // a layer whose entries did not fit its capacity has none laid out (the
    // call reports ARA_E_LIMIT): nothing of it is read or written
    const uint64_t cap = P.ecap[j];
    if (P.eused[j] > cap) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tb = P.tb, G = P.n_ranges;
    const int64_t b = static_cast<int64_t>(P.b0) + bi;
    const int64_t bt0 = b * tb;                                            // the block's first trial
    const int nbt = static_cast<int>(min<int64_t>(tb, P.n_trials - bt0));  // and its trials
    const int64_t gt0 = bt0 + static_cast<int64_t>(w) * P.tg;
    const int64_t gt1 = min(gt0 + P.tg, P.n_trials);
    const bool active = gt0 < gt1 && gt1 > P.t0 && gt0 < P.t1;            // uniform
    const size_t seg0 = static_cast<size_t>(b) * G * kGroups + w;
    const int64_t occ0 = P.t_off[bt0];
    for (int i = tid; i <= tb; i += kSuThreads) acc[i] = 0.0;
    for (int i = tid; i < nbt; i += kSuThreads) offl[i] = static_cast<uint32_t>(P.t_off[bt0 + i] - occ0);
    const int a0 = P.elt_off[j], J = P.elt_off[j + 1] - a0;
    for (int q = tid; q < J; q += kSuThreads) {
        const int k = P.elt_ids[a0 + q];
        ls[q] = P.elt_terms[3 * k + 0];
        lr[q] = P.elt_terms[3 * k + 1];
        ll[q] = P.elt_terms[3 * k + 2];
    }
    const OccTables T = P.tabs[j];
    const uint32_t *ub = P.ubase + static_cast<size_t>(j) * (P.n_sr + 1);
    const SuEntry *E = P.ent + P.eregion[j];
    const double occR = P.layer_terms[4 * j + 0], occL = P.layer_terms[4 * j + 1];
    const double aggR = P.layer_terms[4 * j + 2], aggL = P.layer_terms[4 * j + 3];
    // thread tid's bitmap word of range r (range r is half r & 1 of super-range r >> 1)
    auto slice_word = [&](int r) { return T.br[static_cast<size_t>(r >> 1) * kSrWords + (r & 1) * (kSrWords / 2) + tid]; };
    tbr[tid] = slice_word(0);
    __syncthreads();

    uint2 *qes = q_es[w];
    int qh = 0, qlen = 0;   // uniform: the queue's head slot and length
    auto wrap = [](int x) { return x & (kSuQCap - 1); };
    // A lane whose occurrence is held by further ELTs keeps it and draws one
    // further ELT per round, so that no round waits on a few lanes.
    bool pend = false;
    uint32_t pe = 0;    // its next entry
    int pleft = 0;      // entries still to draw, pe included
    int64_t pi = 0;     // its index in the trial-major YET
    int ps = 0;         // its trial in the block
    double px = 0.0;    // its ELTs' losses so far, summed in listed order
    // one draw per lane: the held occurrences' next ELTs, and the queue's
    // first entries for the other lanes in lane order
    auto round = [&]() {
        const uint64_t freem = __ballot(!pend);
        const int rank = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
            static_cast<uint32_t>(freem >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(freem), 0u)));
        const int taken = min(qlen, static_cast<int>(__popcll(freem)));   // uniform
        const bool take = !pend && rank < taken;
        const bool act = take || pend;
        // Every lane runs the draw (no branch, so no state copies between
        // paths); an idle lane reads entry 0 and a queue slot it ignores, and
        // keeps its state.  Union indexes lie below the entries used, which
        // the layer's check above bounds by the entries allocated.
        const uint2 es = qes[wrap(qh + (take ? rank : 0))];
        const int slot = take ? static_cast<int>(es.y >> 16) : ps;
        const int64_t i = take ? occ0 + static_cast<int64_t>(offl[slot]) + static_cast<int64_t>(es.y & 0xFFFFu) : pi;
        const uint32_t ei = take ? es.x : (pend ? pe : 0u);
        const SuEntry en = su_entry(E + ei);
        const double v = su_draw(en, P.seed, i);
        const double g = xl(ls[en.q] * v, lr[en.q], ll[en.q]);
        const int left = take ? (static_cast<uint64_t>(en.next) + en.more <= cap ? en.more : 0) : pleft - 1;
        px = act ? (take ? g : px + g) : px;
        pi = i;
        ps = slot;
        pe = take ? en.next : pe + (act ? 1u : 0u);
        pleft = act ? left : pleft;
        const bool done = act && left <= 0;
        pend = act && left > 0;
        if (done) atomicAdd(&acc[ps], xl(px, occR, occL));
        qh = wrap(qh + taken);
        qlen -= taken;
    };

    // One step: four codes per lane (offset bits 5..14 pick the bitmap word,
    // bits 0..4 the bit; bit 15 advances the lane's trial first), and the
    // union occurrences among them appended to the queue code by code in
    // lane order.  Skip codes (0xFFFF) read the range's last bit: only when
    // that event is in the union must they be told apart from it.
    auto decode = [&](unsigned long long cx, unsigned long long cy, int &slot, uint32_t ubr, auto tell_tag) {
        constexpr bool kTell = decltype(tell_tag)::value;
        const uint32_t cw[2] = {static_cast<uint32_t>(cx), static_cast<uint32_t>(cx >> 32)};
        const uint32_t pw[2] = {static_cast<uint32_t>(cy), static_cast<uint32_t>(cy >> 32)};
        bool on[kSuChunk];
        uint2 ent[kSuChunk];
#pragma unroll
        for (int u = 0; u < kSuChunk; ++u) {
            const uint32_t c = (u & 1) ? (cw[u >> 1] >> 16) : cw[u >> 1];   // bits 16.. are ignored below
            slot += static_cast<int>(__builtin_amdgcn_ubfe(c, 15, 1));
            const uint2 q = tbr[__builtin_amdgcn_ubfe(c, 5, 10)];
            on[u] = __builtin_amdgcn_ubfe(q.x, c, 1) != 0u;   // bit (c & 31) of the word
            if (kTell) on[u] = on[u] && (c & 0xFFFFu) != 0xFFFFu;
            const uint32_t pos = (u & 1) ? (pw[u >> 1] >> 16) : (pw[u >> 1] & 0xFFFFu);
            ent[u] = make_uint2(ubr + q.y + __popc(__builtin_amdgcn_ubfe(q.x, 0, c)),
                                (static_cast<uint32_t>(slot) << 16) | pos);
        }
#pragma unroll
        for (int u = 0; u < kSuChunk; ++u) {
            const uint64_t m = __ballot(on[u]);
            if (on[u])
                qes[wrap(qh + qlen + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                          static_cast<uint32_t>(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u))))] = ent[u];
            qlen += static_cast<int>(__popcll(m));
        }
        __builtin_amdgcn_wave_barrier();
    };

    // ranges 0 .. G-1, then a last pass (r = G) that draws what is left; the
    // decode and the draw rounds each have one place in the code
    for (int r = 0; r <= G; ++r) {
        const bool flush = r == G;   // uniform
        uint2 nxt = make_uint2(0u, 0u);
        if (r + 1 < G) nxt = slice_word(r + 1);
        int R = 0;                   // uniform: this wavefront's codes per lane in range r
        int slot = 0;                // the lane's trial in the block
        const uint16_t *cp = nullptr, *pp = nullptr;
        unsigned long long X = 0, Y = 0, X2 = 0, Y2 = 0;
        uint32_t ubr = 0;            // union index of the super-range's rank 0
        const bool last_set = (__builtin_amdgcn_readfirstlane(tbr[1023].x) >> 31) != 0u;   // uniform
        if (active && !flush) {
            const size_t si = seg0 + static_cast<size_t>(r) * kGroups;
            R = __builtin_amdgcn_readfirstlane(P.seg_run[si]);
            if (R > 0) {
                ubr = __builtin_amdgcn_readfirstlane(ub[r >> 1]);
                const int64_t sb = P.seg_base[si];
                slot = w * P.tg + static_cast<int>(P.lane_start[si * kWave + lane]);
                cp = P.code + sb + 4 * lane;
                pp = P.pos + sb + 4 * lane;
                X = su_ld4<SHARED>(cp);
                Y = su_ld4<SHARED>(pp);
                if (kSuChunk < R) {
                    X2 = su_ld4<SHARED>(cp + kSuChunk * kWave);
                    Y2 = su_ld4<SHARED>(pp + kSuChunk * kWave);
                }
            }
        }
        for (int step = 0; step < R || flush; step += kSuChunk) {
            if (!flush) {
                const unsigned long long cx = X, cy = Y;
                if (step + kSuChunk < R) {   // uniform; the codes two steps ahead load while this one is decoded
                    X = X2;
                    Y = Y2;
                    if (step + 2 * kSuChunk < R) {
                        X2 = su_ld4<SHARED>(cp + 2 * kSuChunk * kWave);
                        Y2 = su_ld4<SHARED>(pp + 2 * kSuChunk * kWave);
                    }
                    cp += kSuChunk * kWave;
                    pp += kSuChunk * kWave;
                }
                if (last_set)
                    decode(cx, cy, slot, ubr, std::true_type{});
                else
                    decode(cx, cy, slot, ubr, std::false_type{});
            }
            while (qlen >= kWave || (flush && (qlen > 0 || __ballot(pend) != 0ull))) round();
            if (flush) break;
        }
        if (!flush) {
            __syncthreads();   // every wavefront is done with range r's words
            tbr[tid] = nxt;
            __syncthreads();
        }
    }
    if (active) {
        const int64_t lo = max(gt0, P.t0), hi = min(gt1, P.t1);
        const size_t n = static_cast<size_t>(P.t1 - P.t0);
        for (int64_t t = lo + lane; t < hi; t += kWave) {
            const double S = acc[t - bt0];
            const size_t o = static_cast<size_t>(j) * n + static_cast<size_t>(t - P.t0);
            P.ylt[o] = xl(S, aggR, aggL);
            if (P.s_pre) P.s_pre[o] = S;
        }
    }
}

// ---------------------------------------------------------------------------
// Workspace.

struct SuLayout {
    OccLayoutSizes z;
    std::vector<uint64_t> cap, region;   // per layer: entry capacity and first entry
    uint64_t n_ent = 0;
};

static int32_t su_layout(const ara_tables *tables, const ara_layers *layers, const int64_t *elt_records, SuLayout &S) {
    S.z = occ_sizes(tables->catalog, true);
    const int L = layers->n_layers;
    S.cap.assign(static_cast<size_t>(L), 0);
    S.region.assign(static_cast<size_t>(L), 0);
    for (int j = 0; j < L; ++j) {
        uint64_t c = 0;
        for (int q = layers->elt_off[j]; q < layers->elt_off[j + 1]; ++q) {
            const int64_t r = elt_records[layers->elt_ids[q]];
            if (r < 0) return fail(ARA_E_INVAL, "negative record count");
            c += static_cast<uint64_t>(std::min<int64_t>(r, tables->catalog));
        }
        S.cap[j] = c;
        S.region[j] = S.n_ent;
        S.n_ent += c;
    }
    return ARA_OK;
}

static size_t su_workspace(const ara_tables *tables, const ara_layers *layers, const SuLayout &S) {
    const int L = layers->n_layers;
    const int nJ = L > 0 ? layers->elt_off[L] : 0;
    const size_t n_sr = static_cast<size_t>(S.z.n_sr);
    Carver c(nullptr);
    c.take<int32_t>(kWsHeaderBytes / sizeof(int32_t));
    c.take<int32_t>(static_cast<size_t>(L + 1));
    c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    c.take<OccTables>(static_cast<size_t>(std::max(L, 1)));
    c.take<uint64_t>(static_cast<size_t>(std::max(L, 1)));   // capacities
    c.take<uint64_t>(static_cast<size_t>(std::max(L, 1)));   // regions
    c.take<uint64_t>(static_cast<size_t>(std::max(L, 1)));   // entries used
    size_t b = c.bytes();
    b += static_cast<size_t>(L) * S.z.per_layer;
    b += align256(static_cast<size_t>(L) * n_sr * kSr * sizeof(uint32_t));            // ooff
    b += align256(static_cast<size_t>(std::max(L, 1)) * n_sr * sizeof(uint32_t));     // otot
    b += align256(static_cast<size_t>(std::max(L, 1)) * (n_sr + 1) * sizeof(uint32_t));   // ubase
    b += align256(static_cast<size_t>(std::max(L, 1)) * n_sr * sizeof(uint32_t));     // obase
    b += align256(static_cast<size_t>(std::max<uint64_t>(S.n_ent, 1)) * sizeof(SuEntry));
    return b;
}

}  // namespace ara

using namespace ara;

extern "C" int32_t ara_build_elt_sigma(const ara_tables *tables, const int64_t *rec_off, const int32_t *rec_ids,
                                       const float *rec_sigma, float *sigma, void *stream) {
    if (!tables || !rec_off || !sigma) return fail(ARA_E_INVAL, "ara_build_elt_sigma: null pointer");
    const int32_t K = tables->n_elts, C = tables->catalog;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the records are checked on the host (a one-time build), then scattered
    std::vector<int64_t> off(static_cast<size_t>(K) + 1);
    ARA_HIP(hipMemcpyAsync(off.data(), rec_off, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ARA_HIP(hipStreamSynchronize(st));
    int64_t most = 0;
    for (int32_t k = 0; k < K; ++k) {
        if (off[k + 1] < off[k] || off[k] < 0) return fail(ARA_E_RANGE, "ara_build_elt_sigma: decreasing record offsets");
        most = std::max<int64_t>(most, off[k + 1] - off[k]);
    }
    const int64_t nrec = K > 0 ? off[K] - off[0] : 0;
    if (nrec > 0) {
        if (!rec_ids || !rec_sigma) return fail(ARA_E_INVAL, "ara_build_elt_sigma: null records");
        std::vector<int32_t> id(static_cast<size_t>(nrec));
        std::vector<float> sg(static_cast<size_t>(nrec));
        ARA_HIP(hipMemcpyAsync(id.data(), rec_ids + off[0], id.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        ARA_HIP(hipMemcpyAsync(sg.data(), rec_sigma + off[0], sg.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        ARA_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < nrec; ++i) {
            if (id[i] < 0 || id[i] >= C) return fail(ARA_E_RANGE, "ara_build_elt_sigma: an event ID outside [0, catalog)");
            if (!(sg[i] >= 0.0f) || !(sg[i] <= 3.402823466e38f))
                return fail(ARA_E_INVAL, "ara_build_elt_sigma: a negative or non-finite standard deviation");
        }
    }
    ARA_HIP(hipMemsetAsync(sigma, 0, static_cast<size_t>(K) * C * sizeof(float), st));
    if (nrec > 0) {
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((most + 255) / 256, 1024));
        k_sigma_scatter<<<dim3(gx, static_cast<unsigned>(K)), 256, 0, st>>>(rec_off, rec_ids, rec_sigma, C, sigma);
        ARA_HIP(hipGetLastError());
    }
    ARA_HIP(hipStreamSynchronize(st));
    return ARA_OK;
}

extern "C" int32_t ara_su_workspace_bytes(const ara_tables *tables, const ara_layers *layers,
                                          const int64_t *elt_records, size_t *bytes) {
    if (!tables || !bytes || !elt_records) return fail(ARA_E_INVAL, "null argument");
    int32_t rc = check_layers(layers, tables->n_elts);
    if (rc) return rc;
    SuLayout S;
    if ((rc = su_layout(tables, layers, elt_records, S))) return rc;
    *bytes = su_workspace(tables, layers, S);
    return ARA_OK;
}

extern "C" int32_t ara_ylt_forward_su(const ara_tables *tables, const float *sigma, const ara_yet *yet,
                                      const ara_layers *layers, const int64_t *elt_records, const double *elt_terms,
                                      const double *layer_terms, uint64_t seed, int64_t trial_begin,
                                      int64_t trial_end, double *ylt, double *s_pre, void *ws, size_t ws_bytes,
                                      void *stream) {
    if (!tables || !yet || !elt_records) return fail(ARA_E_INVAL, "null tables, YET or record counts");
    if (tables->catalog != yet->catalog) return fail(ARA_E_INVAL, "tables and YET use different catalogues");
    if (yet->range_bits != kRangeBits || yet->groups != kGroups) return fail(ARA_E_INVAL, "YET not prepared by this library");
    if (!yet->pos || !yet->t_off) return fail(ARA_E_INVAL, "YET prepared without ARA_PREP_POSITIONS");
    int32_t rc = check_layers(layers, tables->n_elts);
    if (rc) return rc;
    if (trial_begin < 0 || trial_end < trial_begin || trial_end > yet->n_trials)
        return fail(ARA_E_RANGE, "trial range outside the YET");
    if (!ws) return fail(ARA_E_INVAL, "null workspace");
    const int L = layers->n_layers;
    const int64_t n = trial_end - trial_begin;
    if (L > 0 && n > 0 && (!sigma || !elt_terms || !layer_terms || !ylt)) return fail(ARA_E_INVAL, "null input or output");
    SuLayout S;
    if ((rc = su_layout(tables, layers, elt_records, S))) return rc;
    if (ws_bytes < su_workspace(tables, layers, S)) return fail(ARA_E_NOSPACE, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L == 0 || n == 0) {
        ARA_HIP(hipMemsetAsync(ws, 0, kWsHeaderBytes, st));
        return ARA_OK;
    }
    const int nJ = layers->elt_off[L];
    const int n_sr = S.z.n_sr;
    Carver c(ws);
    int32_t *d_err = c.take<int32_t>(kWsHeaderBytes / sizeof(int32_t));
    int32_t *d_off = c.take<int32_t>(static_cast<size_t>(L + 1));
    int32_t *d_ids = c.take<int32_t>(static_cast<size_t>(std::max(nJ, 1)));
    OccTables *d_tabs = c.take<OccTables>(static_cast<size_t>(L));
    uint64_t *d_cap = c.take<uint64_t>(static_cast<size_t>(L));
    uint64_t *d_region = c.take<uint64_t>(static_cast<size_t>(L));
    uint64_t *d_used = c.take<uint64_t>(static_cast<size_t>(L));
    std::vector<OccTables> tabs(static_cast<size_t>(L));
    for (int j = 0; j < L; ++j) tabs[j] = occ_carve(c, S.z, true);
    uint32_t *ooff = c.take<uint32_t>(static_cast<size_t>(L) * n_sr * kSr);
    uint32_t *otot = c.take<uint32_t>(static_cast<size_t>(L) * n_sr);
    uint32_t *ubase = c.take<uint32_t>(static_cast<size_t>(L) * (n_sr + 1));
    uint32_t *obase = c.take<uint32_t>(static_cast<size_t>(L) * n_sr);
    SuEntry *ent = c.take<SuEntry>(static_cast<size_t>(std::max<uint64_t>(S.n_ent, 1)));
    HeadImage img(ws);
    img.cover(d_err + kWsHeaderBytes / sizeof(int32_t));
    img.put(d_off, layers->elt_off, static_cast<size_t>(L + 1));
    img.put(d_ids, layers->elt_ids, static_cast<size_t>(nJ));
    img.put(d_tabs, tabs.data(), tabs.size());
    img.put(d_cap, S.cap.data(), S.cap.size());
    img.put(d_region, S.region.data(), S.region.size());
    if ((rc = img.send(st))) return rc;

    {
        ProfScope prof(ARA_PROF_OCC, st);
        if ((rc = launch_occ(tables, d_off, d_ids, elt_terms, layer_terms, L, true, false, d_tabs, n_sr, d_err, st)))
            return rc;
        k_su_scan<<<dim3(static_cast<unsigned>(n_sr), static_cast<unsigned>(L)), kSuThreads, 0, st>>>(d_tabs, n_sr,
                                                                                                    ooff, otot);
        k_su_base<<<static_cast<unsigned>(L), kSuThreads, 0, st>>>(d_tabs, otot, n_sr, d_cap, ubase, obase, d_used,
                                                                  d_err);
        k_su_fill<<<dim3(static_cast<unsigned>(n_sr * kSuFillChunks), static_cast<unsigned>(L)), kSuThreads, 0, st>>>(
            tables->loss, sigma, tables->present, tables->catalog, tables->words, d_off, d_ids, d_tabs, n_sr, ooff,
            ubase, obase, d_cap, d_region, ent);
        const uint64_t most = *std::max_element(S.cap.begin(), S.cap.end());
        const unsigned px = static_cast<unsigned>(std::max<uint64_t>(1, std::min<uint64_t>((most + 255) / 256, 4096)));
        k_su_params<<<dim3(px, static_cast<unsigned>(L)), 256, 0, st>>>(d_region, d_cap, d_used, ent);
        ARA_HIP(hipGetLastError());
    }
    const int tb = yet->trials_per_block;
    if (tb < 1 || tb > kMaxTrialsPerBlock || yet->trials_per_group * kGroups != tb)
        return fail(ARA_E_INVAL, "YET not prepared by this library");
    const int b0 = static_cast<int>(trial_begin / tb);
    const int b1 = static_cast<int>((trial_end + tb - 1) / tb);
    SuParams P{};
    P.code = yet->code;
    P.pos = yet->pos;
    P.seg_base = yet->seg_base;
    P.seg_run = yet->seg_run;
    P.lane_start = yet->lane_start;
    P.t_off = yet->t_off;
    P.n_trials = yet->n_trials;
    P.tg = yet->trials_per_group;
    P.tb = tb;
    P.n_ranges = yet->n_ranges;
    P.n_sr = n_sr;
    P.b0 = b0;
    P.nb = b1 - b0;
    P.n_layers = L;
    P.t0 = trial_begin;
    P.t1 = trial_end;
    P.tabs = d_tabs;
    P.ubase = ubase;
    P.eregion = d_region;
    P.ecap = d_cap;
    P.eused = d_used;
    P.ent = ent;
    P.elt_off = d_off;
    P.elt_ids = d_ids;
    P.elt_terms = elt_terms;
    P.layer_terms = layer_terms;
    P.seed = seed;
    P.ylt = ylt;
    P.s_pre = s_pre;
    const int64_t groups = L == 1 ? P.nb : static_cast<int64_t>(kXcds) * ((P.nb + kXcds - 1) / kXcds) * L;
    if (groups > 0x7FFFFFFF) return fail(ARA_E_LIMIT, "too many workgroups");
    ProfScope prof(ARA_PROF_SU, st);
    if (L == 1)
        k_su_fwd<false><<<static_cast<unsigned>(groups), kSuThreads, 0, st>>>(P);
    else
        k_su_fwd<true><<<static_cast<unsigned>(groups), kSuThreads, 0, st>>>(P);
    ARA_HIP(hipGetLastError());
    return ARA_OK;
}
