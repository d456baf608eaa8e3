// Occurrence tables shared by the forward and the backward.
//
// Steps one to three of Algorithm 1 (look up each ELT's loss, apply that
// ELT's financial terms, sum over the layer's ELTs in listed order, apply the
// occurrence retention and limit) depend only on the event, not on the trial.
// They are therefore evaluated once per catalogue event and per call, and the
// result O(e) is stored compactly per "super-range" of 65,536 events:
//   br[s][w]   = {bits of word w (events 32w..32w+31 of super-range s),
//                 number of set bits in words 0..w-1}
//   vals[s][i] = O of the i-th set event of super-range s (binary64)
//   cnt[s][i]  = number of the layer's ELTs holding that event (hits mode)
// built in two steps: each chunk of 4096 events finds its set events, their
// bitmap words and count, and O in event order at the start of the chunk's
// slice of `dense`; then every chunk's ranks start after the earlier chunks'
// counts and its values move into `vals`.
// The set events are those with O != 0 ("hot"), or, when hit counts are
// requested, every event present in at least one of the layer's ELTs.
#pragma once

#include "ara_internal.h"

namespace ara {

constexpr int kMaxJ = ARA_MAX_ELTS_PER_LAYER;
constexpr int kOccChunkWords = 128;                    // 4096 events per chunk
constexpr int kOccChunks = kSrWords / kOccChunkWords;   // 16 chunks per super-range

struct OccTables {
    uint2 *br;          // [n_sr][kSrWords]
    double *vals;       // [n_sr][kSr]
    uint8_t *cnt;       // [n_sr][kSr] or null
    int32_t *count;     // [n_sr]
    int32_t *pcount;    // [n_sr][kOccChunks]  set events per chunk (phase one)
    uint32_t *bits;     // [n_sr][kSrWords]  set-event bitmap (phase one)
    double *dense;      // [n_sr][kSr]       O of each chunk's set events, from the chunk's start (phase one)
    uint8_t *dense_nb;  // [n_sr][kSr]       their ELT counts (hits mode)
};

// min(max(v - R, 0), L), evaluated exactly as the oracle does: a separately
// rounded subtraction and two selects (no fused operations; the build uses
// -ffp-contract=off).
__device__ __forceinline__ double xl(double v, double r, double lim) {
    const double y = v - r;
    const double a = (y > 0.0) ? y : 0.0;
    return (a < lim) ? a : lim;
}

struct OccLayoutSizes {
    int n_sr;
    size_t per_layer;
    size_t br, vals, cnt, count, pcount, bits, dense, dense_nb;
};

inline OccLayoutSizes occ_sizes(int32_t catalog, bool with_cnt) {
    OccLayoutSizes z{};
    z.n_sr = (catalog + kSr - 1) / kSr;
    z.br = align256(static_cast<size_t>(z.n_sr) * kSrWords * sizeof(uint2));
    z.vals = align256(static_cast<size_t>(z.n_sr) * kSr * sizeof(double));
    z.cnt = with_cnt ? align256(static_cast<size_t>(z.n_sr) * kSr) : 0;
    z.count = align256(static_cast<size_t>(z.n_sr) * sizeof(int32_t));
    z.pcount = align256(static_cast<size_t>(z.n_sr) * kOccChunks * sizeof(int32_t));
    z.bits = align256(static_cast<size_t>(z.n_sr) * kSrWords * sizeof(uint32_t));
    z.dense = align256(static_cast<size_t>(z.n_sr) * kSr * sizeof(double));
    z.dense_nb = with_cnt ? align256(static_cast<size_t>(z.n_sr) * kSr) : 0;
    z.per_layer = z.br + z.vals + z.cnt + z.count + z.pcount + z.bits + z.dense + z.dense_nb;
    return z;
}

inline OccTables occ_carve(Carver &c, const OccLayoutSizes &z, bool with_cnt) {
    OccTables t{};
    t.br = c.take<uint2>(static_cast<size_t>(z.n_sr) * kSrWords);
    t.vals = c.take<double>(static_cast<size_t>(z.n_sr) * kSr);
    t.cnt = with_cnt ? c.take<uint8_t>(static_cast<size_t>(z.n_sr) * kSr) : nullptr;
    t.count = c.take<int32_t>(static_cast<size_t>(z.n_sr));
    t.pcount = c.take<int32_t>(static_cast<size_t>(z.n_sr) * kOccChunks);
    t.bits = c.take<uint32_t>(static_cast<size_t>(z.n_sr) * kSrWords);
    t.dense = c.take<double>(static_cast<size_t>(z.n_sr) * kSr);
    t.dense_nb = with_cnt ? c.take<uint8_t>(static_cast<size_t>(z.n_sr) * kSr) : nullptr;
    return t;
}

// Members (layers, or quotes of the server) that one workgroup of the
// grouped forward serves together.
constexpr int kGrpMax = 4;

// The union of a group's set events, per super-range: the union bitmap with
// ranks (as an occurrence table's br), its count, and for every member its
// set events as a bitmap over the union's ranks: word k of sbr[m] holds union
// ranks 32k..32k+31 of the super-range, {bit set iff the member's O != 0 for
// that event, the member's rank of the first of them} -- the member's rank of
// an event is its index in the member's own occurrence-table values.
struct GrpTables {
    uint2 *ubr;                     // [n_sr][kSrWords]
    int32_t *ucount;                // [n_sr]
    uint2 *sbr;                     // [kGrpMax][n_sr][kSrWords]
    const OccTables *mt[kGrpMax];   // the members' occurrence tables (device)
    int32_t n;                      // members
    int32_t pad;
};

// One unit of grouped forward work: the members of one group over one block
// of trials; member m writes its trials in [t0[m], t1[m]) (rows indexed
// t - t0[m]).  block -1 marks an empty slot (the workgroup exits at once).
struct GrpItem {
    const GrpTables *gt;            // device
    int32_t block;
    int32_t n;                      // members
    uint32_t mask;                  // members to serve on this block (bit m); others are skipped
    const double *lterm[kGrpMax];   // (OccR, OccL, AggR, AggL) of each member
    int64_t t0[kGrpMax], t1[kGrpMax];
    double *ylt[kGrpMax];
    double *s_pre[kGrpMax];         // or null
};

// Members one grouped-forward workgroup holds with blocks of tb trials (0 if
// not even one leaves room for the table slices).
int grp_max_members(int tb);
// Builds the union tables of n_groups groups (their mt and n set).
int32_t launch_grp_union(const GrpTables *d_gts, int n_groups, int n_sr, hipStream_t st);
// The grouped forward over a device array of items (one workgroup each, a
// whole CU's LDS per workgroup).
int32_t launch_fwd_group(const ara_yet *yet, const GrpItem *d_items, int n_items, int gmax, hipStream_t st);

// One unit of forward work: one layer over one block of trials, with the
// trial range [t0, t1) whose outputs are written (row bases indexed t - t0).
struct FwdItem {
    const OccTables *tab;      // device pointer to the layer's occurrence tables
    const double *lterm;       // device pointer to the layer's (OccR, OccL, AggR, AggL)
    int32_t block;
    int32_t pad;
    int64_t t0, t1;
    double *ylt;
    double *s_pre;             // or null
    int32_t *hits;             // or null
};

// Enqueue the forward streaming kernel over a device array of items.
// The regular set of forward items: every layer over the blocks b0 ..
// b0 + nb - 1 of one trial range [t0, t1), rows of ylt / s_pre / hits
// indexed t - t0 (formed on the device, so nothing is copied per call).
struct FwdRegular {
    const OccTables *tabs;     // device, [n_layers]
    const double *lterm;       // device, [n_layers][4]
    double *ylt, *s_pre;
    int32_t *hits;
    int64_t t0, t1;
    int32_t b0, nb;
    int32_t nl;                // layers
};

// Workgroups of a regular launch: one per block with one layer; with L
// layers, L per block over whole groups of kXcds blocks (the XCD-aware
// mapping of the forward kernel; workgroups past the last block exit).
inline int fwd_regular_items(int n_layers, int nb) {
    if (n_layers <= 1) return nb;
    return n_layers * kXcds * ((nb + kXcds - 1) / kXcds);
}

// LDS plan of a forward workgroup (bytes of the table-slice buffer, values
// it holds); ARA_E_LIMIT when the layout leaves no room for a slice.
int32_t fwd_lds_plan(int tb, int n_ranges, bool hits, bool f32, int32_t *buf_bytes, int32_t *capv);

// f32: binary32 occurrence values (tables built with f32_vals) and totals.
// Items come from d_items, or (d_items null) from `reg`.
// shared: workgroups of the same block are adjacent on one XCD, so the codes
// are loaded through L2 (a regular set decides this from its layer count).
int32_t launch_forward(const ara_yet *yet, int n_sr, bool hits, bool f32, const FwdItem *d_items, int n_items,
                       hipStream_t st, const FwdRegular *reg = nullptr, bool shared = false);

// Checks the arguments of a forward call (those of ara_ylt_forward but the
// workspace); *need receives the workspace bytes the call takes.
int32_t forward_args(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, const double *elt_terms,
                     const double *layer_terms, int64_t trial_begin, int64_t trial_end, uint32_t flags,
                     const double *ylt, const int32_t *hits, size_t *need);
// Enqueues a checked forward call with at least one layer and one trial on
// `st`, over a workspace of at least the bytes forward_args gave (its first
// int32 receives the device-side status).
int32_t forward_run(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers, const double *elt_terms,
                    const double *layer_terms, int64_t trial_begin, int64_t trial_end, uint32_t flags, double *ylt,
                    double *s_pre, int32_t *hits, void *ws, hipStream_t st);

// A layer's set-event bitmap folded onto 2^20 bits by OR (128 KB, staged in
// LDS by the kernels that stream the trial-major YET): one filter per layer.
constexpr int kFilterWords = 1 << 15;
int32_t launch_set_filter(const OccTables *d_tabs, int n_words, uint32_t *filter, int n_layers, hipStream_t st);

// Validates the layer list on the host; returns ARA_OK or an error.
int32_t check_layers(const ara_layers *layers, int32_t n_elts);

// Enqueue the occurrence-table kernel for every layer.  `tabs` has one entry
// per layer; the layer CSR must already be on the device.  f32_vals stores
// each O rounded to binary32 (vals then holds floats at the same indices).
int32_t launch_occ(const ara_tables *tables, const int32_t *d_elt_off, const int32_t *d_elt_ids,
                   const double *elt_terms, const double *layer_terms, int32_t n_layers, bool union_mode,
                   bool f32_vals, OccTables *d_tabs, int n_sr, int32_t *d_err, hipStream_t st);

}  // namespace ara
