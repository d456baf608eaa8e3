/*
 * ara.h -- C ABI of the MI355X (gfx950) aggregate-risk-analysis library.
 *
 * The operation is the aggregate analysis of Bahl, Baltzer, Rau-Chaplin,
 * Varghese and Whiteway (arXiv 1308.2572), Section II and Algorithm 1: for every
 * layer and every trial of a Year Event Table (YET), look up each event
 * occurrence's loss in the layer's Event Loss Tables (ELTs), apply each ELT's
 * financial terms, sum across the layer's ELTs, apply the layer's occurrence
 * retention and limit, then apply the aggregate retention and limit to the
 * trial's running total; the result per (layer, trial) is the year loss, the
 * rows of the Year Loss Table (YLT).  Tail metrics (mean annual loss, PML,
 * TVaR; named in Section I) and their gradients complete the surface.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int32_t status (ARA_OK on success).  On error
 *    ara_last_error() gives a thread-local detail string.  No C++ exception
 *    crosses this boundary.
 *  - Bulk memory is caller-owned DEVICE memory unless a field says "host".
 *    The library never allocates device memory: each operation that needs
 *    scratch space has a *_bytes query, and the caller passes a device buffer
 *    of at least that size (256-byte aligned).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it and outputs are valid once the stream has completed,
 *    except where a function says it synchronises.
 *  - Event IDs are 0-based int32 in [0, catalog).  Losses are binary32, >= 0
 *    and finite.  Terms are binary64; retentions are finite and >= 0; limits
 *    are > 0 or +infinity; scales are finite and > 0.
 *  - Readings of points the paper leaves open (stated once here):
 *      financial terms of ELT k:  g_k(l) = min(max(s_k*l - R_k, 0), L_k)
 *      every min(max(v - R, 0), L) is evaluated as y = v - R;
 *        a = y > 0 ? y : 0; out = a < L ? a : L   (binary64, no fused ops)
 *      an event absent from an ELT (or stored with loss 0) loses 0
 *      hits(layer, trial) = number of (occurrence, ELT) pairs with loss != 0
 *      tail count r = N - floor(p*N + 1e-9) clamped to [1, N];
 *        PML_p = r-th largest year loss; TVaR_p = mean of the r largest
 */
#ifndef ARA_H
#define ARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ARA_ABI_VERSION 2

/* status codes */
#define ARA_OK        0
#define ARA_E_INVAL   1   /* null pointer, bad size, bad flag, p outside (0,1), invalid term value */
#define ARA_E_RANGE   2   /* event ID outside [0, catalog), decreasing offsets, ELT index out of range */
#define ARA_E_DUP     3   /* the same event twice in one ELT (ELTs are dictionaries, Section III) */
#define ARA_E_NOSPACE 4   /* caller buffer smaller than the *_bytes query */
#define ARA_E_HIP     5   /* HIP runtime error */
#define ARA_E_LIMIT   6   /* size beyond a documented implementation limit */
#define ARA_E_BUSY    7   /* not an error: the quote is not finished yet (poll, cancel) */

/* forward flags */
#define ARA_F_EMIT_HITS   1u  /* also produce per-(layer, trial) hit counts */
#define ARA_F_FP32_ACCUM  2u  /* binary32 occurrence values and trial totals (the precision reduction of the
                                 optimised kernel, Sections III-IV); hits unchanged; YLT within 1e-5 of
                                 the binary64 result relative to max(YLT, total) */

/* implementation limits */
#define ARA_MAX_CATALOG       (1 << 26)   /* events in the catalogue */
#define ARA_MAX_ELTS_PER_LAYER 128
#define ARA_MAX_COTANGENTS     4
#define ARA_MAX_LAYERS         65535      /* layers per call (each layer is one row of a launch grid) */

const char *ara_status_string(int32_t status);
const char *ara_last_error(void);
int32_t ara_abi_version(void);

/* ------------------------------------------------------------------------ */
/* YET: the first input (Section II) -- trials of time-ordered event IDs.    */
/* ------------------------------------------------------------------------ */
/*
 * Preprocessing (the paper's first stage loads the YET into memory; here it
 * is laid out once for the device).  The prepared YET groups each block of
 * consecutive trials by catalogue range: for block b, range r (2^range_bits
 * consecutive event IDs) and trial group g, the occurrences of those trials
 * whose event lies in range r form a segment, in trial order, one 16-bit code
 * per occurrence: bits 0..14 the event's offset in the range, bit 15 "advance
 * to the next trial of the group first".  The code 0xFFFF advances without an
 * event: it stands for a trial of the group with no event in the range, for
 * the advance of an event at offset 0x7FFF that opens a trial (the event then
 * follows as 0x7FFF), and for padding.  The padded segment is dealt to 64
 * lanes as runs of seg_run consecutive codes (a multiple of 4); lane j starts
 * at trial lane_start[j] of its group and its code s sits at
 * seg_base + (s/4)*256 + 4*j + s%4.
 * Order of occurrences inside a trial is kept within a segment but not across
 * ranges: the year loss does not depend on it (the cumulative aggregate steps
 * telescope), and the order of summation, so rounding, is fixed by this
 * layout and deterministic.
 *
 * With ARA_PREP_TRANSPOSED the buffer also holds the event-major copy the
 * backward needs (the adjoint of the per-trial gather is a per-event
 * scatter; stored transposed it becomes a gather again).  The trials are
 * cut into n_slices slices of slice_trials consecutive trials; for slice x
 * and event e the occurrences are the list
 *     tr_ent[tr_off[x*catalog + e] .. tr_off[x*catalog + e + 1])
 * of trial indices local to the slice (trial = x*slice_trials + entry), one
 * entry per occurrence, in no particular order.
 */
typedef struct ara_yet {
    int64_t   n_trials;
    int64_t   nnz;               /* total event occurrences */
    int32_t   catalog;
    int32_t   range_bits;        /* 15 */
    int32_t   n_ranges;          /* ceil(catalog / 2^range_bits) */
    int32_t   groups;            /* trial groups per block (16, one per wavefront) */
    int32_t   trials_per_group;
    int32_t   trials_per_block;  /* groups * trials_per_group, <= 4096 */
    int32_t   n_blocks;          /* ceil(n_trials / trials_per_block) */
    int32_t   max_occ;           /* largest number of occurrences of one event */
    int64_t   n_codes;           /* 16-bit codes including gap codes and padding */
    uint16_t *code;              /* device [n_codes + 256]: the last 256 are skip codes (0xFFFF) */
    int64_t  *seg_base;          /* device [n_blocks][n_ranges][groups]: the segment's first code */
    int32_t  *seg_run;           /* device [n_blocks][n_ranges][groups]: codes per lane */
    uint8_t  *lane_start;        /* device [n_blocks][n_ranges][groups][64]: each lane's first trial */
    /* event-major copy (ARA_PREP_TRANSPOSED; n_slices = 0 and NULL otherwise) */
    int32_t   n_slices;          /* 8 */
    int32_t   reserved;
    int64_t   slice_trials;      /* a multiple of trials_per_block */
    int64_t  *tr_off;            /* device [n_slices * catalog + 1] */
    uint32_t *tr_ent;            /* device [nnz] */
    /* trial-major copy of the input (ARA_PREP_TRIAL_MAJOR; NULL otherwise) */
    int64_t  *t_off;             /* device [n_trials + 1] (also with ARA_PREP_POSITIONS) */
    int32_t  *t_ids;             /* device [nnz] */
    int32_t  *t_cnt;             /* device [catalog]: occurrences of each event */
    /* positions (ARA_PREP_POSITIONS; NULL otherwise) */
    uint16_t *pos;               /* device [n_codes + 256]: at each occurrence code's index, the
                                    occurrence's position in its trial (its index in ids less
                                    offsets[trial]); 0xFFFF at gap codes and padding (the code
                                    itself tells these from an occurrence at position 65535) */
} ara_yet;

/* prepare flags */
#define ARA_PREP_TRANSPOSED 1u   /* also build the event-major copy (needed by ara_ylt_backward) */
#define ARA_PREP_TRIAL_MAJOR 2u  /* also keep a trial-major copy of offsets and ids: lets ara_ylt_backward
                                    handle cotangents that are constant over most trials (the metrics')
                                    from the deviating trials' own events */
#define ARA_PREP_POSITIONS 4u    /* also store each occurrence's position in its trial beside its code
                                    (and a copy of offsets): needed by ara_ylt_forward_su, whose draws
                                    are keyed by the trial-major occurrence index; every trial must then
                                    hold at most 65536 occurrences (ARA_E_LIMIT otherwise) */

/* Upper bound of the device buffer ara_yet_prepare needs for these flags. */
int32_t ara_yet_prepare_bytes(int64_t n_trials, int64_t nnz, int32_t catalog, uint32_t flags, size_t *bytes);

/*
 * offsets: device int64 [n_trials+1], offsets[0] = 0, non-decreasing; trial t
 *          holds ids[offsets[t] .. offsets[t+1]).
 * ids:     device int32 [offsets[n_trials]].
 * flags:   ARA_PREP_TRANSPOSED, ARA_PREP_TRIAL_MAJOR, ARA_PREP_POSITIONS (ARA_E_INVAL
 *          for other bits).
 * buf:     device buffer of at least ara_yet_prepare_bytes (same flags); it
 *          holds the prepared YET afterwards and must outlive every use of *out.
 * Validates every ID (ARA_E_RANGE) and every offset.  SYNCHRONISES `stream`
 * (it sizes the layout from device-side counts); one-time cost.
 * ARA_E_LIMIT if one (slice, catalogue range) of the event-major copy would
 * hold 2^32 occurrences or more, or with ARA_PREP_POSITIONS if a trial holds
 * more than 65536 occurrences.
 */
int32_t ara_yet_prepare(const int64_t *offsets, const int32_t *ids, int64_t n_trials,
                        int32_t catalog, uint32_t flags, void *buf, size_t buf_bytes,
                        void *stream, ara_yet *out);

/* ------------------------------------------------------------------------ */
/* ELTs: the second input (Section II) -- event -> loss dictionaries, held as */
/* direct-access tables over the whole catalogue (Section III).              */
/* ------------------------------------------------------------------------ */
typedef struct ara_tables {
    int32_t   n_elts;
    int32_t   catalog;
    int32_t   words;             /* ceil(catalog / 32) */
    int32_t   reserved;
    float    *loss;              /* device [n_elts][catalog]; 0 = absent */
    uint32_t *present;           /* device [n_elts][words]; bit e%32 of word e/32 set iff loss != 0 */
} ara_tables;

int32_t ara_build_elt_tables_bytes(int32_t n_elts, int32_t catalog, size_t *bytes);

/*
 * rec_off:  device int64 [n_elts+1]; ELT k holds records rec_off[k]..rec_off[k+1]
 * rec_ids:  device int32 event IDs, distinct within one ELT (ARA_E_DUP otherwise)
 * rec_loss: device binary32 losses (>= 0, finite; ARA_E_INVAL otherwise)
 * buf:      device buffer of at least ara_build_elt_tables_bytes; holds the
 *           tables afterwards.  SYNCHRONISES `stream` to report errors.
 */
int32_t ara_build_elt_tables(int32_t n_elts, int32_t catalog, const int64_t *rec_off,
                             const int32_t *rec_ids, const float *rec_loss,
                             void *buf, size_t buf_bytes, void *stream, ara_tables *out);

/* ------------------------------------------------------------------------ */
/* Layers: the third input (Section II) -- ELT lists plus layer terms.       */
/* ------------------------------------------------------------------------ */
typedef struct ara_layers {
    int32_t        n_layers;
    int32_t        reserved;
    const int32_t *elt_off;      /* HOST [n_layers+1] */
    const int32_t *elt_ids;      /* HOST [elt_off[n_layers]] ELT indices, listed order */
} ara_layers;

/* ------------------------------------------------------------------------ */
/* Forward: Algorithm 1 for trials [trial_begin, trial_end) of every layer.  */
/* ------------------------------------------------------------------------ */
int32_t ara_ylt_workspace_bytes(const ara_tables *tables, const ara_yet *yet,
                                const ara_layers *layers, uint32_t flags, size_t *bytes);

/*
 * elt_terms:   device binary64 [n_elts][3] = (scale s_k, retention R_k, limit L_k)
 * layer_terms: device binary64 [n_layers][4] = (OccR, OccL, AggR, AggL)
 * ylt:         device binary64 [n_layers][n], n = trial_end - trial_begin
 * s_pre:       device binary64 [n_layers][n] or NULL: the trial's total of
 *              occurrence losses before aggregate terms (kept for the backward;
 *              with ARA_F_FP32_ACCUM the binary32 total, widened exactly)
 * flags:       ARA_F_EMIT_HITS, ARA_F_FP32_ACCUM (ARA_E_INVAL for other bits)
 * hits:        device int32 [n_layers][n] or NULL; requires ARA_F_EMIT_HITS
 * ws:          device workspace of at least ara_ylt_workspace_bytes
 * Invalid term values are detected on the device: ara_check_device_error.
 */
int32_t ara_ylt_forward(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                        const double *elt_terms, const double *layer_terms,
                        int64_t trial_begin, int64_t trial_end, uint32_t flags,
                        double *ylt, double *s_pre, int32_t *hits,
                        void *ws, size_t ws_bytes, void *stream);

/* Reads (synchronising `stream`) the error word the device side of the
 * forward or backward left in `ws`; ARA_OK if none. */
int32_t ara_check_device_error(const void *ws, void *stream);

/*
 * The forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and results as ara_ylt_forward, with no workspace
 * argument.  Its workspace is a scratch array of ARA_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on, from the first call on
 * that device until the process ends; the call allocates and frees nothing.
 * A call that needs more workspace than the scratch holds (the
 * ara_ylt_workspace_bytes figure: about 32 MiB per layer at a 2,000,000-event
 * catalogue) returns ARA_E_LIMIT before any device work.  Every call on one
 * device shares that device's scratch and leaves its contents behind; each
 * call rewrites what it reads, so no state carries over, but calls that
 * overlap on one device (other streams, other host threads) race: serialise
 * them.
 * dev_status: device int32 or NULL; receives the device-side status of the
 *             call (invalid term values: ARA_E_INVAL), 0 if none, at the end
 *             of the call on `stream`.  ara_check_device_error(dev_status,
 *             stream) reads it.
 * The other arguments are those of ara_ylt_forward.
 */
#define ARA_NOALLOC_SCRATCH_BYTES (160u << 20)
int32_t ara_ylt_forward_noalloc(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                                const double *elt_terms, const double *layer_terms,
                                int64_t trial_begin, int64_t trial_end, uint32_t flags,
                                double *ylt, double *s_pre, int32_t *hits,
                                int32_t *dev_status, void *stream);

/* ------------------------------------------------------------------------ */
/* Per-occurrence losses: step four of Algorithm 1 taken literally, per      */
/* occurrence in storage order (the event-level YLT), and the per-year       */
/* maximum occurrence loss behind occurrence-exceedance metrics.             */
/* ------------------------------------------------------------------------ */
int32_t ara_yelt_workspace_bytes(const ara_tables *tables, const ara_layers *layers, size_t *bytes);

/*
 * offsets, ids: the trial-major YET on the device (as given to
 *              ara_yet_prepare; storage order matters here), n_trials trials.
 * occ_begin:   offsets[trial_begin]; occ_count: offsets[trial_end] - occ_begin
 *              (host values; a mismatch is a device-side ARA_E_RANGE).
 * yelt:        device binary64 [n_layers][occ_count]: occurrence d of trial t
 *              gets f_agg(S_{t,d}) - f_agg(S_{t,d-1}), S_{t,d} the running total
 *              of the trial's occurrence losses (S_{t,0} = 0); a trial's values
 *              sum to its year loss.
 * occ_max:     device binary64 [n_layers][trial_end - trial_begin]: the largest
 *              of the trial's values (0 for an empty trial).
 * Event IDs outside [0, catalog) are a device-side ARA_E_RANGE
 * (ara_check_device_error on ws); the running total is summed in wavefront
 * order, so values agree with a sequential sum to rounding.
 */
int32_t ara_yelt_forward(const ara_tables *tables, const int64_t *offsets, const int32_t *ids,
                         int64_t n_trials, const ara_layers *layers, const double *elt_terms,
                         const double *layer_terms, int64_t trial_begin, int64_t trial_end,
                         int64_t occ_begin, int64_t occ_count, double *yelt, double *occ_max,
                         void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Metrics from the YLT (Section I names PML and TVaR).                      */
/* ------------------------------------------------------------------------ */
int32_t ara_metrics_workspace_bytes(int32_t n_layers, int64_t n, size_t *bytes);

/*
 * ylt:     device binary64 [n_layers][n], every value >= 0
 * out:     device binary64 [n_layers][3] = (AAL, PML_p, TVaR_p)
 * weights: device binary64 [3][n_layers][n] = d(AAL, PML, TVaR)/d ylt, or NULL.
 *          Ties at the PML value share its weight equally; TVaR gives 1/r to
 *          trials above the PML value and (r - #above)/(r * #tied) to ties.
 * p in (0, 1).
 */
int32_t ara_metrics(const double *ylt, int32_t n_layers, int64_t n, double p,
                    double *out, double *weights, void *ws, size_t ws_bytes, void *stream);

/*
 * Vector-Jacobian product of the metrics: grad_ylt[j][t] =
 *   sum_m grad_out[j][m] * weights[m][j][t]   (m = AAL, PML, TVaR)
 * weights as produced by ara_metrics; grad_out device [n_layers][3];
 * grad_ylt device [n_layers][n] (overwritten).
 */
int32_t ara_metrics_vjp(const double *weights, int32_t n_layers, int64_t n, const double *grad_out,
                        double *grad_ylt, void *stream);

/* ------------------------------------------------------------------------ */
/* Backward: gradients of sum_t grad_ylt[c][j][t] * ylt[j][t] with respect to */
/* every ELT term and layer term (the reverse sweep of Algorithm 1).        */
/* ------------------------------------------------------------------------ */
int32_t ara_ylt_backward_workspace_bytes(const ara_tables *tables, const ara_yet *yet,
                                         const ara_layers *layers, int32_t n_cot, size_t *bytes);

/*
 * s_pre:      device [n_layers][n] as produced by ara_ylt_forward for the same
 *             inputs and trial range
 * grad_ylt:   device binary64 [n_cot][n_layers][n], n_cot in [1, ARA_MAX_COTANGENTS]
 * grad_elt:   device binary64 [n_cot][n_elts][3]   (overwritten; ELTs in no layer get 0)
 * grad_layer: device binary64 [n_cot][n_layers][4] (overwritten)
 * Subgradients follow the evaluated branch of each min/max: d/dv = [y>0 && a<L],
 * d/dR = -[y>0 && a<L], d/dL = [a >= L].  Deterministic (fixed-point
 * accumulation of the per-event weights, fixed-order reductions).
 * The YET must have been prepared with ARA_PREP_TRANSPOSED (ARA_E_INVAL
 * otherwise).  With ARA_PREP_TRIAL_MAJOR too, cotangents that take one value
 * on all but a sixteenth of the trials (the metrics' weights) are served from
 * the deviating trials' own events; the result is the same bit for bit.
 */
int32_t ara_ylt_backward(const ara_tables *tables, const ara_yet *yet, const ara_layers *layers,
                         const double *elt_terms, const double *layer_terms,
                         int64_t trial_begin, int64_t trial_end, const double *s_pre,
                         int32_t n_cot, const double *grad_ylt,
                         double *grad_elt, double *grad_layer,
                         void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Secondary uncertainty (named as future work in Section VI): every         */
/* (occurrence, ELT) pair draws its loss instead of looking up the mean.     */
/* ------------------------------------------------------------------------ */
/*
 * The model (the paper gives none): an ELT record carries a standard
 * deviation sigma beside its mean loss mu; occurrence i (its index in the
 * trial-major YET) of an event the ELT holds draws
 *   x = mu                      if sigma = 0,
 *   x = exp(m + s z)            otherwise, s^2 = ln(1 + sigma^2/mu^2),
 *                               m = ln mu - s^2/2 (lognormal, mean mu, sd sigma),
 *   z = sqrt(-2 ln u1) cos(2 pi u2),  u1 = (((w1 2^32 + w0) >> 12) + 1/2) 2^-52,
 *   u2 likewise from (w3, w2), (w0, w1, w2, w3) = Philox4x32-10 block
 *   (Salmon, Moraes, Dror, Shaw, SC'11) of counter words (i mod 2^32,
 *   i div 2^32, k, 0) under key words (seed mod 2^32, seed div 2^32), k the
 *   ELT's index,
 * and x replaces the table lookup of step one of Algorithm 1; steps two to
 * four are unchanged.  The same occurrence and ELT draw the same loss in
 * every layer and every call with the same seed.
 */

/*
 * rec_off, rec_ids: the device CSR given to ara_build_elt_tables
 * rec_sigma:        device binary32 standard deviations, one per record
 *                   (>= 0 and finite; ARA_E_INVAL otherwise)
 * sigma:            caller's device binary32 [n_elts][catalog], filled here
 *                   (0 for events the ELT does not hold)
 * SYNCHRONISES `stream` to report errors.
 */
int32_t ara_build_elt_sigma(const ara_tables *tables, const int64_t *rec_off, const int32_t *rec_ids,
                            const float *rec_sigma, float *sigma, void *stream);

/* elt_records: HOST int64 [n_elts], the records of each ELT (bounds the
 * (event, ELT) pairs each layer draws for). */
int32_t ara_su_workspace_bytes(const ara_tables *tables, const ara_layers *layers, const int64_t *elt_records,
                               size_t *bytes);

/*
 * yet:         prepared with ARA_PREP_POSITIONS (ARA_E_INVAL otherwise): the
 *              draws are keyed by each occurrence's index in the trial-major
 *              YET given to ara_yet_prepare, which the positions recover.
 * ylt, s_pre:  device binary64 [n_layers][trial_end - trial_begin] (s_pre may
 *              be NULL): Algorithm 1 with the draws above.
 * ws:          device workspace of at least ara_su_workspace_bytes for the same
 *              elt_records (ARA_E_NOSPACE otherwise; an ELT holding more
 *              events than its elt_records is a device-side ARA_E_LIMIT).
 * A trial's occurrence losses are summed in an order fixed by the prepared
 * layout (not the trial's storage order), so S and the YLT agree with a
 * sequential sum to rounding, and do not depend on the trial range or on the
 * other layers of the call; everything else follows the definition step by
 * step in binary64.
 */
int32_t ara_ylt_forward_su(const ara_tables *tables, const float *sigma, const ara_yet *yet,
                           const ara_layers *layers, const int64_t *elt_records, const double *elt_terms,
                           const double *layer_terms, uint64_t seed, int64_t trial_begin, int64_t trial_end,
                           double *ylt, double *s_pre, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Quote server: continuous batching of pricing requests over the resident   */
/* YET and ELT tables (the paper motivates real-time pricing, Sections I, V). */
/* ------------------------------------------------------------------------ */
/*
 * A quote is a candidate layer over the resident ELTs with its own terms,
 * over a contiguous trial range.  A scheduler thread admits quotes in arrival
 * order as soon as a slot and enough arena memory are free.  The active
 * quotes are served by a circular scan of the YET's trial blocks: every
 * iteration is ONE forward launch over a window of consecutive blocks,
 * holding each active quote's work on each block of the window in its range,
 * the work items of one block on one XCD back to back so that the quotes
 * sharing the block read its codes from HBM once.  A quote arriving while
 * others run joins at the next iteration and is complete after one
 * revolution over its range.  Results do not depend on the mix.  All device
 * memory comes from the caller's arena; the resident ELT terms are checked
 * once, at create (ARA_E_INVAL).
 */
typedef struct ara_quote {
    int32_t        n_elts;
    int32_t        want_grad;       /* also return d(AAL, PML, TVaR)/d(every term) */
    const int32_t *elt_ids;         /* HOST [n_elts] indices into the resident ELT set, listed order */
    double         layer_terms[4];  /* OccR, OccL, AggR, AggL */
    int64_t        trial_begin, trial_end;
    double         p;               /* tail probability of PML and TVaR, in (0, 1) */
} ara_quote;

typedef struct ara_quote_result {
    int32_t status;
    int32_t n_elts;
    double  metrics[3];             /* AAL, PML_p, TVaR_p */
    double  grad_layer[3][4];       /* [metric][OccR, OccL, AggR, AggL] (want_grad) */
    double *grad_elt;               /* caller's HOST [3][n_elts][3] (scale, retention, limit), or NULL */
    double  t_submit_ms, t_admit_ms, t_done_ms;   /* host steady clock */
} ara_quote_result;

/* Arena bytes that hold `quotes_with_grad` full-range quotes with gradients. */
int32_t ara_server_arena_bytes(const ara_tables *tables, const ara_yet *yet, int32_t quotes_with_grad,
                               size_t *bytes);
/* elt_terms: device [n_elts][3] terms of the resident ELTs; arena: device
 * buffer owned by the caller for the server's lifetime; max_slots <= 256. */
int32_t ara_server_create(const ara_tables *tables, const ara_yet *yet, const double *elt_terms,
                          void *arena, size_t arena_bytes, int32_t max_slots, void **server);
/* Validates and enqueues; ARA_E_NOSPACE if the quote can never fit the arena;
 * ARA_E_INVAL for a quote with gradients when the resident YET was prepared
 * without ARA_PREP_TRANSPOSED. */
int32_t ara_server_submit(void *server, const ara_quote *quote, int64_t *ticket);
/* ARA_OK and *out filled when finished (the ticket is then retired), ARA_E_BUSY otherwise. */
int32_t ara_server_poll(void *server, int64_t ticket, ara_quote_result *out);
/* Blocks until the quote is finished; fills *out and retires the ticket. */
int32_t ara_server_wait(void *server, int64_t ticket, ara_quote_result *out);
/* Cancels a quote still in the queue (ARA_E_BUSY once it is on the device). */
int32_t ara_server_cancel(void *server, int64_t ticket);
/* stats[9] = iterations, packed forward launches, most quotes in one launch,
 * queued, active, free arena bytes, work items launched, items on a block
 * that other items of the same launch share, most quotes finished after one
 * launch (their metrics share one set of launches). */
int32_t ara_server_stats(void *server, int64_t *stats);
/* Stops admitting, drains the active quotes, frees host resources. */
int32_t ara_server_destroy(void *server);

/* ------------------------------------------------------------------------ */
/* Observability: optional per-kernel timing with HIP events recorded on the */
/* caller's stream around each internal launch.                              */
/* ------------------------------------------------------------------------ */
#define ARA_PROF_OCC      0   /* occurrence-table kernel                     */
#define ARA_PROF_FWD      1   /* forward streaming kernel                    */
#define ARA_PROF_METRICS  2   /* all metric kernels of one ara_metrics call  */
#define ARA_PROF_BWD      3   /* backward streaming kernel                   */
#define ARA_PROF_BWD_RED  4   /* backward reductions                         */
#define ARA_PROF_YELT     5   /* per-occurrence (event-level) kernel         */
#define ARA_PROF_SU       6   /* secondary-uncertainty streaming kernel      */
#define ARA_PROF_KINDS    8

/* on != 0 starts recording every kind (process-wide); 0 stops.  Each
 * recorded launch group adds two event records to its stream, which the
 * device executes as barriers between kernels. */
int32_t ara_profile_enable(int32_t on);
/* Records only the kinds whose bit (1 << kind) is set; 0 stops.  ARA_E_INVAL
 * for bits beyond ARA_PROF_KINDS. */
int32_t ara_profile_enable_kinds(uint32_t mask);
/* Synchronises outstanding events of `kind` and returns their total elapsed
 * milliseconds and launch count since the last reset. */
int32_t ara_profile_read(int32_t kind, double *total_ms, int64_t *launches);
int32_t ara_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* ARA_H */
