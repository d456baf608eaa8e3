/*
 * ara_oracle.c -- plain, slow, obviously-correct CPU reference for aggregate
 * risk analysis (Bahl, Baltzer, Rau-Chaplin, Varghese and Whiteway, "Achieving Speedup
 * in Aggregate Risk Analysis using Multiple GPUs", arXiv 1308.2572).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Precision: IEEE binary64 throughout after the binary32 ELT loss is read
 * (the widening is exact).  Build with -ffp-contract=off so that s*l - R is a
 * separately rounded multiply and subtract.
 *
 * Parity pins (checked by tests/test_oracle_*.py, never by this file):
 *   - hand-worked example derived from Algorithm 1 (tests/golden/)
 *   - closed forms: zero retentions / infinite limits, one-event trials,
 *     AggR = 0 with AggL = inf
 *   - invariants: bounds, monotonicity, permutation invariance, additivity
 *   - brute force on tiny inputs through an independent formulation
 *   - Euler's identity for positively homogeneous metrics (backward)
 *   - central finite differences at certified kink-free points (backward)
 *
 * Readings of points the paper leaves open (all stated again in the design
 * notes):
 *   R1  ApplyFinancialTerms (Section II, step two) is read as
 *       g_k(l) = min(max(s_k*l - R_k, 0), L_k): a per-ELT scale (currency
 *       rate) then a per-ELT retention and limit.
 *   R2  every "min(max(v - R, 0), L)" is evaluated as
 *         y = v - R;  a = (y > 0) ? y : 0;  out = (a < L) ? a : L
 *       and L = +infinity means "no limit".
 *   R3  an event absent from an ELT has loss 0 (direct-access tables,
 *       Section III).
 *   R4  lo and lr start at 0 for every (layer, trial); the differencing step
 *       uses lo_0 := 0 and runs from the last occurrence down to the first.
 *   R5  hits(layer, trial) = number of (occurrence, ELT) pairs whose table
 *       entry is non-zero.
 *   R6  tail metrics: r = N - floor(p*N + 1e-9) clamped to [1, N];
 *       PML_p = r-th largest year loss, TVaR_p = mean of the r largest,
 *       AAL = mean year loss.
 *   R7  subgradients follow the evaluated branch: d out/d v = [y>0 && a<L],
 *       d out/d R = -[y>0 && a<L], d out/d L = [a >= L].
 *   R8  ties at the PML threshold share the weight equally.
 *   R9  the per-occurrence loss (event-level YLT) is the occurrence's
 *       increment of the aggregate-clamped running total, lo_d after the
 *       differencing pass; it sums to the year loss.  The per-year maximum
 *       of these increments is the occurrence loss used for occurrence
 *       exceedance metrics.
 *   R10 secondary uncertainty (named as future work in Section VI, not
 *       defined there): an ELT record carries a standard deviation sigma
 *       beside its mean loss mu, and every (occurrence, ELT) pair draws its
 *       loss from the lognormal distribution with that mean and standard
 *       deviation; sigma = 0 draws mu itself.  The draw replaces the table
 *       lookup of step one; steps two to four are unchanged.
 *   R11 the draw of occurrence i (its index in the YET) in ELT k: the
 *       Philox4x32-10 block (Salmon, Moraes, Dror and Shaw, SC'11) of the
 *       32-bit counter words (i mod 2^32, i div 2^32, k, 0) under key words
 *       (seed mod 2^32, seed div 2^32); output words w0..w3 give
 *       u_1 = (((w1 2^32 + w0) >> 12) + 1/2) 2^-52 and u_2 likewise from
 *       (w3, w2); z = sqrt(-2 ln u_1) cos(2 pi u_2) (Box-Muller),
 *       x = exp(m + s z) with s^2 = ln(1 + sigma^2/mu^2), m = ln mu - s^2/2.
 *       The same occurrence and ELT draw the same loss in every layer.
 *
 * Secondary-uncertainty pins: the generator against the published
 * known-answer vectors of Philox4x32-10, sigma = 0 against the deterministic
 * path bit for bit, and the moments of the draws (mean mu, standard
 * deviation sigma, log-mean m, log-variance s^2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_E_INVAL = 1, OR_E_RANGE = 2, OR_E_DUP = 3, OR_E_NOMEM = 4 };

/* min(max(v - R, 0), L) in the evaluation order of reading R2. */
static double clamp_xl(double v, double R, double L)
{
    double y = v - R;
    double a = (y > 0.0) ? y : 0.0;
    return (a < L) ? a : L;
}

/* ------------------------------------------------------------------------ */
/* Preprocessing stage (Section II; direct-access tables, Section III):      */
/* one dense binary32 array per ELT over the whole catalogue, 0 = absent.     */
/* ------------------------------------------------------------------------ */
int oracle_build_tables(int32_t n_elts, int32_t catalog,
                        const int64_t *rec_off, const int32_t *rec_ids,
                        const float *rec_loss, float *tables)
{
    if (n_elts < 0 || catalog <= 0) return OR_E_INVAL;
    unsigned char *seen = (unsigned char *)malloc((size_t)catalog);
    if (!seen) return OR_E_NOMEM;
    int rc = OR_OK;
    for (int32_t k = 0; k < n_elts && rc == OR_OK; ++k) {
        float *tab = tables + (size_t)k * (size_t)catalog;
        memset(seen, 0, (size_t)catalog);
        for (int32_t e = 0; e < catalog; ++e) tab[e] = 0.0f;
        if (rec_off[k + 1] < rec_off[k]) { rc = OR_E_RANGE; break; }
        for (int64_t i = rec_off[k]; i < rec_off[k + 1]; ++i) {
            int32_t id = rec_ids[i];
            if (id < 0 || id >= catalog) { rc = OR_E_RANGE; break; }
            if (seen[id]) { rc = OR_E_DUP; break; }
            seen[id] = 1;
            tab[id] = rec_loss[i];
        }
    }
    free(seen);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, literally: layer -> trial -> ELT -> occurrence, four steps.   */
/* ------------------------------------------------------------------------ */
/*
 * tables      [n_elts][catalog]  binary32 losses (0 = absent)
 * offsets     [n_trials+1]       CSR over ids; trial t is ids[offsets[t]..offsets[t+1])
 * layer_off   [n_layers+1]       CSR over layer_elts (ELT indices, listed order)
 * elt_terms   [n_elts][3]        {s_k, R_k, L_k}
 * layer_terms [n_layers][4]      {OccR, OccL, AggR, AggL}
 * outputs (each [n_layers][t1-t0], any may be NULL):
 *   ylt   year loss lr of the literal algorithm
 *   s_pre S = last prefix sum of occurrence losses (0 for an empty trial)
 *   hits  reading R5
 *   ylt_closed  f_agg(S), the telescoped closed form of step four's
 *         running-total, clamp and differencing passes
 * per-occurrence outputs (any may be NULL):
 *   yelt    [n_layers][offsets[t1]-offsets[t0]]: the occurrence's share of
 *           the year loss after step four, i.e. lo_d after the differencing
 *           pass (reading R9), in storage order
 *   occ_max [n_layers][t1-t0]: the largest of a trial's yelt values (0 for
 *           an empty trial) -- the per-year maximum occurrence loss behind
 *           occurrence-exceedance metrics
 * n_threads: 1 = strictly sequential; >1 splits trials over OpenMP threads
 * (each trial is computed by the same sequential code, so results are
 * bit-identical to the single-thread run).
 */
int oracle_forward(int32_t n_elts, int32_t catalog, const float *tables,
                   int64_t n_trials, const int64_t *offsets, const int32_t *ids,
                   int32_t n_layers, const int32_t *layer_off, const int32_t *layer_elts,
                   const double *elt_terms, const double *layer_terms,
                   int64_t t0, int64_t t1, int32_t n_threads,
                   double *ylt, double *s_pre, int32_t *hits, double *ylt_closed,
                   double *yelt, double *occ_max)
{
    if (t0 < 0 || t1 < t0 || t1 > n_trials) return OR_E_INVAL;
    int64_t nt = t1 - t0;
    int64_t max_len = 0;
    for (int64_t t = t0; t < t1; ++t) {
        int64_t len = offsets[t + 1] - offsets[t];
        if (len < 0) return OR_E_RANGE;
        if (len > max_len) max_len = len;
    }
    for (int64_t t = t0; t < t1; ++t)
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
            if (ids[i] < 0 || ids[i] >= catalog) return OR_E_RANGE;
    for (int32_t a = 0; a < n_layers; ++a)
        for (int32_t c = layer_off[a]; c < layer_off[a + 1]; ++c)
            if (layer_elts[c] < 0 || layer_elts[c] >= n_elts) return OR_E_RANGE;
    int rc = OR_OK;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel num_threads(n_threads)
#endif
    {
        /* per-thread work arrays: x_d (looked-up loss), l_d (net of
         * financial terms) and lo_d (accumulated occurrence loss) */
        double *x = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        double *l = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        double *lo = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        if (!x || !l || !lo) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            rc = OR_E_NOMEM;
        } else {
            for (int32_t a = 0; a < n_layers; ++a) {               /* for all layers */
                const double OccR = layer_terms[4 * a + 0], OccL = layer_terms[4 * a + 1];
                const double AggR = layer_terms[4 * a + 2], AggL = layer_terms[4 * a + 3];
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
                for (int64_t b = t0; b < t1; ++b) {                 /* for all trials */
                    const int32_t *ev = ids + offsets[b];
                    const int64_t n = offsets[b + 1] - offsets[b];
                    int32_t h = 0;
                    for (int64_t d = 0; d < n; ++d) lo[d] = 0.0;    /* reading R4 */
                    for (int32_t c = layer_off[a]; c < layer_off[a + 1]; ++c) {  /* ELTs */
                        const int32_t k = layer_elts[c];
                        const float *tab = tables + (size_t)k * (size_t)catalog;
                        const double s = elt_terms[3 * k + 0];
                        const double R = elt_terms[3 * k + 1];
                        const double L = elt_terms[3 * k + 2];
                        /* step one: look up each occurrence's loss in this ELT */
                        for (int64_t d = 0; d < n; ++d) {
                            float v = tab[ev[d]];
                            x[d] = (double)v;
                            h += (v != 0.0f);
                        }
                        /* step two: financial terms of this ELT (reading R1) */
                        for (int64_t d = 0; d < n; ++d) {
                            double scaled = s * x[d];
                            l[d] = clamp_xl(scaled, R, L);
                        }
                        /* accumulate across the layer's ELTs */
                        for (int64_t d = 0; d < n; ++d) lo[d] = lo[d] + l[d];
                    }
                    /* step three: occurrence retention and limit */
                    for (int64_t d = 0; d < n; ++d) lo[d] = clamp_xl(lo[d], OccR, OccL);
                    /* cumulative sum over the trial, in occurrence order */
                    for (int64_t d = 1; d < n; ++d) lo[d] = lo[d] + lo[d - 1];
                    const double S = (n > 0) ? lo[n - 1] : 0.0;
                    /* step four: aggregate terms on each running total ... */
                    for (int64_t d = 0; d < n; ++d) lo[d] = clamp_xl(lo[d], AggR, AggL);
                    /* ... back to per-occurrence increments (lo_0 := 0, descending) */
                    for (int64_t d = n - 1; d >= 1; --d) lo[d] = lo[d] - lo[d - 1];
                    /* ... and summed into the year loss */
                    double lr = 0.0;
                    for (int64_t d = 0; d < n; ++d) lr = lr + lo[d];
                    const size_t o = (size_t)a * (size_t)nt + (size_t)(b - t0);
                    if (yelt) {
                        const size_t base = (size_t)a * (size_t)(offsets[t1] - offsets[t0]) +
                                            (size_t)(offsets[b] - offsets[t0]);
                        for (int64_t d = 0; d < n; ++d) yelt[base + (size_t)d] = lo[d];
                    }
                    if (occ_max) {
                        double m = 0.0;
                        for (int64_t d = 0; d < n; ++d) m = (lo[d] > m) ? lo[d] : m;
                        occ_max[o] = m;
                    }
                    if (ylt) ylt[o] = lr;
                    if (s_pre) s_pre[o] = S;
                    if (hits) hits[o] = h;
                    if (ylt_closed) ylt_closed[o] = clamp_xl(S, AggR, AggL);
                }
            }
        }
        free(x); free(l); free(lo);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Portfolio risk metrics from the YLT (named in Section I; reading R6).     */
/* ------------------------------------------------------------------------ */
int64_t oracle_tail_count(int64_t n, double p)
{
    int64_t r = n - (int64_t)floor(p * (double)n + 1e-9);
    if (r < 1) r = 1;
    if (r > n) r = n;
    return r;
}

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* out[3*j + {0,1,2}] = {AAL, PML_p, TVaR_p} for each of n_layers rows of n. */
int oracle_metrics(const double *ylt, int32_t n_layers, int64_t n, double p, double *out)
{
    if (n <= 0 || !(p > 0.0 && p < 1.0)) return OR_E_INVAL;
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!v) return OR_E_NOMEM;
    const int64_t r = oracle_tail_count(n, p);
    for (int32_t j = 0; j < n_layers; ++j) {
        const double *y = ylt + (size_t)j * (size_t)n;
        double sum = 0.0;
        for (int64_t t = 0; t < n; ++t) sum += y[t];
        memcpy(v, y, sizeof(double) * (size_t)n);
        qsort(v, (size_t)n, sizeof(double), cmp_desc);
        double top = 0.0;
        for (int64_t i = 0; i < r; ++i) top += v[i];
        out[3 * j + 0] = sum / (double)n;
        out[3 * j + 1] = v[r - 1];
        out[3 * j + 2] = top / (double)r;
    }
    free(v);
    return OR_OK;
}

/* dMetric/dY for each metric (reading R8): w[m][j][t], m = AAL, PML, TVaR. */
int oracle_metric_weights(const double *ylt, int32_t n_layers, int64_t n, double p, double *w)
{
    if (n <= 0 || !(p > 0.0 && p < 1.0)) return OR_E_INVAL;
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!v) return OR_E_NOMEM;
    const int64_t r = oracle_tail_count(n, p);
    for (int32_t j = 0; j < n_layers; ++j) {
        const double *y = ylt + (size_t)j * (size_t)n;
        memcpy(v, y, sizeof(double) * (size_t)n);
        qsort(v, (size_t)n, sizeof(double), cmp_desc);
        const double thr = v[r - 1];
        int64_t n_gt = 0, n_eq = 0;
        for (int64_t t = 0; t < n; ++t) { n_gt += (y[t] > thr); n_eq += (y[t] == thr); }
        double *wa = w + ((size_t)0 * n_layers + j) * (size_t)n;
        double *wp = w + ((size_t)1 * n_layers + j) * (size_t)n;
        double *wt = w + ((size_t)2 * n_layers + j) * (size_t)n;
        for (int64_t t = 0; t < n; ++t) {
            wa[t] = 1.0 / (double)n;
            wp[t] = (y[t] == thr) ? 1.0 / (double)n_eq : 0.0;
            if (y[t] > thr) wt[t] = 1.0 / (double)r;
            else if (y[t] == thr) wt[t] = (double)(r - n_gt) / ((double)r * (double)n_eq);
            else wt[t] = 0.0;
        }
    }
    free(v);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Reverse sweep of Algorithm 1 (not in the paper; the adjoint of steps one  */
/* to four, walked backwards occurrence by occurrence, reading R7).          */
/* ------------------------------------------------------------------------ */
/*
 * cot        [n_cot][n_layers][t1-t0]  cotangent on each year loss
 * grad_elt   [n_cot][n_elts][3]        d/d{s_k, R_k, L_k}   (overwritten)
 * grad_layer [n_cot][n_layers][4]      d/d{OccR,OccL,AggR,AggL} (overwritten)
 * Sequential (single thread), trial order.
 */
int oracle_backward(int32_t n_elts, int32_t catalog, const float *tables,
                    int64_t n_trials, const int64_t *offsets, const int32_t *ids,
                    int32_t n_layers, const int32_t *layer_off, const int32_t *layer_elts,
                    const double *elt_terms, const double *layer_terms,
                    int64_t t0, int64_t t1, int32_t n_cot, const double *cot,
                    int32_t n_threads, double *grad_elt, double *grad_layer)
{
    if (t0 < 0 || t1 < t0 || t1 > n_trials || n_cot < 0) return OR_E_INVAL;
    const int64_t nt = t1 - t0;
    int64_t max_len = 0;
    for (int64_t t = t0; t < t1; ++t) {
        int64_t len = offsets[t + 1] - offsets[t];
        if (len < 0) return OR_E_RANGE;
        if (len > max_len) max_len = len;
    }
    for (int64_t t = t0; t < t1; ++t)
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
            if (ids[i] < 0 || ids[i] >= catalog) return OR_E_RANGE;
    int32_t max_j = 0;
    for (int32_t a = 0; a < n_layers; ++a) {
        if (layer_off[a + 1] - layer_off[a] > max_j) max_j = layer_off[a + 1] - layer_off[a];
        for (int32_t c = layer_off[a]; c < layer_off[a + 1]; ++c)
            if (layer_elts[c] < 0 || layer_elts[c] >= n_elts) return OR_E_RANGE;
    }
    const size_t n_ge = (size_t)n_cot * (size_t)n_elts * 3, n_gl = (size_t)n_cot * (size_t)n_layers * 4;
    memset(grad_elt, 0, sizeof(double) * n_ge);
    memset(grad_layer, 0, sizeof(double) * n_gl);
    if (n_threads < 1) n_threads = 1;
#ifndef _OPENMP
    n_threads = 1;
#endif
    /* each thread sums its own contiguous share of the trials; the shares are
     * added in thread order afterwards, so a given thread count always gives
     * the same result (one thread: trial order throughout) */
    double *part = (double *)calloc((size_t)n_threads * (n_ge + n_gl), sizeof(double));
    if (!part) return OR_E_NOMEM;
    int rc = OR_OK;
#ifdef _OPENMP
#pragma omp parallel num_threads(n_threads)
#endif
    {
#ifdef _OPENMP
    const int tid = omp_get_thread_num(), nth = omp_get_num_threads();
#else
    const int tid = 0, nth = 1;
#endif
    const int64_t chunk = (nt + nth - 1) / nth;
    const int64_t b0 = t0 + (int64_t)tid * chunk;
    const int64_t b1 = (b0 + chunk < t1) ? b0 + chunk : t1;
    double *my_ge = part + (size_t)tid * (n_ge + n_gl);
    double *my_gl = my_ge + n_ge;
    const size_t m = (size_t)(max_len + 1);
    const size_t mj = (size_t)(max_j > 0 ? max_j : 1);
    double *xk = (double *)malloc(sizeof(double) * m * mj);   /* looked-up losses per ELT */
    double *pre = (double *)malloc(sizeof(double) * m * mj);  /* s*x - R per ELT          */
    double *lsum = (double *)malloc(sizeof(double) * m);      /* lo after step two        */
    double *o = (double *)malloc(sizeof(double) * m);         /* after occurrence terms   */
    double *c = (double *)malloc(sizeof(double) * m);         /* running totals           */
    double *f = (double *)malloc(sizeof(double) * m);         /* after aggregate terms    */
    double *adj_f = (double *)malloc(sizeof(double) * m);
    double *adj_c = (double *)malloc(sizeof(double) * m);
    double *adj_o = (double *)malloc(sizeof(double) * m);
    if (!xk || !pre || !lsum || !o || !c || !f || !adj_f || !adj_c || !adj_o) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
        rc = OR_E_NOMEM;
    } else
    for (int32_t a = 0; a < n_layers; ++a) {
        const double OccR = layer_terms[4 * a + 0], OccL = layer_terms[4 * a + 1];
        const double AggR = layer_terms[4 * a + 2], AggL = layer_terms[4 * a + 3];
        const int32_t J = layer_off[a + 1] - layer_off[a];
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t *ev = ids + offsets[b];
            const int64_t n = offsets[b + 1] - offsets[b];
            /* forward, keeping every intermediate */
            for (int64_t d = 0; d < n; ++d) lsum[d] = 0.0;
            for (int32_t q = 0; q < J; ++q) {
                const int32_t k = layer_elts[layer_off[a] + q];
                const float *tab = tables + (size_t)k * (size_t)catalog;
                const double s = elt_terms[3 * k + 0], R = elt_terms[3 * k + 1], L = elt_terms[3 * k + 2];
                for (int64_t d = 0; d < n; ++d) {
                    double xv = (double)tab[ev[d]];
                    xk[(size_t)q * m + (size_t)d] = xv;
                    double sc = s * xv;
                    pre[(size_t)q * m + (size_t)d] = sc - R;
                    lsum[d] = lsum[d] + clamp_xl(sc, R, L);
                }
            }
            for (int64_t d = 0; d < n; ++d) o[d] = clamp_xl(lsum[d], OccR, OccL);
            for (int64_t d = 0; d < n; ++d) c[d] = (d == 0) ? o[0] : c[d - 1] + o[d];
            for (int64_t d = 0; d < n; ++d) f[d] = clamp_xl(c[d], AggR, AggL);
            for (int32_t g = 0; g < n_cot; ++g) {
                const double w = cot[((size_t)g * n_layers + a) * (size_t)nt + (size_t)(b - t0)];
                double *ge = my_ge + (size_t)g * (size_t)n_elts * 3;
                double *gl = my_gl + ((size_t)g * n_layers + a) * 4;
                if (w == 0.0 || n == 0) continue;
                /* lr = sum_d (f_d - f_{d-1}), f_0 := 0: adjoint of the
                 * summation gives w on every increment; the adjoint of the
                 * differencing moves w onto f_d and -w onto f_{d-1}. */
                for (int64_t d = 0; d < n; ++d) adj_f[d] = 0.0;
                for (int64_t d = 0; d < n; ++d) {
                    adj_f[d] += w;
                    if (d >= 1) adj_f[d - 1] -= w;
                }
                /* aggregate terms on each running total */
                for (int64_t d = 0; d < n; ++d) {
                    double y = c[d] - AggR;
                    double aa = (y > 0.0) ? y : 0.0;
                    int lin = (y > 0.0) && (aa < AggL);
                    adj_c[d] = lin ? adj_f[d] : 0.0;
                    if (lin) gl[2] -= adj_f[d];
                    if (aa >= AggL) gl[3] += adj_f[d];
                }
                /* running total: o_i feeds every c_d with d >= i */
                double run = 0.0;
                for (int64_t d = n - 1; d >= 0; --d) { run += adj_c[d]; adj_o[d] = run; }
                /* occurrence terms, then financial terms per ELT */
                for (int64_t d = 0; d < n; ++d) {
                    double y = lsum[d] - OccR;
                    double aa = (y > 0.0) ? y : 0.0;
                    int lin = (y > 0.0) && (aa < OccL);
                    if (lin) gl[0] -= adj_o[d];
                    if (aa >= OccL) gl[1] += adj_o[d];
                    const double adj_l = lin ? adj_o[d] : 0.0;
                    if (adj_l == 0.0) continue;
                    for (int32_t q = 0; q < J; ++q) {
                        const int32_t k = layer_elts[layer_off[a] + q];
                        const double L = elt_terms[3 * k + 2];
                        const double pv = pre[(size_t)q * m + (size_t)d];
                        const double av = (pv > 0.0) ? pv : 0.0;
                        if ((pv > 0.0) && (av < L)) {
                            ge[3 * k + 0] += adj_l * xk[(size_t)q * m + (size_t)d];
                            ge[3 * k + 1] -= adj_l;
                        }
                        if (av >= L) ge[3 * k + 2] += adj_l;
                    }
                }
            }
        }
    }
    free(xk); free(pre); free(lsum); free(o); free(c); free(f);
    free(adj_f); free(adj_c); free(adj_o);
    }
    for (int th = 0; th < n_threads; ++th) {
        const double *pg = part + (size_t)th * (n_ge + n_gl);
        for (size_t i = 0; i < n_ge; ++i) grad_elt[i] += pg[i];
        for (size_t i = 0; i < n_gl; ++i) grad_layer[i] += pg[n_ge + i];
    }
    free(part);
    return rc;
}

int oracle_num_threads_available(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Secondary uncertainty (readings R10, R11).                                */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10: ten rounds of two 32x32->64-bit multiplies (constants
 * 0xD2511F53 and 0xCD9E8D57) with the key bumped by the Weyl constants
 * 0x9E3779B9 and 0xBB67AE85 between rounds. */
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

int oracle_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    philox4x32_10(ctr, key, out);
    return OR_OK;
}

/* One draw of reading R11. */
double oracle_su_draw(double mu, double sigma, uint64_t seed, int64_t occ, int32_t elt)
{
    if (sigma == 0.0) return mu;
    const uint32_t ctr[4] = {(uint32_t)(uint64_t)occ, (uint32_t)((uint64_t)occ >> 32), (uint32_t)elt, 0};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    const uint64_t b1 = ((uint64_t)w[1] << 32) | w[0], b2 = ((uint64_t)w[3] << 32) | w[2];
    const double u1 = ((double)(b1 >> 12) + 0.5) * 0x1p-52;
    const double u2 = ((double)(b2 >> 12) + 0.5) * 0x1p-52;
    const double two_pi = 6.283185307179586476925286766559; /* the binary64 nearest 2 pi */
    const double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    const double r = sigma / mu;
    const double s2 = log1p(r * r);
    const double m = log(mu) - 0.5 * s2;
    return exp(m + sqrt(s2) * z);
}

/*
 * Algorithm 1 with secondary uncertainty: as oracle_forward (steps two to
 * four literally), the lookup of step one replaced by the draw of R10/R11.
 * sigma_tables: dense binary64-widened-from-binary32 standard deviations
 * laid out like `tables`.  Outputs ylt and s_pre [n_layers][t1-t0] (either
 * may be NULL).
 */
int oracle_forward_su(int32_t n_elts, int32_t catalog, const float *tables, const float *sigma_tables,
                      int64_t n_trials, const int64_t *offsets, const int32_t *ids,
                      int32_t n_layers, const int32_t *layer_off, const int32_t *layer_elts,
                      const double *elt_terms, const double *layer_terms, uint64_t seed,
                      int64_t t0, int64_t t1, int32_t n_threads, double *ylt, double *s_pre)
{
    if (t0 < 0 || t1 < t0 || t1 > n_trials) return OR_E_INVAL;
    const int64_t nt = t1 - t0;
    int64_t max_len = 0;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t len = offsets[t + 1] - offsets[t];
        if (len < 0) return OR_E_RANGE;
        if (len > max_len) max_len = len;
    }
    for (int64_t t = t0; t < t1; ++t)
        for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
            if (ids[i] < 0 || ids[i] >= catalog) return OR_E_RANGE;
    for (int32_t a = 0; a < n_layers; ++a)
        for (int32_t c = layer_off[a]; c < layer_off[a + 1]; ++c)
            if (layer_elts[c] < 0 || layer_elts[c] >= n_elts) return OR_E_RANGE;
    int rc = OR_OK;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel num_threads(n_threads)
#endif
    {
        double *net = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        double *occ = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        if (!net || !occ) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            rc = OR_E_NOMEM;
        } else {
            for (int32_t a = 0; a < n_layers; ++a) {
                const double OccR = layer_terms[4 * a + 0], OccL = layer_terms[4 * a + 1];
                const double AggR = layer_terms[4 * a + 2], AggL = layer_terms[4 * a + 3];
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
                for (int64_t b = t0; b < t1; ++b) {
                    const int32_t *ev = ids + offsets[b];
                    const int64_t n = offsets[b + 1] - offsets[b];
                    for (int64_t d = 0; d < n; ++d) occ[d] = 0.0;
                    for (int32_t c = layer_off[a]; c < layer_off[a + 1]; ++c) {
                        const int32_t k = layer_elts[c];
                        const float *tab = tables + (size_t)k * (size_t)catalog;
                        const float *sig = sigma_tables + (size_t)k * (size_t)catalog;
                        const double s = elt_terms[3 * k + 0];
                        const double R = elt_terms[3 * k + 1];
                        const double L = elt_terms[3 * k + 2];
                        /* step one, with secondary uncertainty: a draw per
                         * occurrence of an event the ELT holds (R10) */
                        for (int64_t d = 0; d < n; ++d) {
                            const double mu = (double)tab[ev[d]];
                            const double x = (mu != 0.0)
                                ? oracle_su_draw(mu, (double)sig[ev[d]], seed, offsets[b] + d, k) : 0.0;
                            /* step two */
                            net[d] = clamp_xl(s * x, R, L);
                        }
                        for (int64_t d = 0; d < n; ++d) occ[d] = occ[d] + net[d];
                    }
                    /* step three */
                    for (int64_t d = 0; d < n; ++d) occ[d] = clamp_xl(occ[d], OccR, OccL);
                    /* step four: running totals, aggregate terms, increments, sum */
                    for (int64_t d = 1; d < n; ++d) occ[d] = occ[d] + occ[d - 1];
                    const double S = (n > 0) ? occ[n - 1] : 0.0;
                    for (int64_t d = 0; d < n; ++d) occ[d] = clamp_xl(occ[d], AggR, AggL);
                    for (int64_t d = n - 1; d >= 1; --d) occ[d] = occ[d] - occ[d - 1];
                    double lr = 0.0;
                    for (int64_t d = 0; d < n; ++d) lr = lr + occ[d];
                    const size_t o = (size_t)a * (size_t)nt + (size_t)(b - t0);
                    if (ylt) ylt[o] = lr;
                    if (s_pre) s_pre[o] = S;
                }
            }
        }
        free(net);
        free(occ);
    }
    return rc;
}

