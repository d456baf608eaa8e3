"""Central differences of the HIP forward against the HIP backward, for
every term of a layer: the 15 scales, 15 retentions and 15 limits of its
ELTs and its four layer terms (49 in all), for AAL, PML and TVaR.

The year loss is piecewise affine in each term: with every branch of every
clamp fixed, each step of Algorithm 1 is affine in the inputs.  So at a
point where no branch changes within the step, the central difference of a
metric equals its derivative up to rounding.  The point is certified on the
CPU before any GPU work: for each of the 98 perturbed term sets the oracle
recomputes every trial total and, through one-event trials, every event's
sum over the layer's ELTs; every branch (each ELT record's retention and
limit, each event's occurrence retention and limit, each trial's aggregate
retention and limit) must be the same at both ends of the step as at the
point, and so must the trials the metrics select (the PML's trial and the
set of the r largest).  Affine quantities that keep one side of a kink at
both ends keep it in between, so the metrics are affine over the step.

Tolerance: |FD - gradient| <= 1e-6 * |gradient| + 1e-12 * M / |theta| per
entry (M the metric), the rounding of the two forwards divided by the step.
"""
import numpy as np
import pytest

import oracle
import synth

H = 1e-6                 # relative step
SEED = 1308257203        # the differentiated workload's seed
N_TRIALS, N_EVENTS, CATALOG, ELT_SIZE, P = 4000, 250, 50_000, 500, 0.99


def fd_workload(seed=SEED):
    """The differentiated workload at a reduced size with its density of
    hits (15 ELTs x 500 events over 50,000: 0.15 per event): 4000 trials x
    250 events, terms perturbed by U[0.97, 1.03] as in the full workload,
    and an aggregate limit that caps about 0.5% of the trials (fewer than
    the r = 40 largest, so the PML's trial is not capped)."""
    g = np.random.default_rng(seed)
    yet = synth.fixed_length_yet(seed, N_TRIALS, N_EVENTS, CATALOG)
    elts = synth.lognormal_elts(seed, [ELT_SIZE] * 15, CATALOG)
    elts.terms = elts.terms.copy()
    elts.terms[:, 1] *= g.uniform(0.97, 1.03, size=15)
    elts.terms[:, 2] *= g.uniform(0.97, 1.03, size=15)
    lt = synth.CONFIG_TERMS_LAYER * g.uniform(0.97, 1.03, size=4)
    lt[3] = np.inf
    layers = synth.Layers(np.array([0, 15], np.int32), np.arange(15, dtype=np.int32), lt[None, :].copy())
    w = synth.Workload("fd-4000x250-15elt", yet, elts, layers, P)
    tb = oracle.build_tables(elts)
    s = oracle.forward(tb, yet, layers, elts.terms, layers.terms)["s_pre"][0]
    layers.terms[0, 3] = float(np.quantile(s, 0.995)) - lt[2] + 0.5
    return w


def all_terms(w):
    """(table, row, column) of every finite, non-zero term."""
    out = [("elt", k, c) for k in range(w.elts.n_elts) for c in range(3)]
    out += [("layer", 0, c) for c in range(4)]
    return out


def perturbed(w, which, sign):
    et, lt = w.elts.terms.copy(), w.layers.terms.copy()
    tab, k, c = which
    a = et if tab == "elt" else lt
    d = H * abs(a[k, c])
    a[k, c] += sign * d
    return et, lt, d


def _branches(w, tb, et, lt):
    """Every clamp branch of the point (et, lt) and the trials its metrics
    select, as comparable arrays."""
    j = 0
    occr, occl, aggr, aggl = lt[j]
    # ELT records: s*l - R against 0 and L (the records of events in the YET)
    present = np.zeros(w.elts.catalog, bool)
    present[w.yet.ids] = True
    rec = []
    for k in range(w.elts.n_elts):
        a, b = int(w.elts.rec_off[k]), int(w.elts.rec_off[k + 1])
        ids = w.elts.rec_ids[a:b]
        l = w.elts.rec_loss[a:b].astype(np.float64)[present[ids]]
        pre = et[k, 0] * l - et[k, 1]
        rec.append(pre > 0)
        rec.append(np.where(pre > 0, pre, 0.0) < et[k, 2])
    # each event's sum over the layer's ELTs, from one-event trials through
    # the oracle with the occurrence and aggregate terms switched off
    ev = np.flatnonzero(present).astype(np.int32)
    one = synth.Yet(w.elts.catalog, np.arange(ev.shape[0] + 1, dtype=np.int64), ev)
    free = np.array([[0.0, np.inf, 0.0, np.inf]])
    x = oracle.forward(tb, one, w.layers, et, free, n_threads=8)["s_pre"][0]
    y = x - occr
    occ = [y > 0, np.where(y > 0, y, 0.0) < occl]
    r = oracle.forward(tb, w.yet, w.layers, et, lt[None, 0] if lt.ndim == 1 else lt, n_threads=8)
    S, Y = r["s_pre"][0], r["ylt"][0]
    z = S - aggr
    agg = [z > 0, np.where(z > 0, z, 0.0) < aggl]
    n = Y.shape[0]
    rr = oracle.tail_count(n, w.p)
    order = np.argsort(-Y, kind="stable")
    t_pml = int(order[rr - 1])
    top = np.zeros(n, bool)
    top[order[:rr]] = True
    above = Y > Y[t_pml]
    unique = np.count_nonzero(Y == Y[t_pml]) == 1
    return rec + occ + agg + [top, above], t_pml, unique


def certify(w):
    """True when every branch and the metrics' selected trials are the same
    at both ends of every step as at the point; otherwise the first term
    that moves one, as a string."""
    tb = oracle.build_tables(w.elts)
    base, t0, uniq = _branches(w, tb, w.elts.terms, w.layers.terms)
    if not uniq:
        return "the PML is tied"
    for which in all_terms(w):
        for sign in (+1, -1):
            et, lt, _ = perturbed(w, which, sign)
            br, t1, u1 = _branches(w, tb, et, lt)
            if t1 != t0 or not u1 or any(not np.array_equal(a, b) for a, b in zip(base, br)):
                return f"{which} {sign:+d}"
    return True


def test_fd_point_is_certified():
    """The reduced differentiated workload is a point where no branch and no
    selected trial changes within the step (CPU only)."""
    assert certify(fd_workload()) is True


@pytest.mark.gpu
def test_central_differences_every_term():
    import torch
    import paper_1308_2572_amd as ara
    ara.library()
    w = fd_workload()
    print("[gpu-fd] certifying the point", flush=True)
    assert certify(w) is True
    tables = ara.EltTables.from_numpy(w.elts)
    yet = ara.PreparedYet.from_numpy(w.yet)
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")

    def metric(et, lt):
        y, _, _ = ara.ylt_forward(tables, yet, layers, dev(et), dev(lt), check=True)
        return ara.metrics(y, w.p)[0].cpu().numpy()[0]

    et0, lt0 = dev(w.elts.terms), dev(w.layers.terms)
    y, s_pre, _ = ara.ylt_forward(tables, yet, layers, et0, lt0, want_s_pre=True, check=True)
    m0, wts = ara.metrics(y, w.p, want_weights=True)
    m0 = m0.cpu().numpy()[0]
    ge, gl = ara.ylt_backward(tables, yet, layers, et0, lt0, s_pre, wts)
    ge, gl = ge.cpu().numpy(), gl.cpu().numpy()
    print("[gpu-fd] 98 forwards", flush=True)
    worst = 0.0
    nonzero = 0
    for which in all_terms(w):
        tab, k, c = which
        ep, lp, d = perturbed(w, which, +1)
        em, lm, _ = perturbed(w, which, -1)
        fd = (metric(ep, lp) - metric(em, lm)) / (2 * d)
        g = ge[:, k, c] if tab == "elt" else gl[:, 0, c]
        theta = abs((w.elts.terms if tab == "elt" else w.layers.terms)[k, c])
        for m in range(3):
            bound = 1e-6 * abs(g[m]) + 1e-12 * abs(m0[m]) / theta
            err = abs(fd[m] - g[m])
            assert err <= bound, (which, ["AAL", "PML", "TVaR"][m], fd[m], g[m])
            worst = max(worst, err / max(abs(g[m]), 1e-300))
            nonzero += g[m] != 0.0
    print(f"[gpu-fd] 147 entries, {nonzero} non-zero, worst relative deviation {worst:.2e}", flush=True)
    assert nonzero >= 100
