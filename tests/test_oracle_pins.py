"""Pins of the CPU oracle against facts fixed by the paper's definitions and by
mathematics: a hand-derived example, closed forms, invariants, brute force
through an independent formulation, counting definitions of the metrics,
Euler's identity and finite differences for the reverse sweep."""
import math

import numpy as np
import pytest

import oracle
import synth
from _indep import brute_forward, brute_metrics, brute_yelt, load_hand_example, xl

U = 2.0 ** -53


def run(w, elt_terms=None, layer_terms=None, **kw):
    tb = oracle.build_tables(w.elts)
    et = w.elts.terms if elt_terms is None else elt_terms
    lt = w.layers.terms if layer_terms is None else layer_terms
    return tb, oracle.forward(tb, w.yet, w.layers, et, lt, **kw)


# ---------------------------------------------------------------- golden
def test_hand_example_forward_and_metrics():
    w, g = load_hand_example()
    _, r = run(w)
    assert r["ylt"][0].tolist() == g["ylt"]
    assert r["s_pre"][0].tolist() == g["s_pre"]
    assert r["hits"][0].tolist() == g["hits"]
    for p, m in g["metrics"].items():
        p = float(p)
        assert oracle.tail_count(5, p) == m["r"]
        got = oracle.metrics(r["ylt"], p)[0]
        assert got.tolist() == [m["aal"], m["pml"], m["tvar"]]


def test_hand_example_gradients():
    w, g = load_hand_example()
    tb, r = run(w)
    wts = oracle.metric_weights(r["ylt"], g["grad_p"])
    ge, gl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, wts)
    for i, name in enumerate(["aal", "pml", "tvar"]):
        np.testing.assert_allclose(ge[i], np.array(g["grad"][name]["elt"]), rtol=0, atol=1e-12)
        np.testing.assert_allclose(gl[i, 0], np.array(g["grad"][name]["layer"]), rtol=0, atol=1e-12)


def test_tail_count_definition():
    assert oracle.tail_count(1_000_000, 0.99) == 10_000
    assert oracle.tail_count(10_000, 0.99) == 100
    assert oracle.tail_count(5, 0.6) == 2
    assert oracle.tail_count(10, 0.05) == 10
    assert oracle.tail_count(7, 0.999) == 1


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(6))
def test_closed_form_no_terms_is_scaled_loss_sum(seed):
    """All retentions 0 and all limits infinite: the year loss is the sum over
    occurrences and ELTs of the scaled looked-up losses."""
    w = synth.tiny_random(seed, zero_terms=True, n_trials=30)
    tb, r = run(w)
    for j in range(w.layers.n_layers):
        lst = w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]]
        per_event = np.zeros(w.elts.catalog)
        for k in lst:
            dense = np.zeros(w.elts.catalog)
            a, b = w.elts.rec_off[k], w.elts.rec_off[k + 1]
            dense[w.elts.rec_ids[a:b]] = w.elts.rec_loss[a:b].astype(np.float64)
            per_event += w.elts.terms[k, 0] * dense
        contrib = per_event[w.yet.ids]
        expect = np.add.reduceat(np.append(contrib, 0.0), w.yet.offsets[:-1]) * (np.diff(w.yet.offsets) > 0)
        np.testing.assert_allclose(r["ylt"][j], expect, rtol=1e-12, atol=0)
        np.testing.assert_allclose(r["s_pre"][j], expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_closed_form_one_event_trials(seed):
    """A one-occurrence trial reduces to nested min/max of the three levels."""
    w = synth.tiny_random(seed, n_trials=40, max_events=1)
    _, r = run(w)
    dicts = [dict(zip(w.elts.rec_ids[w.elts.rec_off[k]:w.elts.rec_off[k + 1]].tolist(),
                      w.elts.rec_loss[w.elts.rec_off[k]:w.elts.rec_off[k + 1]].tolist()))
             for k in range(w.elts.n_elts)]
    for j in range(w.layers.n_layers):
        lst = w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]].tolist()
        occr, occl, aggr, aggl = w.layers.terms[j]
        for t in range(w.yet.n_trials):
            ev = w.yet.ids[w.yet.offsets[t]:w.yet.offsets[t + 1]].tolist()
            if not ev:
                assert r["ylt"][j, t] == 0.0
                continue
            x = sum(xl(w.elts.terms[k, 0] * dicts[k].get(ev[0], 0.0), w.elts.terms[k, 1], w.elts.terms[k, 2])
                    for k in lst)
            expect = min(max(min(max(x - occr, 0.0), occl) - aggr, 0.0), aggl)
            assert r["ylt"][j, t] == pytest.approx(expect, rel=1e-13, abs=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_closed_form_no_aggregate_terms(seed):
    """AggR = 0 and AggL = inf: the year loss is the plain sum of occurrence losses."""
    w = synth.tiny_random(seed, n_trials=30)
    lt = w.layers.terms.copy()
    lt[:, 2] = 0.0
    lt[:, 3] = np.inf
    _, r = run(w, layer_terms=lt)
    Y, S, _ = brute_forward(w, layer_terms=lt)
    np.testing.assert_allclose(r["ylt"], S, rtol=1e-13, atol=0)
    np.testing.assert_allclose(r["ylt"], r["s_pre"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", range(8))
def test_literal_cumulative_steps_telescope(seed):
    """The cumulative-sum / aggregate-clamp / difference / sum steps equal the
    aggregate clamp of the final running total, within rounding."""
    w = synth.tiny_random(seed, n_trials=40, max_events=30)
    _, r = run(w)
    n = np.diff(w.yet.offsets)[None, :]
    bound = 4 * np.maximum(n, 1) * U * np.maximum(r["s_pre"], 1.0)
    assert np.all(np.abs(r["ylt"] - r["ylt_closed"]) <= bound)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(10))
def test_bruteforce_dict_formulation(seed):
    w = synth.tiny_random(seed, n_trials=25, n_layers=3)
    _, r = run(w)
    Y, S, H = brute_forward(w)
    assert np.array_equal(r["hits"], H)
    tol = 1e-12 * np.maximum(np.abs(Y), S) + 1e-300
    assert np.all(np.abs(r["ylt"] - Y) <= tol)
    assert np.all(np.abs(r["s_pre"] - S) <= 1e-12 * S + 1e-300)


def test_config0_prefix_matches_bruteforce():
    w = synth.config(0, n_trials=30)
    _, r = run(w)
    Y, S, H = brute_forward(w)
    assert np.array_equal(r["hits"], H)
    np.testing.assert_allclose(r["s_pre"], S, rtol=1e-12)
    np.testing.assert_allclose(r["ylt"], Y, rtol=1e-12)


def test_openmp_split_is_bit_identical():
    w = synth.tiny_random(3, n_trials=200, max_events=40)
    tb = oracle.build_tables(w.elts)
    a = oracle.forward(tb, w.yet, w.layers, w.elts.terms, n_threads=1)
    b = oracle.forward(tb, w.yet, w.layers, w.elts.terms, n_threads=4)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_trial_subrange_matches_full():
    w = synth.tiny_random(5, n_trials=50)
    tb = oracle.build_tables(w.elts)
    full = oracle.forward(tb, w.yet, w.layers, w.elts.terms)
    part = oracle.forward(tb, w.yet, w.layers, w.elts.terms, t0=7, t1=31)
    for k in full:
        assert np.array_equal(full[k][:, 7:31], part[k])


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(6))
def test_bounds(seed):
    w = synth.tiny_random(seed, n_trials=40, max_events=25)
    _, r = run(w)
    aggl = w.layers.terms[:, 3][:, None]
    assert np.all(r["ylt"] >= 0.0)
    assert np.all(r["ylt"] <= aggl)
    assert np.all(r["ylt"] <= r["s_pre"])
    empty = np.diff(w.yet.offsets) == 0
    assert np.all(r["ylt"][:, empty] == 0.0) and np.all(r["hits"][:, empty] == 0)


@pytest.mark.parametrize("seed", range(4))
def test_monotone_in_losses_scales_limits_and_retentions(seed):
    w = synth.tiny_random(seed, n_trials=40, max_events=20)
    _, base = run(w)
    y0 = base["ylt"]
    # raise every loss by 10%
    w2 = synth.tiny_random(seed, n_trials=40, max_events=20)
    w2.elts.rec_loss = (w2.elts.rec_loss * np.float32(1.1)).astype(np.float32)
    _, r = run(w2)
    assert np.all(r["ylt"] >= y0)
    for col, sign in [(0, +1), (2, +1), (1, -1)]:     # scale up, limit up, retention up
        et = w.elts.terms.copy()
        et[:, col] *= 1.2
        _, r = run(w, elt_terms=et)
        assert np.all(sign * (r["ylt"] - y0) >= 0.0)
    for col, sign in [(1, +1), (3, +1), (0, -1), (2, -1)]:
        lt = w.layers.terms.copy()
        lt[:, col] *= 1.2
        _, r = run(w, layer_terms=lt)
        assert np.all(sign * (r["ylt"] - y0) >= 0.0)


@pytest.mark.parametrize("seed", range(4))
def test_permutation_invariance(seed):
    """Event order inside a trial and ELT order inside a layer change the year
    loss only by rounding (telescoping of the aggregate steps)."""
    w = synth.tiny_random(seed, n_trials=40, max_events=25)
    _, r0 = run(w)
    g = np.random.default_rng(seed)
    ids = w.yet.ids.copy()
    for t in range(w.yet.n_trials):
        a, b = w.yet.offsets[t], w.yet.offsets[t + 1]
        ids[a:b] = g.permutation(ids[a:b])
    w.yet.ids = ids
    lst = w.layers.elt_ids.copy()
    for j in range(w.layers.n_layers):
        a, b = w.layers.elt_off[j], w.layers.elt_off[j + 1]
        lst[a:b] = lst[a:b][::-1]
    w.layers.elt_ids = lst
    _, r1 = run(w)
    tol = 1e-12 * np.maximum(r0["ylt"], r0["s_pre"]) + 1e-300
    assert np.all(np.abs(r0["ylt"] - r1["ylt"]) <= tol)
    assert np.array_equal(r0["hits"], r1["hits"])


def test_concatenation_is_additive_without_aggregate_terms():
    w = synth.tiny_random(11, n_trials=20, max_events=10)
    lt = w.layers.terms.copy()
    lt[:, 2], lt[:, 3] = 0.0, np.inf
    _, r = run(w, layer_terms=lt)
    # build trials that are pairwise concatenations (t, t+1)
    off, ids = w.yet.offsets, w.yet.ids
    new_ids, new_off = [], [0]
    for t in range(0, w.yet.n_trials - 1, 2):
        seg = np.concatenate([ids[off[t]:off[t + 1]], ids[off[t + 1]:off[t + 2]]])
        new_ids.append(seg)
        new_off.append(new_off[-1] + len(seg))
    w.yet = synth.Yet(w.yet.catalog, np.array(new_off, np.int64), np.concatenate(new_ids).astype(np.int32))
    _, rc = run(w, layer_terms=lt)
    expect = r["ylt"][:, 0::2][:, :rc["ylt"].shape[1]] + r["ylt"][:, 1::2][:, :rc["ylt"].shape[1]]
    np.testing.assert_allclose(rc["ylt"], expect, rtol=1e-13)


def test_input_validation_codes():
    w = synth.tiny_random(1)
    bad = synth.Elts(w.elts.catalog, w.elts.rec_off.copy(), w.elts.rec_ids.copy(), w.elts.rec_loss, w.elts.terms)
    bad.rec_ids[1] = bad.rec_ids[0] if bad.rec_off[1] > 1 else bad.rec_ids[0]
    if bad.rec_off[1] > 1:
        with pytest.raises(oracle.OracleError):
            oracle.build_tables(bad)
    bad.rec_ids[0] = w.elts.catalog
    with pytest.raises(oracle.OracleError):
        oracle.build_tables(bad)


# ---------------------------------------------------------------- metrics
@pytest.mark.parametrize("seed", range(8))
def test_metrics_counting_definition(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 60))
    y = np.round(g.exponential(100.0, size=n), 0 if seed % 2 else 6)   # ties when rounded
    for p in [0.5, 0.8, 0.9, 0.99, 0.01]:
        aal, pml, tvar, r = brute_metrics(y, p)
        got = oracle.metrics(y[None, :], p)[0]
        assert got[1] == pml
        assert got[0] == pytest.approx(aal, rel=1e-14)
        assert got[2] == pytest.approx(tvar, rel=1e-14)
        assert got[1] <= got[2] * (1 + 1e-15) <= y.max() * (1 + 1e-14)
        assert got[0] <= got[2] * (1 + 1e-14)


def test_metrics_special_cases():
    y = np.full((1, 37), 12.5)
    assert oracle.metrics(y, 0.99)[0].tolist() == [12.5, 12.5, 12.5]
    y = np.arange(10, dtype=np.float64)[None, :]
    m = oracle.metrics(y, 0.05)[0]          # r = n: TVaR is the mean
    assert m[2] == pytest.approx(m[0], rel=1e-15)
    assert m[1] == 0.0


# ---------------------------------------------------------------- reverse sweep
def _all_terms(w):
    return w.elts.terms.copy(), w.layers.terms.copy()


def _metric_vec(w, et, lt, p):
    tb = oracle.build_tables(w.elts)
    r = oracle.forward(tb, w.yet, w.layers, et, lt)
    return oracle.metrics(r["ylt"], p), r


@pytest.mark.parametrize("seed", range(6))
def test_euler_identity(seed):
    """Every metric is positively homogeneous of degree one in (scales, all
    retentions, all limits): sum theta * dM/dtheta = M over finite terms."""
    w = synth.tiny_random(seed, n_trials=60, max_events=20)
    et, lt = _all_terms(w)
    m, r = _metric_vec(w, et, lt, w.p)
    tb = oracle.build_tables(w.elts)
    wts = oracle.metric_weights(r["ylt"], w.p)
    ge, gl = oracle.backward(tb, w.yet, w.layers, et, lt, wts)
    for c in range(3):
        for j in range(w.layers.n_layers):
            used = w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]]
            # layer-j-only gradient via a cotangent restricted to layer j
            cot = np.zeros_like(wts[c:c + 1])
            cot[0, j] = wts[c, j]
            gej, glj = oracle.backward(tb, w.yet, w.layers, et, lt, cot)
            total = 0.0
            for k in used:
                for col in range(3):
                    if np.isfinite(et[k, col]):
                        total += et[k, col] * gej[0, k, col]
            for col in range(4):
                if np.isfinite(lt[j, col]):
                    total += lt[j, col] * glj[0, j, col]
            assert total == pytest.approx(m[j, c], rel=1e-10, abs=1e-9)
        assert np.allclose(ge[c], sum(oracle.backward(tb, w.yet, w.layers, et, lt,
                                                      _only(wts[c], j))[0][0] for j in range(w.layers.n_layers)))


def _only(wc, j):
    cot = np.zeros((1,) + wc.shape)
    cot[0, j] = wc[j]
    return cot


def _kink_margin(w, et, lt):
    """Smallest relative distance of any pre-clamp quantity from its kink."""
    dicts = [dict(zip(w.elts.rec_ids[w.elts.rec_off[k]:w.elts.rec_off[k + 1]].tolist(),
                      w.elts.rec_loss[w.elts.rec_off[k]:w.elts.rec_off[k + 1]].tolist()))
             for k in range(w.elts.n_elts)]
    margin = np.inf
    for j in range(w.layers.n_layers):
        lst = w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]].tolist()
        occr, occl, aggr, aggl = lt[j]
        for t in range(w.yet.n_trials):
            s = 0.0
            for e in w.yet.ids[w.yet.offsets[t]:w.yet.offsets[t + 1]].tolist():
                x = 0.0
                for k in lst:
                    l = dicts[k].get(e, 0.0)
                    if l != 0.0:
                        pre = et[k, 0] * l - et[k, 1]
                        margin = min(margin, abs(pre) / (abs(et[k, 0] * l) + 1), abs(pre - et[k, 2]) / (et[k, 2] + 1))
                    x += xl(et[k, 0] * l, et[k, 1], et[k, 2])
                if x != 0.0:
                    margin = min(margin, abs(x - occr) / (x + 1), abs(x - occr - occl) / (occl + 1))
                s += xl(x, occr, occl)
            if s != 0.0:
                margin = min(margin, abs(s - aggr) / (s + 1), abs(s - aggr - aggl) / (aggl + 1))
    return margin


@pytest.mark.parametrize("seed", range(5))
def test_reverse_sweep_matches_central_differences(seed):
    w = synth.tiny_random(seed + 20, n_trials=30, max_events=10, n_layers=1)
    et, lt = _all_terms(w)
    h = 1e-6
    margin = _kink_margin(w, et, lt)
    if margin < 50 * h:
        pytest.skip(f"seed {seed}: a kink lies within the difference step (margin {margin:.2e})")
    m0, r = _metric_vec(w, et, lt, w.p)
    tb = oracle.build_tables(w.elts)
    wts = oracle.metric_weights(r["ylt"], w.p)
    ge, gl = oracle.backward(tb, w.yet, w.layers, et, lt, wts)
    # the PML/TVaR order statistics must not change within the step
    for k in range(w.elts.n_elts):
        for col in range(3):
            if not np.isfinite(et[k, col]) or et[k, col] == 0.0:
                continue
            d = h * abs(et[k, col])
            ep, em = et.copy(), et.copy()
            ep[k, col] += d
            em[k, col] -= d
            fd = (_metric_vec(w, ep, lt, w.p)[0] - _metric_vec(w, em, lt, w.p)[0])[0] / (2 * d)
            np.testing.assert_allclose(ge[:, k, col], fd, rtol=1e-5, atol=1e-6 * (1 + abs(m0).max()))
    for col in range(4):
        if not np.isfinite(lt[0, col]) or lt[0, col] == 0.0:
            continue
        d = h * abs(lt[0, col])
        lp, lm = lt.copy(), lt.copy()
        lp[0, col] += d
        lm[0, col] -= d
        fd = (_metric_vec(w, et, lp, w.p)[0] - _metric_vec(w, et, lm, w.p)[0])[0] / (2 * d)
        np.testing.assert_allclose(gl[:, 0, col], fd, rtol=1e-5, atol=1e-6 * (1 + abs(m0).max()))


def test_aggregate_term_gradients_are_counts():
    """dAAL/dAggR = -#{trials between the kinks}/N and dAAL/dAggL = #{capped}/N."""
    w = synth.tiny_random(7, n_trials=80, max_events=20)
    tb = oracle.build_tables(w.elts)
    r = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms)
    wts = oracle.metric_weights(r["ylt"], w.p)
    _, gl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, wts)
    n = w.yet.n_trials
    for j in range(w.layers.n_layers):
        aggr, aggl = w.layers.terms[j, 2], w.layers.terms[j, 3]
        z = r["s_pre"][j] - aggr
        a = np.where(z > 0, z, 0.0)
        lin = np.count_nonzero((z > 0) & (a < aggl))
        cap = np.count_nonzero(a >= aggl)
        assert gl[0, j, 2] == pytest.approx(-lin / n, rel=1e-12, abs=1e-15)
        assert gl[0, j, 3] == pytest.approx(cap / n, rel=1e-12, abs=1e-15)


# ------------------------------------------------- per-occurrence losses
def test_hand_example_yelt():
    w, g = load_hand_example()
    _, r = run(w, want_yelt=True)
    flat = [v for t in g["yelt"] for v in t]
    assert r["yelt"][0].tolist() == flat
    assert r["occ_max"][0].tolist() == g["occ_max"]


@pytest.mark.parametrize("seed", range(8))
def test_yelt_sums_to_year_loss_and_bounds(seed):
    w = synth.tiny_random(seed, n_trials=40, max_events=30, n_layers=2)
    _, r = run(w, want_yelt=True)
    off = w.yet.offsets
    for j in range(w.layers.n_layers):
        aggl = w.layers.terms[j, 3]
        y = r["yelt"][j]
        assert np.all(y >= 0.0) and np.all(y <= aggl)
        for t in range(w.yet.n_trials):
            seg = y[off[t]:off[t + 1]]
            n = len(seg)
            S = r["s_pre"][j, t]
            assert abs(math.fsum(seg) - r["ylt"][j, t]) <= 4 * max(n, 1) * U * S
            assert r["occ_max"][j, t] == (seg.max() if n else 0.0)
            assert r["occ_max"][j, t] <= r["ylt"][j, t] or n == 0


@pytest.mark.parametrize("seed", range(8))
def test_yelt_bruteforce_running_totals(seed):
    w = synth.tiny_random(seed, n_trials=30, max_events=25, n_layers=2)
    _, r = run(w, want_yelt=True)
    ref, mx = brute_yelt(w)
    off = w.yet.offsets
    for j in range(w.layers.n_layers):
        for t in range(w.yet.n_trials):
            a, b = off[t], off[t + 1]
            S = r["s_pre"][j, t]
            tol = 4 * max(b - a, 1) * U * S
            assert np.all(np.abs(r["yelt"][j][a:b] - ref[j][a:b]) <= tol)
            assert abs(r["occ_max"][j, t] - mx[j, t]) <= tol


def test_yelt_zero_before_retention_and_after_limit():
    """An occurrence whose running total stays at or below AggR, or which
    comes after the running total has used up AggL, adds exactly 0."""
    w = synth.tiny_random(5, n_trials=50, max_events=40, n_layers=1)
    lt = w.layers.terms.copy()
    _, r0 = run(w, layer_terms=lt)
    S = r0["s_pre"][0]
    lt[0, 2] = float(np.median(S[S > 0])) * 0.3
    lt[0, 3] = float(np.median(S[S > 0])) * 0.4
    _, r = run(w, layer_terms=lt, want_yelt=True)
    off = w.yet.offsets
    dicts = None
    for t in range(w.yet.n_trials):
        seg = r["yelt"][0][off[t]:off[t + 1]]
        if len(seg) == 0:
            continue
        # running totals of the increments identify the phases
        run_c = np.cumsum(seg)
        capped = np.nonzero(run_c >= lt[0, 3])[0]
        if len(capped):
            assert np.all(seg[capped[0] + 1:] == 0.0)
        assert r["occ_max"][0, t] <= lt[0, 3]


def test_yelt_without_aggregate_terms_is_occurrence_loss():
    """AggR = 0 and AggL = inf: each increment is the occurrence loss o_d up to
    the rounding of the running total."""
    w = synth.tiny_random(3, n_trials=30, max_events=20, n_layers=1)
    lt = w.layers.terms.copy()
    lt[0, 2], lt[0, 3] = 0.0, np.inf
    _, r = run(w, layer_terms=lt, want_yelt=True)
    ref, _ = brute_yelt(w, layer_terms=lt)
    off = w.yet.offsets
    for t in range(w.yet.n_trials):
        a, b = off[t], off[t + 1]
        S = r["s_pre"][0, t]
        assert np.all(np.abs(r["yelt"][0][a:b] - ref[0][a:b]) <= 4 * max(b - a, 1) * U * S)


def test_threaded_reverse_sweep_matches_sequential():
    """The trial split of the reverse sweep changes only the order in which
    per-trial contributions are added."""
    w = synth.tiny_random(4, n_trials=400, max_events=40, n_layers=2)
    tb, r = run(w)
    cot = np.random.default_rng(9).normal(size=(3,) + r["ylt"].shape)
    ge1, gl1 = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot)
    ge4, gl4 = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot, n_threads=4)
    ge4b, gl4b = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot, n_threads=4)
    assert np.array_equal(ge4, ge4b) and np.array_equal(gl4, gl4b)
    scale_e = np.abs(ge1).max() + 1e-300
    scale_l = np.abs(gl1).max() + 1e-300
    assert np.abs(ge4 - ge1).max() <= 1e-12 * scale_e
    assert np.abs(gl4 - gl1).max() <= 1e-12 * scale_l
