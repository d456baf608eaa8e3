"""Parity of the HIP backward (reverse sweep of Algorithm 1) against the
oracle's literal reverse sweep, plus properties that hold at full size:
Euler's identity for the positively homogeneous metrics, the aggregate-term
gradients as counts, central differences, bitwise repeatability.

Tolerance, entry by entry: |g_gpu - g_ref| <= 1e-9 * A, where A is the sum
of the absolute contributions to that entry, sum_t |c_t| |dY_t/dtheta|.
For every term theta the per-trial derivative dY_t/dtheta has one sign over
all trials (scales and limits non-negative, retentions non-positive), so A
is the oracle's sweep fed |c|, and for a cotangent row without negative
entries (the metric weights) A = |g_ref|: plain relative error.  An entry
with A = 0 must be exactly 0.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from _indep import load_hand_example

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _say(msg):
    print(f"[gpu-backward] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


class Engine:
    def __init__(self, ara, w, device="cuda"):
        import torch
        self.ara, self.w = ara, w
        self.tables = ara.EltTables.from_numpy(w.elts, device)
        self.yet = ara.PreparedYet.from_numpy(w.yet, device)
        self.layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
        self.et = torch.tensor(w.elts.terms, dtype=torch.float64, device=device)
        self.lt = torch.tensor(w.layers.terms, dtype=torch.float64, device=device)

    def forward(self, t0=0, t1=None, et=None, lt=None):
        return self.ara.ylt_forward(self.tables, self.yet, self.layers, self.et if et is None else et,
                                    self.lt if lt is None else lt, t0, t1, want_s_pre=True, check=True)

    def backward(self, s_pre, cot, t0=0, t1=None, et=None, lt=None):
        import torch
        c = torch.tensor(cot, dtype=torch.float64, device="cuda") if isinstance(cot, np.ndarray) else cot
        ge, gl = self.ara.ylt_backward(self.tables, self.yet, self.layers, self.et if et is None else et,
                                       self.lt if lt is None else lt, s_pre, c, t0, t1)
        return ge.cpu().numpy(), gl.cpu().numpy()


def abs_contrib(tb, w, cots, ref, t0=0, t1=None, threads=1):
    """Sum of the absolute contributions to every gradient entry: |ref| when
    no cotangent entry is negative, else the oracle's sweep fed |c|."""
    cots = np.asarray(cots)
    if np.all(cots >= 0):
        return np.abs(ref[0]), np.abs(ref[1])
    ge, gl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, np.abs(cots), t0, t1,
                             n_threads=threads)
    return np.abs(ge), np.abs(gl)


def close(got, ref, absref, tol=TOL):
    err = np.abs(got - ref)
    bad = err > tol * absref
    if bad.any():
        i = np.unravel_index(np.argmax(np.where(bad, err / np.maximum(absref, 1e-300), 0)), err.shape)
        raise AssertionError(f"{bad.sum()} entries off; worst at {i}: gpu {got[i]!r} oracle {ref[i]!r} "
                             f"(sum of |contributions| {absref[i]!r})")


def test_hand_example_gradients(ara):
    w, g = load_hand_example()
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    _, wts = ara.metrics(ylt, g["grad_p"], want_weights=True)
    ge, gl = e.backward(s_pre, wts)
    for i, name in enumerate(["aal", "pml", "tvar"]):
        np.testing.assert_allclose(ge[i], np.array(g["grad"][name]["elt"]), rtol=0, atol=1e-12)
        np.testing.assert_allclose(gl[i, 0], np.array(g["grad"][name]["layer"]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_tiny_random_vs_oracle_sweep(ara, seed):
    w = synth.tiny_random(seed + 40, n_trials=60 + 17 * seed, max_events=25, catalog=48 + 61 * seed, n_layers=3)
    _say(f"tiny seed {seed}")
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms)
    g = np.random.default_rng(seed)
    cots = np.concatenate([oracle.metric_weights(ref["ylt"], w.p),
                           g.normal(size=(1,) + ref["ylt"].shape)], axis=0)     # 4 rows, one of mixed sign
    ge, gl = e.backward(s_pre, cots)
    rge, rgl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cots)
    ae, al = abs_contrib(tb, w, cots, (rge, rgl))
    close(ge, rge, ae)
    close(gl, rgl, al)


def test_trial_subrange_vs_oracle(ara):
    w = synth.config(2, n_trials=6000)
    e = Engine(ara, w)
    t0, t1 = 1234, 5000
    ylt, s_pre, _ = e.forward(t0, t1)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, t0, t1, n_threads=8)
    cot = oracle.metric_weights(ref["ylt"], 0.9)
    ge, gl = e.backward(s_pre, cot, t0, t1)
    rge, rgl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot, t0, t1)
    ae, al = abs_contrib(tb, w, cot, (rge, rgl), t0, t1)
    close(ge, rge, ae)
    close(gl, rgl, al)


def test_config0_all_capped(ara):
    """Every trial of the 10k x 1000 case exceeds the aggregate limit: only
    the aggregate limit has a non-zero AAL gradient (= 1)."""
    w = synth.config(0)
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    _, wts = ara.metrics(ylt, w.p, want_weights=True)
    ge, gl = e.backward(s_pre, wts)
    assert np.all(ge[0] == 0.0)
    assert gl[0, 0, :3].tolist() == [0.0, 0.0, 0.0]
    assert gl[0, 0, 3] == pytest.approx(1.0, rel=1e-12)     # sum of 10,000 weights of 1e-4


def _euler(ara, e, ge, gl, m, w):
    for c in range(3):
        tot = 0.0
        for k in range(w.elts.n_elts):
            for col in range(3):
                if np.isfinite(w.elts.terms[k, col]):
                    tot += w.elts.terms[k, col] * ge[c, k, col]
        for col in range(4):
            if np.isfinite(w.layers.terms[0, col]):
                tot += w.layers.terms[0, col] * gl[c, 0, col]
        assert abs(tot - m[c]) <= 1e-9 * abs(m[c]), (c, tot, m[c])


def test_config3_prefix_vs_oracle_and_euler(ara):
    _say("workload 3 prefix (30k trials)")
    w = synth.config(3, n_trials=30_000)
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    m, wts = ara.metrics(ylt, w.p, want_weights=True)
    ge, gl = e.backward(s_pre, wts)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=8)
    cot = wts.cpu().numpy()                          # the same cotangent rows on both sides
    np.testing.assert_array_equal(cot, oracle.metric_weights(ref["ylt"], w.p))
    rge, rgl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot)
    ae, al = abs_contrib(tb, w, cot, (rge, rgl))
    close(ge, rge, ae)
    close(gl, rgl, al)
    _euler(ara, e, ge, gl, m.cpu().numpy()[0], w)


def test_config3_full_size_properties(ara):
    """1M x 1000 x 15 with perturbed terms: Euler's identity, aggregate-term
    gradients as counts, central differences for AggR and AggL (a kink-sparse
    direction), and a bitwise-identical second run."""
    import torch
    _say("workload 3 full size")
    w = synth.config(3)
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    m, wts = ara.metrics(ylt, w.p, want_weights=True)
    ge, gl = e.backward(s_pre, wts)
    ge2, gl2 = e.backward(s_pre, wts)
    assert np.array_equal(ge, ge2) and np.array_equal(gl, gl2)
    mm = m.cpu().numpy()[0]
    _euler(ara, e, ge, gl, mm, w)
    S = s_pre.cpu().numpy()[0]
    aggR, aggL = w.layers.terms[0, 2], w.layers.terms[0, 3]
    z = S - aggR
    a = np.where(z > 0, z, 0.0)
    n = S.shape[0]
    assert gl[0, 0, 2] == pytest.approx(-np.count_nonzero((z > 0) & (a < aggL)) / n, rel=1e-12)
    assert gl[0, 0, 3] == pytest.approx(np.count_nonzero(a >= aggL) / n, rel=1e-12, abs=1e-15)
    for col in (2, 3):
        h = 1e-4 * w.layers.terms[0, col]
        vals = []
        for sgn in (+1, -1):
            lt = e.lt.clone()
            lt[0, col] += sgn * h
            y2, _, _ = e.forward(lt=lt)
            vals.append(ara.metrics(y2, w.p)[0].cpu().numpy()[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        for c in range(3):
            scale = max(abs(fd[c]), abs(gl[c, 0, col]), 1e-12)
            assert abs(fd[c] - gl[c, 0, col]) <= 2e-2 * scale + 1e-9, (col, c, fd[c], gl[c, 0, col])


def test_config3_full_size_vs_oracle(ara):
    """1M x 1000 x 15 with perturbed terms: the gradients of AAL, PML and TVaR
    with respect to every term against the oracle's literal reverse sweep
    over every trial, fed the same cotangent rows."""
    _say("workload 3 full size: GPU forward, metrics, backward")
    w = synth.config(3)
    e = Engine(ara, w)
    ylt, s_pre, _ = e.forward()
    _, wts = ara.metrics(ylt, w.p, want_weights=True)
    ge, gl = e.backward(s_pre, wts)
    _say("workload 3 full size: oracle reverse sweep")
    tb = oracle.build_tables(w.elts)
    cot = wts.cpu().numpy()
    rge, rgl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, cot,
                               n_threads=oracle.num_threads_available())
    ae, al = abs_contrib(tb, w, cot, (rge, rgl), threads=oracle.num_threads_available())
    close(ge, rge, ae)
    close(gl, rgl, al)


def test_autograd_matches_direct_call(ara):
    import torch
    w = synth.config(2, n_trials=3000)
    e = Engine(ara, w)
    et = e.et.clone().requires_grad_(True)
    lt = e.lt.clone().requires_grad_(True)
    ylt = ara.YLT.apply(et, lt, (e.tables, e.yet, e.layers, 0, w.yet.n_trials))
    m = ara.Metrics.apply(ylt, 0.95)
    coef = torch.tensor([[1.0, 0.5, 2.0]] * w.layers.n_layers, dtype=torch.float64, device="cuda")
    (m * coef).sum().backward()
    y, s, _ = e.forward()
    _, wts = ara.metrics(y, 0.95, want_weights=True)
    cot = (coef[:, 0:1] * wts[0] + coef[:, 1:2] * wts[1] + coef[:, 2:3] * wts[2]).contiguous()
    ge, gl = e.backward(s, cot)
    np.testing.assert_allclose(et.grad.cpu().numpy(), ge, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(lt.grad.cpu().numpy(), gl, rtol=1e-12, atol=1e-15)


def test_cotangent_row_limit(ara):
    import torch
    w = synth.tiny_random(3)
    e = Engine(ara, w)
    _, s_pre, _ = e.forward()
    with pytest.raises(ara.AraError) as ex:
        e.backward(s_pre, torch.zeros((5, w.layers.n_layers, w.yet.n_trials), dtype=torch.float64, device="cuda"))
    assert ex.value.status == 6


# ---------------------------------------------------------- the two forms of W
def _both_forms(ara, w):
    import torch
    tables = ara.EltTables.from_numpy(w.elts)
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")
    with_tm = ara.PreparedYet.from_numpy(w.yet, trial_major=True)
    without = ara.PreparedYet.from_numpy(w.yet, trial_major=False)

    def run(yet, s_pre, cot, t0=0, t1=None):
        ge, gl = ara.ylt_backward(tables, yet, layers, et, lt, s_pre, cot, t0, t1)
        return ge.cpu().numpy(), gl.cpu().numpy()

    ylt, s_pre, _ = ara.ylt_forward(tables, with_tm, layers, et, lt, want_s_pre=True)
    sparse = lambda *a, **k: run(with_tm, *a, **k)   # noqa: E731
    sparse.slice_trials = int(with_tm.handle.slice_trials)
    return ylt, s_pre, sparse, (lambda *a, **k: run(without, *a, **k))


def test_deviating_trial_form_is_bitwise_the_gather(ara):
    """Cotangents constant over most trials take W from the deviating trials'
    events; the same call on a YET without the trial-major copy takes the
    gather.  The fixed-point sums are exact, so the results are identical
    bit for bit: metric weights (AAL nearly constant, PML and TVaR nearly
    zero), deviating-trial counts at the sixteenth of the trials and one above,
    and sub-ranges with a non-zero common value (the occurrence counts then
    come from the event-major slices the range covers whole and a count over
    the slices it cuts) and with zero: cutting two slices, one, none (the
    range on slice boundaries), and lying inside one slice."""
    import torch
    _say("workload 2 prefix (24k trials, 4 layers): both forms of W")
    w = synth.config(2, n_trials=24_000)
    ylt, s_pre, sparse, dense = _both_forms(ara, w)
    n = w.yet.n_trials
    _, wts = ara.metrics(ylt, 0.99, want_weights=True)
    cases = [("metric weights", wts, 0, None), ("PML and TVaR rows", wts[1:].contiguous(), 0, None)]
    g = np.random.default_rng(8)
    for nd in (n // 16, n // 16 + 1, 1, 0):
        c = np.full((2, w.layers.n_layers, n), 1.0 / n)
        c[1] = 0.0
        idx = g.choice(n, size=nd, replace=False)
        c[0, :, idx] = g.uniform(-2.0, 2.0, size=(nd, w.layers.n_layers)) / n
        c[1, :, idx[: nd // 2]] = 3.0
        cases.append((f"{nd} deviating trials", torch.tensor(c, device="cuda"), 0, None))
    # one row (packed one wide) and four rows (the most: packed four wide)
    cases.append(("AAL row alone", wts[:1].contiguous(), 0, None))
    four = torch.cat([wts, wts[2:3] * 0.5], dim=0).contiguous()
    four[3, :, :7] = 1.0
    cases.append(("four rows", four, 0, None))
    _, wts_sub = ara.metrics(ylt[:, 5000:17000].contiguous(), 0.95, want_weights=True)
    cases.append(("sub-range, AAL row", wts_sub, 5000, 17000))
    st = sparse.slice_trials
    assert 5000 % st and 17000 % st and 5000 // st != 17000 // st   # two cut slices
    for a0, a1, label in [(st, 5 * st, "on slice boundaries"), (0, 2 * st + st // 3, "one cut slice"),
                          (st + 17, 2 * st - 5, "inside one slice"), (3 * st + 1, 3 * st + 3, "two trials")]:
        a1 = min(a1, n)
        _, wts_r = ara.metrics(ylt[:, a0:a1].contiguous(), 0.9, want_weights=True)
        cases.append((f"sub-range {label}, every row", wts_r, a0, a1))
    # most of the trials
    _, wts_near = ara.metrics(ylt[:, 400:23400].contiguous(), 0.99, want_weights=True)
    cases.append(("near-full sub-range, every row", wts_near, 400, 23400))
    cases.append(("near-full sub-range, AAL row", wts_near[:1].contiguous(), 400, 23400))
    cases.append(("sub-range, PML and TVaR rows", wts_sub[1:].contiguous(), 5000, 17000))
    for label, cot, t0, t1 in cases:
        _say(label)
        sp = s_pre if t1 is None else s_pre[:, t0:t1].contiguous()
        a = sparse(sp, cot, t0, t1)
        b = dense(sp, cot, t0, t1)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), label


def test_deviating_trial_form_full_size_vs_oracle(ara):
    """1M x 1000 x 15 (the differentiated workload), where every trial's
    aggregate clamp is linear: the metric weights go through the
    deviating-trial form (AAL constant, PML and TVaR zero outside about
    10,000 trials) and give the gather's gradients bit for bit."""
    _say("workload 3: generating 1M x 1000")
    w = synth.config(3)
    ylt, s_pre, sparse, dense = _both_forms(ara, w)
    _, wts = ara.metrics(ylt, w.p, want_weights=True)
    _say("workload 3: both forms")
    a = sparse(s_pre, wts)
    b = dense(s_pre, wts)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a range over 96% of the trials: its first and last slices are cut
    t0, t1 = 20_000, w.yet.n_trials - 20_000
    _say("workload 3: both forms over trials [20000, 980000)")
    _, wsub = ara.metrics(ylt[:, t0:t1].contiguous(), w.p, want_weights=True)
    sp = s_pre[:, t0:t1].contiguous()
    a = sparse(sp, wsub, t0, t1)
    b = dense(sp, wsub, t0, t1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
