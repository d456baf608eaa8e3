"""The grouped forward: four layers served by one workgroup per block (one
decode and one union-table probe per code, the per-layer work on queued
union hits).  It serves the full groups of four layers of a call without
hit counts; the other layers, and every call with hit counts, take the
one-layer kernel, which the grouped results are compared with, besides the
oracle.

Tolerances as in test_gpu_forward: hits bit-exact, Y within
1e-9 * max(Y, S), S within 1e-9 relative."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _say(msg):
    print(f"[gpu-grouped] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


def _run(ara, w, t0=0, t1=None, hits=False):
    import torch
    tables = ara.EltTables.from_numpy(w.elts)
    yet = ara.PreparedYet.from_numpy(w.yet, transposed=False, trial_major=False)
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")
    y, s, h = ara.ylt_forward(tables, yet, layers, et, lt, t0, t1, want_s_pre=True, want_hits=hits, check=True)
    return y.cpu().numpy(), s.cpu().numpy(), (None if h is None else h.cpu().numpy())


def _check(y, s, ref):
    bound = TOL * np.maximum(np.abs(ref["ylt"]), ref["s_pre"])
    bad = np.abs(y - ref["ylt"]) > bound
    assert not bad.any(), f"{bad.sum()} year losses off"
    assert not (np.abs(s - ref["s_pre"]) > TOL * ref["s_pre"]).any()


def _layers(w, lists, terms):
    off = np.zeros(len(lists) + 1, np.int32)
    np.cumsum([len(x) for x in lists], out=off[1:])
    ids = np.concatenate([np.asarray(x, np.int32) for x in lists]) if off[-1] else np.zeros(0, np.int32)
    return synth.Layers(off, ids, np.asarray(terms, np.float64))


def test_uneven_four_layers_vs_oracle_and_one_layer_kernel(ara):
    """The uneven workload's first 20,000 trials: four layers in one group."""
    w = synth.config(2, n_trials=20_000)
    _say("workload 2 prefix: grouped and one-layer kernels")
    y, s, _ = _run(ara, w)
    yh, sh, h = _run(ara, w, hits=True)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=8)
    _check(y, s, ref)
    _check(yh, sh, ref)
    assert np.array_equal(h, ref["hits"])
    # the same additions in the same order per trial: equal bit for bit
    assert np.array_equal(s, sh) and np.array_equal(y, yh)


@pytest.mark.parametrize("n_layers", [2, 3, 5, 9])
def test_group_sizes_vs_oracle(ara, n_layers):
    """Two and three layers (the one-layer kernel each), five (a group of
    four and one more) and nine (two groups and one more), with ELT lists
    sharing ELTs and a layer with no ELTs among them."""
    g = np.random.default_rng(n_layers)
    w = synth.config(2, n_trials=6_000)
    lists = [g.choice(55, size=int(g.integers(1, 16)), replace=False) for _ in range(n_layers)]
    if n_layers >= 5:
        lists[2] = []
    w.layers = _layers(w, lists, synth.random_layer_terms(g, n_layers))
    _say(f"{n_layers} layers")
    y, s, _ = _run(ara, w)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=8)
    _check(y, s, ref)
    if n_layers >= 5:
        assert np.all(y[2] == 0.0) and np.all(s[2] == 0.0)


def test_trial_subranges(ara):
    w = synth.config(2, n_trials=9_000)
    y, s, _ = _run(ara, w)
    for t0, t1 in [(0, 1), (17, 4099), (4096, 4097), (8000, 9000), (123, 123), (1, 8999)]:
        ys, ss, _ = _run(ara, w, t0, t1)
        assert np.array_equal(ys, y[:, t0:t1]) and np.array_equal(ss, s[:, t0:t1])


def test_tables_beyond_lds_and_many_ranges(ara):
    """Members whose set events do not fit the workgroup's LDS (every event
    of dense ELTs set: values read from global memory) over a catalogue of
    5,000,000 events (153 ranges: the range counts are staged in windows of
    64), against the oracle."""
    g = np.random.default_rng(3)
    cat = 5_000_000
    n = 3000
    lens = g.integers(0, 400, size=n)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    ids = g.integers(0, cat, size=int(off[-1])).astype(np.int32)
    ids[: int(off[-1]) // 2] = g.integers(0, 300_000, size=int(off[-1]) // 2)   # crowd the first ranges
    sizes = [200_000, 150_000, 40_000, 5_000]
    recs, losses = [], []
    for k, sz in enumerate(sizes):
        pool = 300_000 if k < 2 else cat
        recs.append(np.sort(g.choice(pool, size=sz, replace=False)))
        losses.append(np.exp(g.normal(10.0, 1.0, size=sz)))
    rec_off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=rec_off[1:])
    elts = synth.Elts(cat, rec_off, np.concatenate(recs).astype(np.int32),
                      np.concatenate(losses).astype(np.float32),
                      np.array([[1.0, 0.0, np.inf], [1.2, 0.0, np.inf], [1.0, 5e3, 1e6], [0.7, 0.0, 5e5]]))
    layers = _layers(None, [[0, 1], [1], [2, 3], [0, 2, 3]],
                     [[0.0, np.inf, 0.0, np.inf], [1e3, 1e7, 1e5, 1e9], [0.0, 2e6, 0.0, np.inf], [5e3, 5e6, 1e6, 5e8]])
    w = synth.Workload("dense", synth.Yet(cat, off, ids), elts, layers, 0.9)
    _say("dense tables over a 5M catalogue")
    y, s, _ = _run(ara, w)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=8)
    _check(y, s, ref)


def test_repeatable(ara):
    w = synth.config(2, n_trials=5000)
    a = _run(ara, w)
    b = _run(ara, w)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
