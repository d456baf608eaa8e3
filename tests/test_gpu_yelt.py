"""Parity of the per-occurrence losses (event-level YLT) and the per-year
maximum occurrence loss with the oracle's literal step four.  The running
total is summed in wavefront order on the GPU and sequentially in the
oracle, so values agree to rounding: |gpu - ref| <= 1e-9 * S (S the trial's
total before aggregate terms, which bounds every running total); exact on
the integer-valued worked example."""
import sys

import numpy as np
import pytest

import oracle
import synth
from _indep import load_hand_example

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _say(msg):
    print(f"[gpu-yelt] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


def run(ara, w, t0=0, t1=None, lt=None, check=True):
    import torch
    tables = ara.EltTables.from_numpy(w.elts, "cuda")
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    off = torch.from_numpy(np.ascontiguousarray(w.yet.offsets, np.int64)).cuda()
    ids = torch.from_numpy(np.ascontiguousarray(w.yet.ids, np.int32)).cuda()
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms if lt is None else lt, dtype=torch.float64, device="cuda")
    y, m = ara.yelt_forward(tables, off, ids, layers, et, lt, t0, t1, check=check)
    return y.cpu().numpy(), m.cpu().numpy()


def oracle_ref(w, t0=0, t1=None, lt=None, threads=1):
    tb = oracle.build_tables(w.elts)
    return oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms if lt is None else lt, t0, t1,
                          n_threads=threads, want_yelt=True)


def assert_close(y, m, ref, off, t0=0):
    S = ref["s_pre"]
    base = off[t0]
    for j in range(S.shape[0]):
        per_occ_S = np.repeat(S[j], np.diff(off[t0:t0 + S.shape[1] + 1]))
        assert np.all(np.abs(y[j] - ref["yelt"][j]) <= TOL * per_occ_S), f"layer {j}"
        assert np.all(np.abs(m[j] - ref["occ_max"][j]) <= TOL * S[j]), f"layer {j}"
    assert base >= 0


def test_hand_example_exact(ara):
    w, g = load_hand_example()
    y, m = run(ara, w)
    assert y[0].tolist() == [v for t in g["yelt"] for v in t]
    assert m[0].tolist() == g["occ_max"]


@pytest.mark.parametrize("seed", range(8))
def test_tiny_random_vs_oracle(ara, seed):
    w = synth.tiny_random(seed, n_trials=300, max_events=200, n_layers=3)
    _say(f"seed {seed}")
    y, m = run(ara, w)
    assert_close(y, m, oracle_ref(w), w.yet.offsets)


def test_long_trials_and_many_ranges(ara):
    """Trials of 0..3000 occurrences (many 256-occurrence steps, ragged
    tails) over a 300,000-event catalogue; one event repeated in a trial."""
    g = np.random.default_rng(21)
    lens = g.integers(0, 3001, size=400)
    lens[::9] = 0
    lens[5] = 1
    off = np.zeros(401, np.int64)
    np.cumsum(lens, out=off[1:])
    ids = g.integers(0, 300_000, size=int(off[-1]), dtype=np.int32)
    ids[off[3]:off[3] + 500] = 4242
    elts = synth.lognormal_elts(5, [40_000, 25_000, 60_000], 300_000, mu=11.0)
    if 4242 not in elts.rec_ids[:elts.rec_off[1]]:
        elts.rec_ids[0] = 4242
    layers = synth.Layers(np.array([0, 3, 4], np.int32), np.array([0, 1, 2, 1], np.int32),
                          np.array([[1e4, 5e6, 1e6, 5e7], [0.0, np.inf, 0.0, np.inf]]))
    w = synth.Workload("long", synth.Yet(300_000, off, ids), elts, layers, 0.9)
    y, m = run(ara, w)
    ref = oracle_ref(w, threads=oracle.num_threads_available())
    assert_close(y, m, ref, off)
    # without aggregate terms the year loss is the plain sum of the increments
    assert np.allclose([y[1][off[t]:off[t + 1]].sum() for t in range(400)], ref["ylt"][1], rtol=1e-12, atol=0)


def test_trial_subranges_are_slices(ara):
    w = synth.config(2, n_trials=3000)
    y, m = run(ara, w)
    off = w.yet.offsets
    for t0, t1 in [(0, 1), (17, 2099), (2999, 3000), (5, 5)]:
        ys, ms = run(ara, w, t0, t1)
        assert np.array_equal(ys, y[:, off[t0]:off[t1]]) and np.array_equal(ms, m[:, t0:t1])


def test_sums_match_year_loss_of_forward(ara):
    import torch
    w = synth.config(1, n_trials=5000)
    y, m = run(ara, w)
    tables = ara.EltTables.from_numpy(w.elts, "cuda")
    yet = ara.PreparedYet.from_numpy(w.yet, "cuda", transposed=False)
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")
    ylt, s_pre, _ = ara.ylt_forward(tables, yet, layers, et, lt)
    ylt, s_pre = ylt.cpu().numpy(), s_pre.cpu().numpy()
    off = w.yet.offsets
    sums = np.array([y[0][off[t]:off[t + 1]].sum() for t in range(w.yet.n_trials)])
    assert np.all(np.abs(sums - ylt[0]) <= TOL * s_pre[0])
    assert np.all(m[0] <= ylt[0] * (1 + 1e-12))


def test_invalid_id_and_empty(ara):
    w = synth.tiny_random(3, n_trials=20)
    ids = w.yet.ids.copy()
    if len(ids):
        ids[len(ids) // 2] = w.yet.catalog
    bad = synth.Workload("bad", synth.Yet(w.yet.catalog, w.yet.offsets, ids), w.elts, w.layers, w.p)
    with pytest.raises(ara.AraError):
        run(ara, bad)
    empty = synth.Workload("empty", synth.Yet(w.yet.catalog, np.zeros(11, np.int64), np.zeros(0, np.int32)),
                           w.elts, w.layers, w.p)
    y, m = run(ara, empty)
    assert y.shape == (w.layers.n_layers, 0) and np.all(m == 0.0)


def test_config1_full_size_sampled(ara):
    """1,000,000 trials x 1000 occurrences (the benchmark workload): every
    trial's maximum and a sample of trials' increments against the oracle."""
    import torch
    w = synth.config(1)
    _say("config 1 generated")
    y, m = run(ara, w)
    _say("yelt done")
    off = w.yet.offsets
    for t0 in (0, 123_457, 999_000):
        t1 = t0 + 1000
        ref = oracle_ref(w, t0, t1, threads=oracle.num_threads_available())
        ys = y[:, off[t0]:off[t1]]
        ms = m[:, t0:t1]
        per_occ_S = np.repeat(ref["s_pre"][0], np.diff(off[t0:t1 + 1]))
        assert np.all(np.abs(ys[0] - ref["yelt"][0]) <= TOL * per_occ_S)
        assert np.all(np.abs(ms[0] - ref["occ_max"][0]) <= TOL * ref["s_pre"][0])
    del y
    torch.cuda.empty_cache()
