"""The binary32 accumulation mode of the forward (ARA_F_FP32_ACCUM: the
precision reduction of the paper's optimised kernel, Sections III-IV)
against the binary64 oracle, through the C ABI.

Each occurrence value O is rounded once to binary32 and a trial's total is
accumulated in binary32 (about 140 additions per trial at 1000 events over
15 ELTs), so the totals carry a relative error of a few 1e-7 and at most
n * 2^-24 for n additions; the tolerance is
  year loss Y     |Y - Y_ref| <= 1e-5 * max(Y_ref, S_ref)
  S               |S - S_ref| <= 1e-5 * S_ref
  hits            bit-exact (they do not depend on the values)
  AAL, PML, TVaR  within 1e-5 * max_t S_ref[t] (each metric moves by at most
                  the largest change of one year loss)
and a one-occurrence trial reproduces float32(O) exactly."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _say(msg):
    print(f"[gpu-fp32] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


class Engine:
    def __init__(self, ara, w):
        import torch
        self.ara, self.w = ara, w
        self.tables = ara.EltTables.from_numpy(w.elts)
        self.yet = ara.PreparedYet.from_numpy(w.yet)
        self.layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
        self.et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
        self.lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")

    def forward(self, t0=0, t1=None, hits=False, fp32=True):
        y, s, h = self.ara.ylt_forward(self.tables, self.yet, self.layers, self.et, self.lt, t0, t1,
                                       want_s_pre=True, want_hits=hits, check=True, fp32_accum=fp32)
        return y.cpu().numpy(), s.cpu().numpy(), None if h is None else h.cpu().numpy()


def oracle_ref(w, t0=0, t1=None, threads=1):
    tb = oracle.build_tables(w.elts)
    return oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, t0, t1, n_threads=threads)


def assert_close32(y, s, ref):
    bound = TOL32 * np.maximum(np.abs(ref["ylt"]), ref["s_pre"])
    bad = np.abs(y - ref["ylt"]) > bound
    assert not bad.any(), f"{bad.sum()} year losses off; worst {np.abs(y - ref['ylt'])[bad].max()}"
    sb = np.abs(s - ref["s_pre"]) > TOL32 * ref["s_pre"]
    assert not sb.any(), f"{sb.sum()} totals off"


def assert_metrics32(ara, y, ref, p):
    import torch
    out, _ = ara.metrics(torch.tensor(y, device="cuda"), p)
    want = oracle.metrics(ref["ylt"], p)
    scale = ref["s_pre"].max(axis=1)
    assert np.all(np.abs(out.cpu().numpy() - want) <= TOL32 * scale[:, None])


@pytest.mark.parametrize("seed", range(8))
def test_tiny_random_vs_oracle(ara, seed):
    _say(f"tiny seed {seed}")
    w = synth.tiny_random(seed, n_trials=41 + 11 * seed, max_events=40, catalog=60 + 50 * seed, n_layers=3)
    e = Engine(ara, w)
    ref = oracle_ref(w)
    y, s, h = e.forward(hits=True)
    assert np.array_equal(h, ref["hits"])
    assert_close32(y, s, ref)
    y2, s2, _ = e.forward(hits=False)
    assert_close32(y2, s2, ref)


def test_one_occurrence_trials_round_once(ara):
    """Every trial holds one occurrence: its total is that event's O, so the
    binary32 mode returns float32(O) exactly (one rounding, no sum)."""
    g = np.random.default_rng(3)
    base = synth.tiny_random(9, n_trials=10, catalog=5000, n_layers=2)
    n = 4000
    ids = g.integers(0, base.yet.catalog, size=n).astype(np.int32)
    hot = np.unique(base.elts.rec_ids)
    ids[: n // 2] = g.choice(hot, size=n // 2)
    w = synth.Workload("one-event", synth.Yet(base.yet.catalog, np.arange(n + 1, dtype=np.int64), ids),
                       base.elts, base.layers, 0.9)
    e = Engine(ara, w)
    ref = oracle_ref(w)
    _, s, _ = e.forward()
    assert np.array_equal(s, ref["s_pre"].astype(np.float32).astype(np.float64))
    assert (ref["s_pre"] > 0).sum() > n // 4


def test_binary64_mode_unchanged_beside_binary32(ara):
    """The same engine alternates both modes; each gives its own answer
    every time."""
    w = synth.config(0, n_trials=2000)
    e = Engine(ara, w)
    a64 = e.forward(fp32=False)
    a32 = e.forward()
    b64 = e.forward(fp32=False)
    b32 = e.forward()
    assert np.array_equal(a64[0], b64[0]) and np.array_equal(a32[0], b32[0])
    ref = oracle_ref(w, threads=4)
    assert_close32(a32[0], a32[1], ref)
    assert np.all(np.abs(a64[0] - ref["ylt"]) <= 1e-9 * np.maximum(ref["ylt"], ref["s_pre"]))


def test_config0_every_trial_and_metrics(ara):
    _say("workload 0 (10k x 1000, 15 ELTs)")
    w = synth.config(0)
    e = Engine(ara, w)
    ref = oracle_ref(w, threads=oracle.num_threads_available())
    y, s, h = e.forward(hits=True)
    assert np.array_equal(h, ref["hits"])
    assert_close32(y, s, ref)
    assert_metrics32(ara, y, ref, w.p)


def test_config2_prefix_four_layers(ara):
    _say("workload 2 prefix (20k x Poisson(1000), 4 layers)")
    w = synth.config(2, n_trials=20_000)
    e = Engine(ara, w)
    ref = oracle_ref(w, threads=oracle.num_threads_available())
    y, s, h = e.forward(hits=True)
    assert np.array_equal(h, ref["hits"])
    assert_close32(y, s, ref)
    assert_metrics32(ara, y, ref, w.p)
    ys, ss, _ = e.forward(4097, 13_001)
    assert np.array_equal(ys, y[:, 4097:13_001]) and np.array_equal(ss, s[:, 4097:13_001])


def test_config1_full_size_sampled(ara):
    """1,000,000 trials x 1,000 events, 15 ELTs, in the benchmark's launch:
    the oracle on three trial ranges; the metrics of the full binary32 YLT
    against those of the full binary64 YLT."""
    import torch
    _say("workload 1: generating 1M x 1000")
    w = synth.config(1)
    e = Engine(ara, w)
    _say("workload 1: binary32 and binary64 forwards")
    y, s, _ = e.forward()
    y64, s64, _ = e.forward(fp32=False)
    th = oracle.num_threads_available()
    tb = oracle.build_tables(w.elts)
    for t0, t1 in [(0, 2000), (500_000, 501_000), (w.yet.n_trials - 1500, w.yet.n_trials)]:
        _say(f"workload 1: oracle on trials [{t0}, {t1})")
        ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, t0, t1, n_threads=th)
        assert_close32(y[:, t0:t1], s[:, t0:t1], ref)
    assert np.all(np.abs(y - y64) <= TOL32 * np.maximum(y64, s64))
    m32, _ = ara.metrics(torch.tensor(y, device="cuda"), w.p)
    m64, _ = ara.metrics(torch.tensor(y64, device="cuda"), w.p)
    assert np.all(np.abs(m32.cpu().numpy() - m64.cpu().numpy()) <= TOL32 * s64.max())
