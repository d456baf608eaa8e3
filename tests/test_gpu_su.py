"""Secondary uncertainty on the GPU (ara_ylt_forward_su) against the oracle:
every trial at small sizes, sampled trial ranges at 1M x 1000, sigma = 0
against the deterministic path, determinism, subranges, layers alone and
together, and errors.

Tolerance: the draws use the device's binary64 log, cos and exp (within an
ulp or two of the host's), and a trial's occurrence losses are summed in the
order of the prepared layout (by catalogue range), not in storage order, so
YLT and S agree with the oracle to 1e-9 of the trial's total before
aggregate terms."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _say(msg):
    print(f"[gpu-su] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


class Su:
    def __init__(self, ara, w, rec_sigma):
        import torch
        self.ara, self.w = ara, w
        self.tables = ara.EltTables.from_numpy(w.elts)
        self.sigma = ara.SigmaTables.from_numpy(self.tables, rec_sigma)
        self.layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
        self.yet = ara.PreparedYet.from_numpy(w.yet, transposed=False, positions=True)
        self.et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
        self.lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")

    def run(self, seed, t0=0, t1=None, layers=None, lt=None):
        y, s = self.ara.ylt_forward_su(self.tables, self.sigma, self.yet, layers or self.layers, self.et,
                                       self.lt if lt is None else lt, seed, t0, t1, check=True)
        return y.cpu().numpy(), s.cpu().numpy()


def oracle_su(w, rec_sigma, seed, t0=0, t1=None, threads=1):
    tb = oracle.build_tables(w.elts)
    st = oracle.build_sigma_tables(w.elts, rec_sigma)
    return oracle.forward_su(tb, st, w.yet, w.layers, w.elts.terms, w.layers.terms, seed, t0, t1, n_threads=threads)


def assert_close(y, s, ref):
    bound = TOL * np.maximum(np.abs(ref["ylt"]), ref["s_pre"])
    bad = np.abs(y - ref["ylt"]) > bound
    assert not bad.any(), f"{bad.sum()} year losses off; worst {np.abs(y - ref['ylt'])[bad].max()}"
    sb = np.abs(s - ref["s_pre"]) > TOL * ref["s_pre"]
    assert not sb.any(), f"{sb.sum()} totals off"


@pytest.mark.parametrize("seed", range(5))
def test_tiny_random_vs_oracle(ara, seed):
    _say(f"tiny seed {seed}")
    w = synth.tiny_random(seed, n_trials=60, max_events=20, n_layers=2)
    sg = synth.record_sigmas(seed + 100, w.elts, zero_frac=0.2)
    y, s = Su(ara, w, sg).run(1000 + seed)
    assert_close(y, s, oracle_su(w, sg, 1000 + seed))


def test_sigma_zero_is_the_deterministic_forward(ara):
    _say("sigma = 0 on workload 0 (2000 trials)")
    w = synth.config(0, n_trials=2000)
    sg = np.zeros(w.elts.rec_loss.shape[0], np.float32)
    y, s = Su(ara, w, sg).run(5)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=4)
    assert_close(y, s, ref)


def test_config0_every_trial(ara):
    _say("workload 0 (10k x 1000, 15 ELTs): every trial")
    w = synth.config(0)
    sg = synth.record_sigmas(synth.SEED_BASE, w.elts)
    e = Su(ara, w, sg)
    y, s = e.run(42)
    assert_close(y, s, oracle_su(w, sg, 42, threads=oracle.num_threads_available()))
    # not the deterministic answer: the draws move most year losses
    ref_det = oracle.forward(oracle.build_tables(w.elts), w.yet, w.layers, w.elts.terms, w.layers.terms,
                             n_threads=oracle.num_threads_available())
    assert np.mean(np.abs(s - ref_det["s_pre"]) > 1e-6 * ref_det["s_pre"]) > 0.9


def test_config2_prefix_four_layers(ara):
    _say("workload 2 prefix (6000 x Poisson(1000), 4 layers over 55 ELTs)")
    w = synth.config(2, n_trials=6000)
    sg = synth.record_sigmas(synth.SEED_BASE + 2, w.elts)
    y, s = Su(ara, w, sg).run(7)
    assert_close(y, s, oracle_su(w, sg, 7, threads=oracle.num_threads_available()))


def test_run_twice_subranges_and_seeds(ara):
    _say("determinism, subranges, seeds")
    w = synth.config(0, n_trials=3000)
    sg = synth.record_sigmas(3, w.elts)
    e = Su(ara, w, sg)
    y1, s1 = e.run(9)
    y2, s2 = e.run(9)
    assert np.array_equal(y1, y2) and np.array_equal(s1, s2)
    ys, ss = e.run(9, 1234, 2345)
    assert np.array_equal(ys, y1[:, 1234:2345]) and np.array_equal(ss, s1[:, 1234:2345])
    y3, s3 = e.run(10)
    assert np.mean(s3 != s1) > 0.9


def test_layers_alone_and_together(ara):
    """Each layer run alone gives, bit for bit, its row of the call over all
    layers (the layers of one block run back to back and share its codes)."""
    import torch
    _say("workload 2 prefix: four layers together and one at a time")
    w = synth.config(2, n_trials=3000)
    sg = synth.record_sigmas(11, w.elts)
    e = Su(ara, w, sg)
    y, s = e.run(3)
    off, ids = w.layers.elt_off, w.layers.elt_ids
    for j in range(w.layers.n_layers):
        lay = ara.Layers(np.array([0, off[j + 1] - off[j]], np.int32), ids[off[j]:off[j + 1]])
        lt = torch.tensor(np.asarray(w.layers.terms)[j:j + 1], dtype=torch.float64, device="cuda")
        yj, sj = e.run(3, layers=lay, lt=lt)
        assert np.array_equal(yj[0], y[j]) and np.array_equal(sj[0], s[j]), j


def test_long_trials_and_ragged_blocks(ara):
    """Trials of up to 20,000 occurrences (positions past 2^14), empty trials,
    and a trial count that leaves the last block and group ragged."""
    _say("long and empty trials against the oracle")
    rng = np.random.default_rng(130825)
    w = synth.config(0, n_trials=700)
    lens = rng.integers(0, 3000, size=700)
    lens[::97] = 0
    lens[5] = 20_000
    lens[400] = 12_345
    off = np.zeros(701, np.int64)
    off[1:] = np.cumsum(lens)
    ids = rng.integers(0, w.yet.catalog, size=int(off[-1])).astype(np.int32)
    w = synth.Workload("long trials", synth.Yet(w.yet.catalog, off, ids), w.elts, w.layers, w.p)
    sg = synth.record_sigmas(5, w.elts)
    y, s = Su(ara, w, sg).run(77)
    assert_close(y, s, oracle_su(w, sg, 77, threads=oracle.num_threads_available()))


def test_config1_full_size_sampled(ara):
    """1M x 1000 x 15 with deviations; the oracle on three trial ranges."""
    _say("workload 1: generating 1M x 1000")
    w = synth.config(1)
    sg = synth.record_sigmas(synth.SEED_BASE + 1, w.elts)
    e = Su(ara, w, sg)
    _say("workload 1: secondary-uncertainty forward")
    y, s = e.run(2024)
    th = oracle.num_threads_available()
    tb = oracle.build_tables(w.elts)
    st = oracle.build_sigma_tables(w.elts, sg)
    for t0, t1 in [(0, 1500), (499_000, 500_000), (w.yet.n_trials - 1000, w.yet.n_trials)]:
        _say(f"workload 1: oracle on trials [{t0}, {t1})")
        ref = oracle.forward_su(tb, st, w.yet, w.layers, w.elts.terms, w.layers.terms, 2024, t0, t1, n_threads=th)
        assert_close(y[:, t0:t1], s[:, t0:t1], ref)


def test_config2_full_size_sampled_and_layers_alone(ara):
    """1M x Poisson(1000), four layers over 55 ELTs: the layers of a block
    dealt to one XCD back to back over all blocks; the oracle on three trial
    windows, and one layer run alone equal to its row bit for bit."""
    import torch
    _say("workload 2: generating 1M x Poisson(1000), 4 layers")
    w = synth.config(2)
    sg = synth.record_sigmas(synth.SEED_BASE + 22, w.elts)
    e = Su(ara, w, sg)
    _say("workload 2: secondary-uncertainty forward, four layers")
    y, s = e.run(2026)
    th = oracle.num_threads_available()
    tb = oracle.build_tables(w.elts)
    st = oracle.build_sigma_tables(w.elts, sg)
    for t0, t1 in [(0, 600), (333_000, 333_700), (w.yet.n_trials - 600, w.yet.n_trials)]:
        _say(f"workload 2: oracle on trials [{t0}, {t1})")
        ref = oracle.forward_su(tb, st, w.yet, w.layers, w.elts.terms, w.layers.terms, 2026, t0, t1, n_threads=th)
        assert_close(y[:, t0:t1], s[:, t0:t1], ref)
    off, ids = w.layers.elt_off, w.layers.elt_ids
    j = 2
    lay = ara.Layers(np.array([0, off[j + 1] - off[j]], np.int32), ids[off[j]:off[j + 1]])
    lt = torch.tensor(np.asarray(w.layers.terms)[j:j + 1], dtype=torch.float64, device="cuda")
    _say("workload 2: layer 2 alone")
    yj, sj = e.run(2026, layers=lay, lt=lt)
    assert np.array_equal(yj[0], y[j]) and np.array_equal(sj[0], s[j])


def test_errors(ara):
    import torch
    w = synth.tiny_random(2, n_trials=30, max_events=10, n_layers=1)
    sg = synth.record_sigmas(1, w.elts)
    e = Su(ara, w, sg)
    # a record count smaller than the ELT: the entry layout does not fit
    saved = e.tables.records.copy()
    e.tables.records[:] = 0
    with pytest.raises(ara.AraError) as ex:
        e.run(1)
    assert ex.value.status == 6
    e.tables.records[:] = saved
    # a YET prepared without positions
    plain = ara.PreparedYet.from_numpy(w.yet, transposed=False)
    with pytest.raises(ara.AraError) as ex:
        ara.ylt_forward_su(e.tables, e.sigma, plain, e.layers, e.et, e.lt, 1)
    assert ex.value.status == 1
    # a trial of more than 65536 occurrences cannot carry positions
    off = torch.tensor([0, 70_000], dtype=torch.int64, device="cuda")
    ids = torch.zeros(70_000, dtype=torch.int32, device="cuda")
    with pytest.raises(ara.AraError) as ex:
        ara.PreparedYet(off, ids, w.yet.catalog, transposed=False, positions=True)
    assert ex.value.status == 6
    ok = torch.tensor([0, 65_536], dtype=torch.int64, device="cuda")   # the longest trial that fits
    ara.PreparedYet(ok, ids[:65_536], w.yet.catalog, transposed=False, positions=True)
    # a negative standard deviation
    bad = sg.copy()
    bad[0] = -1.0
    with pytest.raises(ara.AraError) as ex:
        ara.SigmaTables.from_numpy(e.tables, bad)
    assert ex.value.status == 1
    # empty trial range
    y, s = ara.ylt_forward_su(e.tables, e.sigma, e.yet, e.layers, e.et, e.lt, 1, 5, 5)
    assert y.shape == (1, 0)
    torch.cuda.synchronize()
