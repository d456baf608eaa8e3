"""The event-major copy of the YET that the backward reads (an index
transposition: exact).  For every trial slice x and event e the list of
slice-local trial indices must hold exactly the occurrences of e in the
slice's trials, with multiplicity; the list offsets are the running counts.
Checked against a numpy construction from the raw trials.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-prepare] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


def read_dev(yet, ptr, count, dtype):
    import torch
    itemsize = torch.tensor([], dtype=dtype).element_size()
    off = ptr - yet.buf.data_ptr()
    assert 0 <= off and off + count * itemsize <= yet.buf.numel()
    return yet.buf[off: off + count * itemsize].view(dtype).cpu().numpy()


def expected(yet_np, slice_trials, n_slices):
    n = yet_np.n_trials
    lens = np.diff(yet_np.offsets)
    t = np.repeat(np.arange(n, dtype=np.int64), lens)
    x = t // slice_trials
    key = x * yet_np.catalog + yet_np.ids.astype(np.int64)
    local = t - x * slice_trials
    counts = np.bincount(key, minlength=n_slices * yet_np.catalog)
    off = np.zeros(n_slices * yet_np.catalog + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    order = np.lexsort((local, key))
    return off, key[order], local[order]


def check_codes(py, yet_np):
    """Decode every segment of the 16-bit code stream on the host and compare
    it with the raw trials: same (trial, offset) sequence, in trial order and
    storage order inside a trial; with positions, each occurrence's position
    in its trial beside its code and 0xFFFF beside the other codes."""
    import torch
    h = py.handle
    G, groups, tg, tb = h.n_ranges, h.groups, h.trials_per_group, h.trials_per_block
    nseg = h.n_blocks * G * groups
    codes = read_dev(py, h.code, max(h.n_codes, 1), torch.int16).view(np.uint16).astype(np.int64)
    base = read_dev(py, h.seg_base, max(nseg, 1), torch.int64)
    run = read_dev(py, h.seg_run, max(nseg, 1), torch.int32).astype(np.int64)
    start = read_dev(py, h.lane_start, max(nseg * 64, 1), torch.uint8).astype(np.int64)
    n = yet_np.n_trials
    t = np.repeat(np.arange(n, dtype=np.int64), np.diff(yet_np.offsets))
    ids = yet_np.ids.astype(np.int64)
    key = ((t // tb) * G + (ids >> 15)) * groups + (t % tb) // tg
    order = np.argsort(key, kind="stable")
    key_s, trial_s, local_s = key[order], (t % tb % tg)[order], (ids & 0x7FFF)[order]
    pos_s = (np.arange(yet_np.nnz, dtype=np.int64) - yet_np.offsets[t])[order]
    pos = read_dev(py, h.pos, max(h.n_codes, 1), torch.int16).view(np.uint16).astype(np.int64) if h.pos else None
    bounds = np.searchsorted(key_s, np.arange(nseg + 1))
    lanes = np.arange(64)
    for si in range(nseg):
        R = int(run[si])
        a, b = bounds[si], bounds[si + 1]
        if R == 0:
            assert a == b, f"segment {si}: events but no codes"
            continue
        assert R % 4 == 0
        s = np.arange(R)
        slot = base[si] + (s[None, :] // 4) * 256 + 4 * lanes[:, None] + s[None, :] % 4   # [64, R]
        c = codes[slot]
        tr = start[si * 64: si * 64 + 64][:, None] + np.cumsum(c >> 15, axis=1)
        valid = c != 0xFFFF
        got_t, got_l = tr[valid], (c & 0x7FFF)[valid]      # row-major: lane by lane, in order
        assert np.array_equal(got_t, trial_s[a:b]), f"segment {si}: trials differ"
        assert np.array_equal(got_l, local_s[a:b]), f"segment {si}: offsets differ"
        if pos is not None:
            p = pos[slot]
            assert np.array_equal(p[valid], pos_s[a:b]), f"segment {si}: positions differ"
            assert np.all(p[~valid] == 0xFFFF), f"segment {si}: a gap or padding code has a position"
    assert h.n_codes >= yet_np.nnz


def check(ara, yet_np):
    import torch
    _say(f"trials {yet_np.n_trials} nnz {yet_np.nnz} catalog {yet_np.catalog}")
    py = ara.PreparedYet.from_numpy(yet_np, "cuda", positions=True)
    h = py.handle
    torch.cuda.synchronize()
    check_codes(py, yet_np)
    assert h.n_slices == 8
    assert h.slice_trials % h.trials_per_block == 0 and h.slice_trials * h.n_slices >= yet_np.n_trials
    off_ref, key_ref, loc_ref = expected(yet_np, h.slice_trials, h.n_slices)
    off = read_dev(py, h.tr_off, h.n_slices * yet_np.catalog + 1, torch.int64)
    assert np.array_equal(off, off_ref)
    # the trial-major copy and every event's occurrence count
    assert np.array_equal(read_dev(py, h.t_off, yet_np.n_trials + 1, torch.int64), yet_np.offsets)
    cnt = read_dev(py, h.t_cnt, yet_np.catalog, torch.int32)
    assert np.array_equal(cnt, np.bincount(yet_np.ids, minlength=yet_np.catalog))
    assert h.max_occ == (cnt.max() if yet_np.nnz else 0)
    if yet_np.nnz == 0:
        return
    assert np.array_equal(read_dev(py, h.t_ids, yet_np.nnz, torch.int32), yet_np.ids)
    ent = read_dev(py, h.tr_ent, yet_np.nnz, torch.int32).astype(np.int64)
    key = np.repeat(np.arange(h.n_slices * yet_np.catalog, dtype=np.int64), np.diff(off))
    order = np.lexsort((ent, key))
    assert np.array_equal(key[order], key_ref)
    assert np.array_equal(ent[order], loc_ref)


@pytest.mark.parametrize("seed", range(4))
def test_tiny_random(ara, seed):
    w = synth.tiny_random(seed)
    check(ara, w.yet)


def test_many_ranges_ragged_and_empty_trials(ara):
    g = np.random.default_rng(11)
    lens = g.integers(0, 300, size=5000)
    lens[::7] = 0
    off = np.zeros(5001, np.int64)
    np.cumsum(lens, out=off[1:])
    ids = g.integers(0, 300_000, size=int(off[-1]), dtype=np.int32)
    ids[:40] = 299_999                     # last event of a ragged last range
    ids[40:90] = 7                         # one event many times in one trial
    check(ara, synth.Yet(300_000, off, ids))


def test_fewer_blocks_than_slices(ara):
    g = np.random.default_rng(3)
    off = np.array([0, 3, 3, 10], np.int64)
    ids = g.integers(0, 70_000, size=10, dtype=np.int32)
    check(ara, synth.Yet(70_000, off, ids))


def test_no_trials_and_no_occurrences(ara):
    check(ara, synth.Yet(1000, np.zeros(1, np.int64), np.zeros(0, np.int32)))
    check(ara, synth.Yet(1000, np.zeros(50, np.int64), np.zeros(0, np.int32)))


def test_config0_layout(ara):
    check(ara, synth.config(0, n_trials=20_000).yet)


def test_gap_and_edge_offset_codes(ara):
    """Trials with no event in a range between trials that have some (gap
    codes), events at offset 0x7FFF opening a trial (their advance cannot sit
    on the code), a trial of 300 events in one range (several 64-ID chunks)."""
    g = np.random.default_rng(17)
    trials = []
    for k in range(40_000):   # 10 trials per group, so gaps occur inside segments
        kind = k % 7
        if kind == 0:
            trials.append([])
        elif kind == 1:
            trials.append([32767, 32767 + 32768, 5])
        elif kind == 2:
            trials.append(list(g.integers(0, 100_000, size=300)))
        elif kind == 3:
            trials.append([32767] * 3 + [0])
        else:
            trials.append(list(g.integers(0, 100_000, size=int(g.integers(1, 6)))))
    off = np.zeros(len(trials) + 1, np.int64)
    np.cumsum([len(x) for x in trials], out=off[1:])
    ids = np.array([e for x in trials for e in x], np.int32)
    check(ara, synth.Yet(100_000, off, ids))


def test_forward_only_prepare_and_backward_refusal(ara):
    import torch
    w = synth.tiny_random(1)
    yet = ara.PreparedYet.from_numpy(w.yet, "cuda", transposed=False)
    assert yet.handle.n_slices == 0 and not yet.handle.tr_off
    assert not yet.handle.t_off and not yet.handle.t_ids and not yet.handle.t_cnt
    tables = ara.EltTables.from_numpy(w.elts, "cuda")
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")
    ylt, s_pre, _ = ara.ylt_forward(tables, yet, layers, et, lt, want_s_pre=True)
    cot = torch.ones((1,) + tuple(ylt.shape), dtype=torch.float64, device="cuda")
    with pytest.raises(ara.AraError, match="TRANSPOSED"):
        ara.ylt_backward(tables, yet, layers, et, lt, s_pre, cot)
