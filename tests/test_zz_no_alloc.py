"""ara_ylt_forward_noalloc, the forward whose workspace is the library's own
per-device scratch, against ara_ylt_forward with a caller workspace: the
same kernels, so the results must be identical bit for bit.  Two calls in a
row, the second on a smaller input (the scratch keeps the first call's
contents), a call over part of the trials, a device-side term error
reported through the status word and cleared by the next call, and a call
needing more than the scratch refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ara():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    return ara


def _inputs(ara, w):
    import torch
    tables = ara.EltTables.from_numpy(w.elts)
    yet = ara.PreparedYet.from_numpy(w.yet, transposed=False, trial_major=False)
    layers = ara.Layers(w.layers.elt_off, w.layers.elt_ids)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    lt = torch.tensor(w.layers.terms, dtype=torch.float64, device="cuda")
    return tables, yet, layers, et, lt


def _compare(ara, w, hits, t0=0, t1=None):
    import torch
    tables, yet, layers, et, lt = _inputs(ara, w)
    t1 = w.yet.n_trials if t1 is None else t1
    L, n = w.layers.n_layers, t1 - t0
    y, s, h = ara.ylt_forward(tables, yet, layers, et, lt, t0, t1, want_s_pre=True, want_hits=hits, check=True)
    y2 = torch.full((L, n), -1.0, dtype=torch.float64, device="cuda")
    s2 = torch.full((L, n), -1.0, dtype=torch.float64, device="cuda")
    h2 = torch.full((L, n), -1, dtype=torch.int32, device="cuda") if hits else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ara.ylt_forward_noalloc(tables, yet, layers, et, lt, y2, s2, h2, st, t0, t1)
    torch.cuda.synchronize()
    assert st.item() == 0
    assert torch.equal(y, y2) and torch.equal(s, s2)
    if hits:
        assert torch.equal(h, h2)
    return y2.cpu().numpy(), s2.cpu().numpy()


def test_noalloc_equals_workspace_forward(ara):
    print("[no-alloc] 20k trials x Poisson(1000), 4 layers, hit counts", flush=True)
    _compare(ara, synth.config(2, n_trials=20_000), hits=True)
    print("[no-alloc] then 3000 trials x 1000, one layer, 200k catalogue", flush=True)
    w = synth.config(0, n_trials=3000)
    y, s = _compare(ara, w, hits=False)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, n_threads=8)
    assert np.all(np.abs(y - ref["ylt"]) <= 1e-9 * np.maximum(ref["ylt"], ref["s_pre"]))
    print("[no-alloc] part of the trials", flush=True)
    _compare(ara, w, hits=True, t0=777, t1=2100)


def test_noalloc_status_word(ara):
    import torch
    w = synth.tiny_random(4, n_trials=50, n_layers=2)
    tables, yet, layers, et, lt = _inputs(ara, w)
    L, n = w.layers.n_layers, w.yet.n_trials
    y = torch.empty((L, n), dtype=torch.float64, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    bad = et.clone()
    bad[int(w.layers.elt_ids[0]), 0] = float("nan")      # an ELT of the first layer
    ara.ylt_forward_noalloc(tables, yet, layers, bad, lt, y, status=st)
    lib = ara.library()
    assert lib.ara_check_device_error(ara._dptr(st), ara._stream()) == ara.ARA_E_INVAL
    ara.ylt_forward_noalloc(tables, yet, layers, et, lt, y, status=st)
    assert lib.ara_check_device_error(ara._dptr(st), ara._stream()) == 0
    # no layers: nothing to compute, the status still written
    none = ara.Layers([0], [])
    st.fill_(-1)
    ara.ylt_forward_noalloc(tables, yet, none, et, lt, y[:0], status=st)
    torch.cuda.synchronize()
    assert st.item() == 0


def test_noalloc_refuses_beyond_the_scratch(ara):
    """A 2^26-event catalogue with one layer needs about 1 GiB of workspace:
    refused with ARA_E_LIMIT from the host-side checks (no device work)."""
    lib = ara.library()
    cat = 1 << 26
    tables = ara.ara_tables(n_elts=1, catalog=cat, words=cat // 32)
    yet = ara.ara_yet(n_trials=1000, catalog=cat, range_bits=15, groups=16, trials_per_group=8,
                      trials_per_block=128, n_blocks=8, n_ranges=2048)
    lay = ara.Layers([0, 1], [0])
    nb = ctypes.c_size_t()
    assert lib.ara_ylt_workspace_bytes(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), 0,
                                       ctypes.byref(nb)) == 0
    assert nb.value > (160 << 20)
    p = ctypes.c_void_p(256)
    assert lib.ara_ylt_forward_noalloc(ctypes.byref(tables), ctypes.byref(yet), ctypes.byref(lay.handle), p, p, 0, 10,
                                       0, p, None, None, None, None) == ara.ARA_E_LIMIT
    assert b"no-allocation scratch" in lib.ara_last_error()
