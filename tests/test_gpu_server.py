"""The continuous-batching quote server: results equal the stand-alone batch
entry points (alone and in a mix of concurrent quotes), match the oracle,
queue under memory pressure, and support cancellation of queued quotes."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-server] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2572_amd as ara
    ara.library()
    w = synth.config(4, n_trials=40_000)
    tables = ara.EltTables.from_numpy(w.elts)
    yet = ara.PreparedYet.from_numpy(w.yet)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    reqs = synth.serving_requests(24, w.yet.n_trials, n_elts=w.elts.n_elts, min_trials=2_000, max_trials=40_000)
    return ara, w, tables, yet, et, reqs


def direct(ara, tables, yet, et, r, p):
    import torch
    layers = ara.Layers(np.array([0, len(r.elt_ids)], np.int32), r.elt_ids)
    lt = torch.tensor(np.asarray(r.layer_terms)[None, :], dtype=torch.float64, device="cuda")
    y, s, _ = ara.ylt_forward(tables, yet, layers, et, lt, r.trial_begin, r.trial_end, want_s_pre=True)
    m, w = ara.metrics(y, p, want_weights=True)
    out = {"metrics": m.cpu().numpy()[0]}
    if r.want_grad:
        ge, gl = ara.ylt_backward(tables, yet, layers, et, lt, s, w, r.trial_begin, r.trial_end)
        out["grad_layer"] = gl.cpu().numpy()[:, 0, :]
        out["grad_elt"] = ge.cpu().numpy()[:, r.elt_ids, :]
    return out


def same(a, b):
    assert np.array_equal(a["metrics"], b["metrics"]), (a["metrics"], b["metrics"])
    if "grad_layer" in b:
        assert np.array_equal(a["grad_layer"], b["grad_layer"])
        assert np.array_equal(a["grad_elt"], b["grad_elt"])


def test_alone_and_in_mix_equal_direct_calls(env):
    ara, w, tables, yet, et, reqs = env
    srv = ara.QuoteServer(tables, yet, et, quotes_with_grad=6, max_slots=16)
    try:
        _say("mix: all quotes submitted at once")
        tickets = [srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, 0.99, r.want_grad) for r in reqs]
        mix = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["max_quotes_per_launch"] >= 2, st       # quotes really shared forward launches
        assert st["shared_block_items"] > 0, st           # and blocks: their codes read once per launch
        _say("alone: one quote at a time")
        alone = [srv.wait(srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, 0.99, r.want_grad))
                 for r in reqs]
    finally:
        srv.close()
    for r, a, m in zip(reqs, alone, mix):
        same(m, a)
        same(a, direct(ara, tables, yet, et, r, 0.99))


def test_quotes_finishing_together_equal_direct_calls(env):
    """Quotes admitted together whose trial ranges all end in the YET's last
    block finish after the same forward launch, and their metrics then run
    as rows of one set of launches: rows of different lengths (one block to
    the whole YET), tail probabilities and ranks, with and without weights.
    Every quote equals its direct calls bit for bit."""
    import dataclasses
    ara, w, tables, yet, et, reqs = env
    N = w.yet.n_trials
    starts = [0, 1, N // 3, N // 2 + 7, N - 2_500, N - 100, 3, N - 1, N // 4, 17, N - 40, N // 5]
    ps = [0.5, 0.9, 0.99, 0.995, 0.999, 0.99, 0.75, 0.99, 0.95, 0.999, 0.5, 0.99]
    qs = [dataclasses.replace(r, trial_begin=b, trial_end=N, want_grad=(i % 3 == 0))
          for i, (r, b) in enumerate(zip(reqs, starts))]
    srv = ara.QuoteServer(tables, yet, et, quotes_with_grad=4, max_slots=16)
    try:
        _say("12 quotes ending in the last block, submitted at once")
        tickets = [srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, p, r.want_grad)
                   for r, p in zip(qs, ps)]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    _say(f"stats {st}")
    assert st["max_finished_per_launch"] >= 2, st     # metrics rows really ran together
    for r, p, g in zip(qs, ps, got):
        same(g, direct(ara, tables, yet, et, r, p))


def test_results_survive_slot_reuse(env):
    """Two result slots, eight quotes, results collected last-first: every
    quote's result must be its own even after later quotes reused its slot."""
    ara, w, tables, yet, et, reqs = env
    srv = ara.QuoteServer(tables, yet, et, quotes_with_grad=6, max_slots=2)
    try:
        tickets = [srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, 0.99, r.want_grad)
                   for r in reqs[:8]]
        got = {t: srv.wait(t) for t in reversed(tickets)}
    finally:
        srv.close()
    for r, t in zip(reqs[:8], tickets):
        same(got[t], direct(ara, tables, yet, et, r, 0.99))


def test_quotes_match_oracle(env):
    ara, w, tables, yet, et, reqs = env
    tb = oracle.build_tables(w.elts)
    srv = ara.QuoteServer(tables, yet, et, quotes_with_grad=4, max_slots=8)
    try:
        for r in reqs[:4]:
            got = srv.wait(srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, 0.99, r.want_grad))
            layers = synth.Layers(np.array([0, len(r.elt_ids)], np.int32), r.elt_ids, np.asarray(r.layer_terms)[None, :])
            ref = oracle.forward(tb, w.yet, layers, w.elts.terms, layers.terms, r.trial_begin, r.trial_end, n_threads=8)
            np.testing.assert_allclose(got["metrics"], oracle.metrics(ref["ylt"], 0.99)[0], rtol=1e-9)
    finally:
        srv.close()


def test_memory_pressure_queues_and_cancel(env):
    ara, w, tables, yet, et, reqs = env
    import ctypes
    nb = ctypes.c_size_t()
    ara.library().ara_server_arena_bytes(ctypes.byref(tables.handle), ctypes.byref(yet.handle), 1, ctypes.byref(nb))
    srv = ara.QuoteServer(tables, yet, et, arena_bytes=nb.value, max_slots=4)   # room for one gradient quote
    try:
        g = [r for r in reqs if r.want_grad][:3]
        tickets = [srv.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, 0.99, True) for r in g]
        extra = srv.submit(g[0].elt_ids, g[0].layer_terms, g[0].trial_begin, g[0].trial_end, 0.99, True)
        cancelled = srv.cancel(extra)
        res = [srv.wait(t) for t in tickets]
        for r, x in zip(g, res):
            same(x, direct(ara, tables, yet, et, r, 0.99))
        if cancelled:
            with pytest.raises(ara.AraError):
                srv.wait(extra)
        else:
            srv.wait(extra)
    finally:
        srv.close()


def test_invalid_resident_terms_refused_at_create(env):
    ara, w, tables, yet, et, reqs = env
    bad = et.clone()
    bad[3, 2] = 0.0                       # a limit of zero
    with pytest.raises(ara.AraError) as ex:
        ara.QuoteServer(tables, yet, bad, quotes_with_grad=1, max_slots=2)
    assert ex.value.status == 1


def test_submit_validation(env):
    ara, w, tables, yet, et, reqs = env
    srv = ara.QuoteServer(tables, yet, et, quotes_with_grad=1, max_slots=2)
    try:
        with pytest.raises(ara.AraError) as ex:
            srv.submit([0, w.elts.n_elts], [1e4, 1e6, 1e5, 1e7], 0, 100)
        assert ex.value.status == 2
        with pytest.raises(ara.AraError):
            srv.submit([0, 1], [1e4, 1e6, 1e5, 1e7], 10, 10)
        with pytest.raises(ara.AraError):
            srv.submit([0, 1], [-1.0, 1e6, 1e5, 1e7], 0, 10)
    finally:
        srv.close()
