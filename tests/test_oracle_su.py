"""Pins of the oracle's secondary-uncertainty path (readings R10, R11): the
Philox4x32-10 block against the generator's published known-answer vectors,
sigma = 0 against the deterministic path bit for bit, and the moments and
independence of the draws.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from _indep import load_hand_example


# The known-answer vectors published with the generator (Salmon, Moraes,
# Dror and Shaw, SC'11): counter, key, output block.
_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", _KAT)
def test_philox_known_answers(ctr, key, want):
    assert oracle.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32)).tolist() == list(want)


def _sigma_elts(w, frac_zero=1.0, seed=5):
    sg = synth.record_sigmas(seed, w.elts, zero_frac=frac_zero)
    return oracle.build_sigma_tables(w.elts, sg), sg


@pytest.mark.parametrize("seed", range(6))
def test_sigma_zero_is_the_deterministic_path(seed):
    w = synth.tiny_random(seed, n_trials=40, max_events=15, n_layers=2)
    tb = oracle.build_tables(w.elts)
    st, _ = _sigma_elts(w, frac_zero=1.0)
    assert not st.any()
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms)
    su = oracle.forward_su(tb, st, w.yet, w.layers, w.elts.terms, w.layers.terms, seed=99)
    assert np.array_equal(su["ylt"], ref["ylt"]) and np.array_equal(su["s_pre"], ref["s_pre"])


def test_sigma_zero_hand_example_and_config0_prefix():
    w, g = load_hand_example()
    tb = oracle.build_tables(w.elts)
    su = oracle.forward_su(tb, np.zeros_like(tb), w.yet, w.layers, w.elts.terms, w.layers.terms, seed=1)
    assert su["ylt"][0].tolist() == g["ylt"]
    w0 = synth.config(0, n_trials=300)
    tb0 = oracle.build_tables(w0.elts)
    ref = oracle.forward(tb0, w0.yet, w0.layers, w0.elts.terms, w0.layers.terms)
    su0 = oracle.forward_su(tb0, np.zeros_like(tb0), w0.yet, w0.layers, w0.elts.terms, w0.layers.terms, seed=3)
    assert np.array_equal(su0["ylt"], ref["ylt"])


@pytest.mark.parametrize("mu,sigma", [(100.0, 40.0), (5e5, 5e5), (2.5e4, 3.75e4)])
def test_draw_moments(mu, sigma):
    """Over 60,000 occurrences the draws have mean mu and standard deviation
    sigma, and their logarithms mean m = ln mu - s^2/2 and variance
    s^2 = ln(1 + sigma^2/mu^2) (each within six standard errors)."""
    n = 60_000
    x = np.array([oracle.su_draw(mu, sigma, 2024, i, 3) for i in range(n)])
    assert np.all(x > 0)
    s2 = np.log1p((sigma / mu) ** 2)
    m = np.log(mu) - s2 / 2
    lx = np.log(x)
    assert abs(lx.mean() - m) <= 6 * np.sqrt(s2 / n)
    assert abs(lx.var() - s2) <= 6 * s2 * np.sqrt(2.0 / n)
    assert abs(x.mean() - mu) <= 6 * sigma / np.sqrt(n)
    # the spread of the sample standard deviation of a lognormal is wide:
    # 10% is many standard errors at these sizes
    assert abs(x.std() / sigma - 1.0) < 0.1


def test_draws_independent_across_occurrences_elts_and_seeds():
    n = 20_000
    z = {}
    for key in [(7, 0), (7, 1), (8, 0)]:
        seed, k = key
        x = np.array([oracle.su_draw(1.0, 0.5, seed, i, k) for i in range(n)])
        z[key] = np.log(x)
    lim = 6 / np.sqrt(n)
    for a, b in [((7, 0), (7, 1)), ((7, 0), (8, 0))]:
        assert abs(np.corrcoef(z[a], z[b])[0, 1]) < lim
    za = z[(7, 0)]
    assert abs(np.corrcoef(za[:-1], za[1:])[0, 1]) < lim   # consecutive occurrences


def test_draw_is_the_same_in_every_layer():
    """Two layers over the same ELT with the same terms see the same draws."""
    w = synth.tiny_random(3, n_trials=30, max_events=12, n_layers=1)
    k = int(w.layers.elt_ids[0])
    layers = synth.Layers(np.array([0, 1, 2], np.int32), np.array([k, k], np.int32),
                          np.vstack([w.layers.terms[0], w.layers.terms[0]]))
    tb = oracle.build_tables(w.elts)
    st, _ = _sigma_elts(w, frac_zero=0.0)
    su = oracle.forward_su(tb, st, w.yet, layers, w.elts.terms, layers.terms, seed=11)
    assert np.array_equal(su["ylt"][0], su["ylt"][1])


def test_mean_year_loss_matches_the_deterministic_path_when_terms_are_linear():
    """With no retention and no limit anywhere, the year loss is linear in
    the draws, so its mean over many trials holding the same events equals
    the deterministic year loss (mean draw = mu), within six standard errors."""
    cat = 64
    n = 20_000
    offsets = np.arange(n + 1, dtype=np.int64) * 3
    ids = np.tile(np.array([5, 17, 40], np.int32), n)
    rec_off = np.array([0, 3, 5], np.int64)
    rec_ids = np.array([5, 17, 40, 17, 63], np.int32)
    rec_loss = np.array([1000.0, 250.0, 4000.0, 800.0, 1.0], np.float32)
    rec_sigma = np.array([500.0, 0.0, 4000.0, 1200.0, 1.0], np.float32)
    elts = synth.Elts(cat, rec_off, rec_ids, rec_loss, np.array([[1.0, 0.0, np.inf], [2.0, 0.0, np.inf]]))
    layers = synth.Layers(np.array([0, 2], np.int32), np.array([0, 1], np.int32),
                          np.array([[0.0, np.inf, 0.0, np.inf]]))
    yet = synth.Yet(cat, offsets, ids)
    tb = oracle.build_tables(elts)
    st = oracle.build_sigma_tables(elts, rec_sigma)
    det = oracle.forward(tb, yet, layers, elts.terms, layers.terms)["ylt"][0, 0]
    assert det == 1000.0 + 250.0 + 4000.0 + 2 * 800.0
    y = oracle.forward_su(tb, st, yet, layers, elts.terms, layers.terms, seed=5, n_threads=4)["ylt"][0]
    sd = np.sqrt(500.0 ** 2 + 4000.0 ** 2 + (2 * 1200.0) ** 2)
    assert abs(y.mean() - det) <= 6 * sd / np.sqrt(n)
    assert abs(y.std() / sd - 1.0) < 0.1
