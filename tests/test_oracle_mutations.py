"""Planted mistakes: each mutant of the oracle source (a dropped term, a wrong
sign, a swapped operand, an off-by-one, a wrong loop direction) must fail at
least one of the pins.  The mutants are compiled on the CPU into a temporary
directory and never touch the real oracle library."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from _indep import brute_forward, brute_metrics, load_hand_example

MUTATIONS = {
    "dropped-scale": ("double scaled = s * x[d];", "double scaled = x[d];"),
    "dropped-elt-retention": ("l[d] = clamp_xl(scaled, R, L);", "l[d] = clamp_xl(scaled, 0.0, L);"),
    "swapped-occ-terms": ("lo[d] = clamp_xl(lo[d], OccR, OccL);", "lo[d] = clamp_xl(lo[d], OccL, OccR);"),
    "no-floor-at-zero": ("double a = (y > 0.0) ? y : 0.0;\n    return", "double a = y;\n    return"),
    "cumsum-wrong-sign": ("lo[d] = lo[d] + lo[d - 1];", "lo[d] = lo[d] - lo[d - 1];"),
    "difference-ascending": ("for (int64_t d = n - 1; d >= 1; --d) lo[d] = lo[d] - lo[d - 1];",
                             "for (int64_t d = 1; d < n; ++d) lo[d] = lo[d] - lo[d - 1];"),
    "swapped-agg-terms": ("lo[d] = clamp_xl(lo[d], AggR, AggL);", "lo[d] = clamp_xl(lo[d], AggL, AggR);"),
    "hits-count-all": ("h += (v != 0.0f);", "h += 1;"),
    "pml-off-by-one": ("out[3 * j + 1] = v[r - 1];", "out[3 * j + 1] = v[r < n ? r : r - 1];"),
    "tvar-wrong-denominator": ("out[3 * j + 2] = top / (double)r;", "out[3 * j + 2] = top / (double)n;"),
    "tail-count-ceil": ("int64_t r = n - (int64_t)floor(p * (double)n + 1e-9);",
                        "int64_t r = n - (int64_t)floor(p * (double)n + 1e-9) + 1;"),
    "grad-scale-missing-loss": ("ge[3 * k + 0] += adj_l * xk[(size_t)q * m + (size_t)d];",
                                "ge[3 * k + 0] += adj_l;"),
    "grad-aggr-sign": ("if (lin) gl[2] -= adj_f[d];", "if (lin) gl[2] += adj_f[d];"),
    "grad-occ-mask-ignored": ("const double adj_l = lin ? adj_o[d] : 0.0;", "const double adj_l = adj_o[d];"),
    "tvar-tie-weight": ("wt[t] = (double)(r - n_gt) / ((double)r * (double)n_eq);",
                        "wt[t] = 1.0 / ((double)r * (double)n_eq);"),
    "elt-limit-grad-dropped": ("if (av >= L) ge[3 * k + 2] += adj_l;", "if (av >= L) ge[3 * k + 2] += 0.0;"),
    "occ-limit-grad-dropped": ("if (aa >= OccL) gl[1] += adj_o[d];", "if (aa >= OccL) gl[1] += 0.0;"),
    "occ-max-is-last": ("m = (lo[d] > m) ? lo[d] : m;", "m = lo[d];"),
    "yelt-reversed-order": ("for (int64_t d = 0; d < n; ++d) yelt[base + (size_t)d] = lo[d];",
                            "for (int64_t d = 0; d < n; ++d) yelt[base + (size_t)d] = lo[n - 1 - d];"),
}


def _battery():
    """True iff every pin in this small battery holds."""
    w, g = load_hand_example()
    tb = oracle.build_tables(w.elts)
    r = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, want_yelt=True)
    if r["ylt"][0].tolist() != g["ylt"] or r["hits"][0].tolist() != g["hits"]:
        return False
    if r["yelt"][0].tolist() != [v for t in g["yelt"] for v in t] or r["occ_max"][0].tolist() != g["occ_max"]:
        return False
    for p, m in g["metrics"].items():
        if oracle.metrics(r["ylt"], float(p))[0].tolist() != [m["aal"], m["pml"], m["tvar"]]:
            return False
    wts = oracle.metric_weights(r["ylt"], g["grad_p"])
    ge, gl = oracle.backward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms, wts)
    for i, name in enumerate(["aal", "pml", "tvar"]):
        if not np.allclose(ge[i], g["grad"][name]["elt"], atol=1e-12):
            return False
        if not np.allclose(gl[i, 0], g["grad"][name]["layer"], atol=1e-12):
            return False
    for seed in range(4):
        wr = synth.tiny_random(seed, n_trials=25, n_layers=2)
        tbr = oracle.build_tables(wr.elts)
        rr = oracle.forward(tbr, wr.yet, wr.layers, wr.elts.terms, wr.layers.terms)
        Y, S, H = brute_forward(wr)
        if not np.array_equal(rr["hits"], H):
            return False
        if not np.all(np.abs(rr["ylt"] - Y) <= 1e-12 * np.maximum(Y, S) + 1e-300):
            return False
    # Euler's identity on random cases whose limits bind at the ELT level and
    # at the occurrence level respectively
    we = synth.tiny_random(2, n_trials=60, max_events=20, n_layers=1)
    tbe = oracle.build_tables(we.elts)
    for mode in ("elt", "occ"):
        et, lt = we.elts.terms.copy(), we.layers.terms.copy()
        if mode == "elt":
            et[:, 2] = 60.0
            lt[:, 0], lt[:, 1], lt[:, 2], lt[:, 3] = 10.0, 1e6, 10.0, 1e9
        else:
            lt[:, 0], lt[:, 1], lt[:, 2], lt[:, 3] = 10.0, 40.0, 10.0, 1e9
        re_ = oracle.forward(tbe, we.yet, we.layers, et, lt)
        me = oracle.metrics(re_["ylt"], we.p)[0]
        wte = oracle.metric_weights(re_["ylt"], we.p)
        gee, gle = oracle.backward(tbe, we.yet, we.layers, et, lt, wte)
        used = we.layers.elt_ids
        for c in range(3):
            tot = sum(et[k, col] * gee[c, k, col] for k in used for col in range(3))
            tot += sum(lt[0, col] * gle[c, 0, col] for col in range(4))
            if abs(tot - me[c]) > 1e-9 * (1 + abs(me[c])):
                return False
    # explicit ties at the threshold: r = 2, three trials tied at the PML
    yt = np.array([[5.0, 5.0, 5.0, 1.0]])
    wt = oracle.metric_weights(yt, 0.5)
    if not np.allclose(wt[2, 0], [1 / 3, 1 / 3, 1 / 3, 0.0]) or not np.allclose(wt[1, 0], [1 / 3, 1 / 3, 1 / 3, 0.0]):
        return False
    gen = np.random.default_rng(0)
    for _ in range(4):
        y = np.round(gen.exponential(50.0, size=int(gen.integers(3, 40))))
        aal, pml, tvar, _r = brute_metrics(y, 0.9)
        m = oracle.metrics(y[None, :], 0.9)[0]
        if m[1] != pml or abs(m[2] - tvar) > 1e-12 * tvar or abs(m[0] - aal) > 1e-12 * aal:
            return False
        # tie handling of the TVaR weight: weights sum to one and reproduce TVaR
        wv = oracle.metric_weights(y[None, :], 0.9)
        if abs(wv[2, 0].sum() - 1.0) > 1e-12 or abs((wv[2, 0] * y).sum() - m[2]) > 1e-9 * (1 + m[2]):
            return False
    return True


SU_MUTATIONS = {
    "su-philox-multiplier": ("(uint64_t)0xD2511F53u * c[0]", "(uint64_t)0xD2511F55u * c[0]"),
    "su-philox-key-bump": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    "su-philox-word-order": ("c[1] = lo1;\n        c[2] = n2;", "c[1] = n2;\n        c[2] = lo1;"),
    "su-no-half-variance": ("const double m = log(mu) - 0.5 * s2;", "const double m = log(mu);"),
    "su-sigma-not-relative": ("const double r = sigma / mu;", "const double r = sigma;"),
    "su-draw-ignores-elt": ("(uint32_t)((uint64_t)occ >> 32), (uint32_t)elt, 0};",
                            "(uint32_t)((uint64_t)occ >> 32), 0, 0};"),
    "su-sigma-zero-not-special": ("if (sigma == 0.0) return mu;", "if (sigma < 0.0) return mu;"),
    "su-lookup-not-drawn": ("? oracle_su_draw(mu, (double)sig[ev[d]], seed, offsets[b] + d, k) : 0.0;",
                            "? mu : 0.0;"),
    "su-same-uniform-twice": ("const double u2 = ((double)(b2 >> 12) + 0.5) * 0x1p-52;",
                              "const double u2 = ((double)(b1 >> 12) + 0.5) * 0x1p-52;"),
    "su-high-word-dropped": ("const uint64_t b1 = ((uint64_t)w[1] << 32) | w[0]", "const uint64_t b1 = (uint64_t)w[0]"),
}


def _battery_su():
    """True iff every pin of the secondary-uncertainty path holds (small
    versions of tests/test_oracle_su.py)."""
    for ctr, key, want in [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
                           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
                            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]:
        if oracle.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32)).tolist() != list(want):
            return False
    w = synth.tiny_random(1, n_trials=30, max_events=12, n_layers=2)
    tb = oracle.build_tables(w.elts)
    ref = oracle.forward(tb, w.yet, w.layers, w.elts.terms, w.layers.terms)
    su = oracle.forward_su(tb, np.zeros_like(tb), w.yet, w.layers, w.elts.terms, w.layers.terms, seed=4)
    if not np.array_equal(su["ylt"], ref["ylt"]):
        return False
    n = 20_000
    for mu, sg in [(100.0, 40.0), (5e5, 5e5)]:
        x = np.array([oracle.su_draw(mu, sg, 2024, i, 3) for i in range(n)])
        s2 = np.log1p((sg / mu) ** 2)
        if not np.all(np.isfinite(x)) or not np.all(x > 0):
            return False
        lx = np.log(x)
        if abs(lx.mean() - (np.log(mu) - s2 / 2)) > 6 * np.sqrt(s2 / n) or abs(lx.var() - s2) > 6 * s2 * np.sqrt(2 / n):
            return False
    za = np.log([oracle.su_draw(1.0, 0.5, 7, i, 0) for i in range(n)])
    zb = np.log([oracle.su_draw(1.0, 0.5, 7, i, 1) for i in range(n)])
    if abs(np.corrcoef(za, zb)[0, 1]) > 6 / np.sqrt(n):
        return False
    # linear terms: the year loss's spread is that of the draws
    cat, nt = 16, 4000
    elts = synth.Elts(cat, np.array([0, 2], np.int64), np.array([3, 9], np.int32),
                      np.array([1000.0, 400.0], np.float32), np.array([[1.0, 0.0, np.inf]]))
    layers = synth.Layers(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([[0.0, np.inf, 0.0, np.inf]]))
    yet = synth.Yet(cat, np.arange(nt + 1, dtype=np.int64) * 2, np.tile(np.array([3, 9], np.int32), nt))
    y = oracle.forward_su(oracle.build_tables(elts), oracle.build_sigma_tables(elts, np.array([300.0, 100.0], np.float32)),
                          yet, layers, elts.terms, layers.terms, seed=2)["ylt"][0]
    sd = np.hypot(300.0, 100.0)
    if abs(y.mean() - 1400.0) > 6 * sd / np.sqrt(nt) or abs(y.std() / sd - 1.0) > 0.15:
        return False
    return True


def test_real_oracle_passes_battery():
    assert _battery()
    assert _battery_su()


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory(prefix="ara_oracle_mut_") as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTATIONS) + sorted(SU_MUTATIONS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTATIONS[name] if name in MUTATIONS else SU_MUTATIONS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(workdir, f"{name}.c")
    path_so = os.path.join(workdir, f"lib{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", path_so, path_c, "-lm"])
    with oracle.use_library(path_so):
        caught = not (_battery() and _battery_su())
    assert caught, f"mutant {name} survived every pin"
