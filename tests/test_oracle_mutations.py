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


def test_real_oracle_passes_battery():
    assert _battery()


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory(prefix="ara_oracle_mut_") as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTATIONS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(workdir, f"{name}.c")
    path_so = os.path.join(workdir, f"lib{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", path_so, path_c, "-lm"])
    with oracle.use_library(path_so):
        caught = not _battery()
    assert caught, f"mutant {name} survived every pin"
