"""Independent formulations used to pin the oracle (pure Python / numpy).

These are deliberately written along a different route from the oracle's
literal loops: ELTs as Python dicts, the year loss through the telescoped
closed form f_agg(sum of occurrence losses), metrics through counting
definitions.  Test code only.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def xl(v: float, r: float, lim: float) -> float:
    """Excess-of-loss layer: the part of v above r, capped at lim."""
    return min(max(v - r, 0.0), lim)


def load_hand_example():
    with open(os.path.join(GOLDEN, "hand_example.json")) as f:
        g = json.load(f)
    catalog = g["catalog"]
    rec_off = [0]
    rec_ids, rec_loss, terms = [], [], []
    for e in g["elts"]:
        for k, v in e["records"].items():
            rec_ids.append(int(k))
            rec_loss.append(float(v))
        rec_off.append(len(rec_ids))
        terms.append([float(x) for x in e["terms"]])
    elts = synth.Elts(catalog, np.array(rec_off, np.int64), np.array(rec_ids, np.int32),
                      np.array(rec_loss, np.float32), np.array(terms, np.float64))
    trials = g["trials"]
    offsets = np.zeros(len(trials) + 1, np.int64)
    np.cumsum([len(t) for t in trials], out=offsets[1:])
    ids = np.array([e for t in trials for e in t], np.int32)
    lay = g["layer"]
    layers = synth.Layers(np.array([0, len(lay["elts"])], np.int32), np.array(lay["elts"], np.int32),
                          np.array([lay["terms"]], np.float64))
    w = synth.Workload("hand-example", synth.Yet(catalog, offsets, ids), elts, layers, 0.6)
    return w, g


def elt_dicts(elts):
    out = []
    for k in range(elts.n_elts):
        a, b = int(elts.rec_off[k]), int(elts.rec_off[k + 1])
        out.append({int(i): float(l) for i, l in zip(elts.rec_ids[a:b], elts.rec_loss[a:b])})
    return out


def brute_forward(w, elt_terms=None, layer_terms=None):
    """Year losses via the closed form, S and hits, all in Python floats."""
    dicts = elt_dicts(w.elts)
    et = w.elts.terms if elt_terms is None else elt_terms
    lt = w.layers.terms if layer_terms is None else layer_terms
    nl, nt = w.layers.n_layers, w.yet.n_trials
    Y = np.zeros((nl, nt))
    S = np.zeros((nl, nt))
    H = np.zeros((nl, nt), np.int64)
    for j in range(nl):
        lst = [int(k) for k in w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]]]
        occr, occl, aggr, aggl = (float(v) for v in lt[j])
        for t in range(nt):
            s = 0.0
            h = 0
            for e in w.yet.ids[w.yet.offsets[t]:w.yet.offsets[t + 1]]:
                x = 0.0
                for k in lst:
                    loss = dicts[k].get(int(e), 0.0)
                    if loss != 0.0:
                        h += 1
                    x += xl(et[k][0] * loss, et[k][1], et[k][2])
                s += xl(x, occr, occl)
            S[j, t] = s
            Y[j, t] = xl(s, aggr, aggl)
            H[j, t] = h
    return Y, S, H


def brute_metrics(y, p):
    """Counting definitions: PML is the v with #{Y > v} < r <= #{Y >= v};
    TVaR = (sum of Y above v + (r - #{Y > v}) * v) / r."""
    y = [float(v) for v in y]
    n = len(y)
    r = n - math.floor(p * n + 1e-9)
    r = max(1, min(n, r))
    pml = None
    for v in y:
        gt = sum(1 for u in y if u > v)
        ge = sum(1 for u in y if u >= v)
        if gt < r <= ge:
            pml = v
            break
    gt = [u for u in y if u > pml]
    tvar = (math.fsum(gt) + (r - len(gt)) * pml) / r
    return math.fsum(y) / n, pml, tvar, r


def brute_yelt(w, elt_terms=None, layer_terms=None):
    """Per-occurrence losses as increments of f_agg over correctly rounded
    running totals (math.fsum of the occurrence losses so far): a different
    route from a running sum.  Returns (list per layer of per-occurrence
    arrays in storage order, per-trial maxima [n_layers, n_trials])."""
    dicts = elt_dicts(w.elts)
    et = w.elts.terms if elt_terms is None else elt_terms
    lt = w.layers.terms if layer_terms is None else layer_terms
    nl, nt = w.layers.n_layers, w.yet.n_trials
    out = []
    mx = np.zeros((nl, nt))
    for j in range(nl):
        lst = [int(k) for k in w.layers.elt_ids[w.layers.elt_off[j]:w.layers.elt_off[j + 1]]]
        occr, occl, aggr, aggl = (float(v) for v in lt[j])
        row = []
        for t in range(nt):
            occ = []
            for e in w.yet.ids[w.yet.offsets[t]:w.yet.offsets[t + 1]]:
                x = 0.0
                for k in lst:
                    x += xl(et[k][0] * dicts[k].get(int(e), 0.0), et[k][1], et[k][2])
                occ.append(xl(x, occr, occl))
            prev = 0.0
            incs = []
            for d in range(len(occ)):
                c = xl(math.fsum(occ[: d + 1]), aggr, aggl)
                incs.append(c - prev)
                prev = c
            row.extend(incs)
            mx[j, t] = max(incs) if incs else 0.0
        out.append(np.array(row))
    return out, mx
