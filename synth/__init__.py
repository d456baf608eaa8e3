"""Seeded synthetic inputs for aggregate risk analysis.

This module only draws random inputs and holds them in plain containers; it
contains none of the method's arithmetic (no lookups, terms, sums or metrics).
Both the HIP path's tests/benchmark and the CPU oracle take their inputs from
here, so the two sides see bit-identical data.

Shapes follow the paper's statement of the inputs (Section II): a Year Event
Table of trials, each a time-ordered sequence of (event ID, timestamp) pairs;
Event Loss Tables holding (event ID, loss) records plus per-ELT financial
terms; layers holding an ordered ELT list plus occurrence and aggregate terms.

Random streams: numpy's counter-based Philox bit generator keyed by
(seed, stream id), drawn sequentially, so the first n trials of a workload do
not depend on how many trials were generated in total.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 1308257200

# stream ids (the second Philox key word) for the independent draws
_S_LEN, _S_IDS, _S_TS, _S_ELT, _S_TERMS, _S_REQ, _S_SIGMA = 1, 2, 3, 4, 5, 6, 7


def _rng(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    key = (int(seed) & 0xFFFFFFFFFFFFFFFF) ^ ((stream * 0x9E3779B97F4A7C15 + sub) & 0xFFFFFFFFFFFFFFFF)
    return np.random.Generator(np.random.Philox(key=key))


@dataclass
class Yet:
    """Year Event Table in CSR form: trial t is ids[offsets[t]:offsets[t+1]]."""
    catalog: int
    offsets: np.ndarray            # int64 [n_trials + 1]
    ids: np.ndarray                # int32 [nnz]
    ts: Optional[np.ndarray] = None  # float32 [nnz], ascending within a trial

    @property
    def n_trials(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])


@dataclass
class Elts:
    """Event Loss Tables in CSR form: ELT k is records rec_off[k]:rec_off[k+1]."""
    catalog: int
    rec_off: np.ndarray            # int64 [n_elts + 1]
    rec_ids: np.ndarray            # int32 [n_records]
    rec_loss: np.ndarray           # float32 [n_records]
    terms: np.ndarray              # float64 [n_elts, 3] = (scale, retention, limit)

    @property
    def n_elts(self) -> int:
        return int(self.rec_off.shape[0] - 1)


@dataclass
class Layers:
    """Layers: ordered ELT lists (CSR) plus (OccR, OccL, AggR, AggL) each."""
    elt_off: np.ndarray            # int32 [n_layers + 1]
    elt_ids: np.ndarray            # int32 [sum of ELT counts]
    terms: np.ndarray              # float64 [n_layers, 4]

    @property
    def n_layers(self) -> int:
        return int(self.elt_off.shape[0] - 1)


@dataclass
class Workload:
    name: str
    yet: Yet
    elts: Elts
    layers: Layers
    p: float = 0.99
    notes: str = ""


@dataclass
class Request:
    """One pricing quote for the serving workload."""
    arrival_s: float
    elt_ids: np.ndarray            # int32 [J], indices into the resident ELT set
    layer_terms: np.ndarray        # float64 [4]
    trial_begin: int
    trial_end: int
    want_grad: bool


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

TRIAL_CHUNK = 16384   # trials per independently keyed ID stream


def _uniform_ids(seed: int, offsets: np.ndarray, catalog: int) -> np.ndarray:
    """i.i.d. uniform IDs; chunk c of TRIAL_CHUNK trials draws from its own
    Philox key, so chunks are generated in parallel and any prefix of trials
    is identical whatever the total."""
    n_trials = offsets.shape[0] - 1
    ids = np.empty(int(offsets[-1]), dtype=np.int32)
    chunks = range((n_trials + TRIAL_CHUNK - 1) // TRIAL_CHUNK)

    def fill(c):
        a = int(offsets[c * TRIAL_CHUNK])
        b = int(offsets[min((c + 1) * TRIAL_CHUNK, n_trials)])
        ids[a:b] = _rng(seed, _S_IDS, c).integers(0, catalog, size=b - a, dtype=np.int32)

    if len(chunks) <= 1:
        for c in chunks:
            fill(c)
    else:
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(fill, chunks))
    return ids


def fixed_length_yet(seed: int, n_trials: int, n_events: int, catalog: int,
                     with_ts: bool = False) -> Yet:
    """n_trials trials of exactly n_events i.i.d. uniform event IDs."""
    offsets = np.arange(n_trials + 1, dtype=np.int64) * n_events
    ids = _uniform_ids(seed, offsets, catalog)
    ts = _timestamps(seed, offsets) if with_ts else None
    return Yet(catalog, offsets, ids, ts)


def poisson_yet(seed: int, n_trials: int, mean_events: float, catalog: int,
                with_ts: bool = False) -> Yet:
    """Trials with Poisson(mean_events) event counts, uniform event IDs."""
    lens = _rng(seed, _S_LEN).poisson(mean_events, size=n_trials).astype(np.int64)
    offsets = np.zeros(n_trials + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    ids = _uniform_ids(seed, offsets, catalog)
    ts = _timestamps(seed, offsets) if with_ts else None
    return Yet(catalog, offsets, ids, ts)


def _timestamps(seed: int, offsets: np.ndarray) -> np.ndarray:
    """float32 U[0, 365) sorted ascending within each trial."""
    nnz = int(offsets[-1])
    ts = (_rng(seed, _S_TS).random(nnz, dtype=np.float32) * np.float32(365.0)).astype(np.float32)
    lens = np.diff(offsets)
    if nnz and np.all(lens == lens[0]):
        ts = np.sort(ts.reshape(-1, int(lens[0])), axis=1).reshape(-1)
    else:
        trial = np.repeat(np.arange(lens.shape[0], dtype=np.int64), lens)
        order = np.lexsort((ts, trial))
        ts = ts[order]
    return np.ascontiguousarray(ts, dtype=np.float32)


def lognormal_elts(seed: int, sizes: Sequence[int], catalog: int, mu: float = 12.0,
                   sigma: float = 1.5, scale: float = 1.0, retention: float = 5e4,
                   limit: float = 5e6) -> Elts:
    """ELTs of the given sizes: distinct IDs drawn without replacement, binary32
    losses exp(mu + sigma*Z) rounded to float32, identical per-ELT terms."""
    n = len(sizes)
    rec_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=rec_off[1:])
    rec_ids = np.empty(int(rec_off[-1]), dtype=np.int32)
    rec_loss = np.empty(int(rec_off[-1]), dtype=np.float32)
    for k, sz in enumerate(sizes):
        g = _rng(seed, _S_ELT, k)
        rec_ids[rec_off[k]:rec_off[k + 1]] = g.choice(catalog, size=int(sz), replace=False).astype(np.int32)
        rec_loss[rec_off[k]:rec_off[k + 1]] = g.lognormal(mu, sigma, size=int(sz)).astype(np.float32)
    terms = np.tile(np.array([scale, retention, limit], dtype=np.float64), (n, 1))
    return Elts(catalog, rec_off, rec_ids, rec_loss, terms)


def record_sigmas(seed: int, elts: Elts, cv_lo: float = 0.25, cv_hi: float = 1.5,
                  zero_frac: float = 0.1) -> np.ndarray:
    """Standard deviations of the ELT records for secondary uncertainty:
    sigma = cv * loss with cv ~ U[cv_lo, cv_hi] per record, and a fraction
    zero_frac of the records with sigma = 0 (no uncertainty), binary32."""
    out = np.empty(elts.rec_loss.shape[0], dtype=np.float32)
    for k in range(elts.n_elts):
        a, b = int(elts.rec_off[k]), int(elts.rec_off[k + 1])
        g = _rng(seed, _S_SIGMA, k)
        cv = g.uniform(cv_lo, cv_hi, size=b - a)
        cv[g.random(b - a) < zero_frac] = 0.0
        out[a:b] = (cv * elts.rec_loss[a:b].astype(np.float64)).astype(np.float32)
    return out


def log_uniform(g: np.random.Generator, lo: float, hi: float, size=None):
    return np.exp(g.uniform(np.log(lo), np.log(hi), size=size))


def random_layer_terms(g: np.random.Generator, n: int) -> np.ndarray:
    """Occurrence retention 1e4-1e6, occurrence limit 1e6-1e8, aggregate
    retention 1e5-1e7, aggregate limit 1e7-1e9, all log-uniform."""
    t = np.empty((n, 4), dtype=np.float64)
    t[:, 0] = log_uniform(g, 1e4, 1e6, n)
    t[:, 1] = log_uniform(g, 1e6, 1e8, n)
    t[:, 2] = log_uniform(g, 1e5, 1e7, n)
    t[:, 3] = log_uniform(g, 1e7, 1e9, n)
    return t


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

CONFIG_TERMS_LAYER = np.array([1e5, 2e7, 1e6, 1e8], dtype=np.float64)


def config(i: int, n_trials: Optional[int] = None, with_ts: bool = False) -> Workload:
    """Workloads 0-4.  n_trials (optional) keeps only the first n trials
    (identical to those of the full workload)."""
    seed = SEED_BASE + i
    if i == 0:
        N = 10_000 if n_trials is None else n_trials
        yet = fixed_length_yet(seed, N, 1000, 200_000, with_ts)
        elts = lognormal_elts(seed, [10_000] * 15, 200_000)
        layers = Layers(np.array([0, 15], np.int32), np.arange(15, dtype=np.int32),
                        CONFIG_TERMS_LAYER[None, :].copy())
        return Workload("tiny-10k-x1000-15elt", yet, elts, layers, 0.99)
    if i in (1, 3):
        N = 1_000_000 if n_trials is None else n_trials
        yet = fixed_length_yet(SEED_BASE + 1, N, 1000, 2_000_000, with_ts)
        elts = lognormal_elts(SEED_BASE + 1, [20_000] * 15, 2_000_000)
        layers = Layers(np.array([0, 15], np.int32), np.arange(15, dtype=np.int32),
                        CONFIG_TERMS_LAYER[None, :].copy())
        if i == 1:
            return Workload("paper-1Mx1000-15elt", yet, elts, layers, 0.99)
        # differentiated: scales 1.0, terms perturbed by U[0.97, 1.03]
        g = _rng(seed, _S_TERMS)
        elts.terms = elts.terms.copy()
        elts.terms[:, 1] *= g.uniform(0.97, 1.03, size=15)
        elts.terms[:, 2] *= g.uniform(0.97, 1.03, size=15)
        layers.terms = layers.terms * g.uniform(0.97, 1.03, size=(1, 4))
        return Workload("differentiated-1Mx1000-15elt", yet, elts, layers, 0.99)
    if i == 2:
        N = 1_000_000 if n_trials is None else n_trials
        yet = poisson_yet(seed, N, 1000.0, 2_000_000, with_ts)
        g = _rng(seed, _S_TERMS)
        sizes = g.integers(5_000, 30_001, size=55)
        elts = lognormal_elts(seed, list(sizes), 2_000_000)
        counts = [8, 12, 15, 20]
        elt_off = np.zeros(5, np.int32)
        np.cumsum(counts, out=elt_off[1:])
        layers = Layers(elt_off, np.arange(55, dtype=np.int32), random_layer_terms(g, 4))
        return Workload("uneven-1Mxpoisson1000-4layers", yet, elts, layers, 0.99)
    if i == 4:
        N = 1_000_000 if n_trials is None else n_trials
        yet = poisson_yet(seed, N, 1000.0, 2_000_000, with_ts)
        g = _rng(seed, _S_TERMS)
        sizes = g.integers(10_000, 30_001, size=200)
        elts = lognormal_elts(seed, list(sizes), 2_000_000)
        layers = Layers(np.array([0, 0], np.int32), np.zeros(0, np.int32),
                        np.zeros((1, 4), np.float64))
        return Workload("serving-1Mxpoisson1000-200elt", yet, elts, layers, 0.99)
    raise ValueError(f"no workload {i}")


def serving_requests(n_requests: int, n_trials: int, n_elts: int = 200, rate_per_s: float = 50.0,
                     seed: int = SEED_BASE + 4, min_trials: int = 100_000,
                     max_trials: int = 1_000_000) -> List[Request]:
    """Poisson arrivals; each request a layer of 5-25 distinct resident ELTs,
    log-uniform layer terms, a contiguous trial range, half asking for grads."""
    g = _rng(seed, _S_REQ)
    t = 0.0
    out: List[Request] = []
    hi = min(max_trials, n_trials)
    lo = min(min_trials, hi)
    for _ in range(n_requests):
        t += g.exponential(1.0 / rate_per_s)
        J = int(g.integers(5, 26))
        elts = g.choice(n_elts, size=J, replace=False).astype(np.int32)
        terms = random_layer_terms(g, 1)[0]
        n = int(g.integers(lo, hi + 1))
        b = int(g.integers(0, n_trials - n + 1))
        out.append(Request(t, elts, terms, b, b + n, bool(g.random() < 0.5)))
    return out


def tiny_random(seed: int, n_trials: int = 20, max_events: int = 12, catalog: int = 48,
                n_elts: int = 4, max_records: int = 20, n_layers: int = 2,
                zero_terms: bool = False, integer_losses: bool = False) -> Workload:
    """Small random case for brute force: mixed trial lengths (including empty
    trials), repeated events, small ELTs, layers over random ELT subsets."""
    g = _rng(seed, 99)
    lens = g.integers(0, max_events + 1, size=n_trials).astype(np.int64)
    offsets = np.zeros(n_trials + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    ids = g.integers(0, catalog, size=int(offsets[-1]), dtype=np.int32)
    sizes = g.integers(1, min(max_records, catalog) + 1, size=n_elts)
    rec_off = np.zeros(n_elts + 1, np.int64)
    np.cumsum(sizes, out=rec_off[1:])
    rec_ids = np.concatenate([g.choice(catalog, size=int(s), replace=False) for s in sizes]).astype(np.int32)
    if integer_losses:
        rec_loss = g.integers(1, 1000, size=int(rec_off[-1])).astype(np.float32)
    else:
        rec_loss = g.lognormal(5.0, 1.0, size=int(rec_off[-1])).astype(np.float32)
    if zero_terms:
        et = np.column_stack([g.uniform(0.5, 2.0, n_elts), np.zeros(n_elts), np.full(n_elts, np.inf)])
    else:
        et = np.column_stack([g.uniform(0.5, 2.0, n_elts), g.uniform(0.0, 100.0, n_elts),
                              g.uniform(100.0, 2000.0, n_elts)])
    elts = Elts(catalog, rec_off, rec_ids, rec_loss.astype(np.float32), et.astype(np.float64))
    elt_lists = []
    for _ in range(n_layers):
        J = int(g.integers(1, n_elts + 1))
        elt_lists.append(g.choice(n_elts, size=J, replace=False).astype(np.int32))
    elt_off = np.zeros(n_layers + 1, np.int32)
    np.cumsum([len(e) for e in elt_lists], out=elt_off[1:])
    if zero_terms:
        lt = np.tile(np.array([0.0, np.inf, 0.0, np.inf]), (n_layers, 1))
    else:
        lt = np.column_stack([g.uniform(0, 200, n_layers), g.uniform(200, 3000, n_layers),
                              g.uniform(0, 1500, n_layers), g.uniform(1000, 20000, n_layers)])
    layers = Layers(elt_off, np.concatenate(elt_lists).astype(np.int32), lt.astype(np.float64))
    return Workload(f"tiny-random-{seed}", Yet(catalog, offsets, ids, None), elts, layers, 0.8)


def hand_example() -> Workload:
    """Hand-worked example: catalogue of 8 events, two ELTs, one layer, five
    trials (one empty, one with a repeated event)."""
    catalog = 8
    rec_off = np.array([0, 3, 6], np.int64)
    rec_ids = np.array([1, 3, 5, 3, 5, 6], np.int32)
    rec_loss = np.array([100, 50, 300, 70, 10, 500], np.float32)
    terms = np.array([[1.0, 20.0, 200.0], [2.0, 0.0, np.inf]], np.float64)
    elts = Elts(catalog, rec_off, rec_ids, rec_loss, terms)
    trials = [[1, 3, 5, 6, 7], [3], [], [7, 7, 0], [1, 1]]
    offsets = np.zeros(6, np.int64)
    np.cumsum([len(t) for t in trials], out=offsets[1:])
    ids = np.array([e for t in trials for e in t], np.int32)
    layers = Layers(np.array([0, 2], np.int32), np.array([0, 1], np.int32),
                    np.array([[50.0, 250.0, 100.0, 400.0]], np.float64))
    return Workload("hand-example", Yet(catalog, offsets, ids, None), elts, layers, 0.6)
