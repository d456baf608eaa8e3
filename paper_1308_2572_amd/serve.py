"""Serving benchmark: replay Poisson-arriving pricing quotes through the
continuous-batching quote server and report latency percentiles, throughput,
and each quote's plain (stand-alone, synchronous) batch time for comparison.
"""
from __future__ import annotations

import time
from typing import Dict, List

import numpy as np
import torch

from . import Layers, QuoteServer, metrics, ylt_backward, ylt_forward


def plain_time_ms(tables, yet, elt_terms, req, p: float, reps: int = 3) -> float:
    """Synchronous stand-alone time of one quote through the batch entry points
    (forward, metrics, and the backward when the quote asks for gradients)."""
    dev = yet.device
    layers = Layers(np.array([0, len(req.elt_ids)], np.int32), req.elt_ids)
    lt = torch.tensor(np.asarray(req.layer_terms, np.float64)[None, :], device=dev)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        y, s, _ = ylt_forward(tables, yet, layers, elt_terms, lt, req.trial_begin, req.trial_end,
                              want_s_pre=req.want_grad)
        _, w = metrics(y, p, want_weights=req.want_grad)
        if req.want_grad:
            ylt_backward(tables, yet, layers, elt_terms, lt, s, w, req.trial_begin, req.trial_end)
        torch.cuda.synchronize(dev)
        best = min(best, (time.perf_counter() - t) * 1e3)
    return best


def run_benchmark(tables, yet, elt_terms, requests: List, p: float = 0.99, quotes_with_grad: int = 16,
                  max_slots: int = 64, plain_sample: int = 20) -> Dict:
    server = QuoteServer(tables, yet, elt_terms, quotes_with_grad=quotes_with_grad, max_slots=max_slots)
    try:
        # warm-up: kernels, LDS attributes, allocator
        for r in requests[:2]:
            server.wait(server.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, p, r.want_grad))
        t0 = time.perf_counter()
        tickets = []
        for r in requests:
            delay = t0 + r.arrival_s - requests[0].arrival_s - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(server.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, p, r.want_grad))
        results = [server.wait(t) for t in tickets]
        stats = server.stats()
    finally:
        server.close()
    lat = np.array([x["t_done_ms"] - x["t_submit_ms"] for x in results])
    queue = np.array([x["t_admit_ms"] - x["t_submit_ms"] for x in results])
    span_s = (max(x["t_done_ms"] for x in results) - min(x["t_submit_ms"] for x in results)) / 1e3
    lookups = sum((int(yet.handle.nnz) * (r.trial_end - r.trial_begin) / max(int(yet.handle.n_trials), 1))
                  * len(r.elt_ids) for r in requests)
    sample = requests[:: max(1, len(requests) // max(plain_sample, 1))][:plain_sample]
    plain = np.array([plain_time_ms(tables, yet, elt_terms, r, p) for r in sample])
    return {
        "requests": len(requests),
        "with_grad": int(sum(r.want_grad for r in requests)),
        "offered_rate_per_s": len(requests) / max(requests[-1].arrival_s - requests[0].arrival_s, 1e-9),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "queue_p99_ms": float(np.percentile(queue, 99)),
        "throughput_req_per_s": len(requests) / span_s,
        "lookups_per_s": lookups / span_s,
        "plain_batch_ms_p50": float(np.percentile(plain, 50)),
        "plain_batch_ms_p99": float(np.percentile(plain, 99)),
        "p99_over_plain_p99": float(np.percentile(lat, 99) / np.percentile(plain, 99)),
        "server": stats,
    }
