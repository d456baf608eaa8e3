"""Serving benchmark: replay Poisson-arriving pricing quotes through the
continuous-batching quote server and report latency percentiles, throughput,
how the quotes were packed, and each quote's plain (stand-alone, synchronous)
batch time for comparison.
"""
from __future__ import annotations

import time
from typing import Dict, List

import numpy as np
import torch

from . import Layers, QuoteServer, metrics, ylt_backward, ylt_forward


def plain_call(tables, yet, elt_terms, req, p: float):
    """One quote through the batch entry points (forward, metrics, and the
    backward when the quote asks for gradients), synchronised."""
    dev = yet.device
    layers = Layers(np.array([0, len(req.elt_ids)], np.int32), req.elt_ids)
    lt = torch.tensor(np.asarray(req.layer_terms, np.float64)[None, :], device=dev)
    y, s, _ = ylt_forward(tables, yet, layers, elt_terms, lt, req.trial_begin, req.trial_end, want_s_pre=req.want_grad)
    _, w = metrics(y, p, want_weights=req.want_grad)
    if req.want_grad:
        ylt_backward(tables, yet, layers, elt_terms, lt, s, w, req.trial_begin, req.trial_end)
    torch.cuda.synchronize(dev)


def plain_time_ms(tables, yet, elt_terms, req, p: float, reps: int = 3) -> float:
    """Synchronous stand-alone time of one quote (best of reps)."""
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize(yet.device)
        t = time.perf_counter()
        plain_call(tables, yet, elt_terms, req, p)
        best = min(best, (time.perf_counter() - t) * 1e3)
    return best


def serial_throughput(tables, yet, elt_terms, requests: List, p: float) -> float:
    """Quotes per second when the same quotes run one after another through
    the batch entry points (no batching, no overlap)."""
    torch.cuda.synchronize(yet.device)
    t = time.perf_counter()
    for r in requests:
        plain_call(tables, yet, elt_terms, r, p)
    return len(requests) / (time.perf_counter() - t)


def run_benchmark(tables, yet, elt_terms, requests: List, p: float = 0.99, quotes_with_grad: int = 16,
                  max_slots: int = 64, plain_sample: int = 20, progress=None) -> Dict:
    server = QuoteServer(tables, yet, elt_terms, quotes_with_grad=quotes_with_grad, max_slots=max_slots)
    try:
        # warm-up: kernels, LDS attributes, allocator
        for r in requests[:2]:
            server.wait(server.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, p, r.want_grad))
        base = server.stats()
        t0 = time.perf_counter()
        tickets = []
        next_note = t0 + 10.0
        for r in requests:
            delay = t0 + r.arrival_s - requests[0].arrival_s - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets.append(server.submit(r.elt_ids, r.layer_terms, r.trial_begin, r.trial_end, p, r.want_grad))
            if progress and time.perf_counter() > next_note:
                progress(f"{len(tickets)} of {len(requests)} quotes submitted")
                next_note += 10.0
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
    launches = stats["packed_launches"] - base["packed_launches"]
    items = stats["items"] - base["items"]
    return {
        "requests": len(requests),
        "with_grad": int(sum(r.want_grad for r in requests)),
        "offered_rate_per_s": len(requests) / max(requests[-1].arrival_s - requests[0].arrival_s, 1e-9),
        "duration_s": span_s,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "queue_p99_ms": float(np.percentile(queue, 99)),
        "throughput_req_per_s": len(requests) / span_s,
        "lookups_per_s": lookups / span_s,
        "plain_batch_ms_p50": float(np.percentile(plain, 50)),
        "plain_batch_ms_p99": float(np.percentile(plain, 99)),
        "p99_over_plain_p99": float(np.percentile(lat, 99) / np.percentile(plain, 99)),
        "launches": launches,
        "items_per_launch": items / max(launches, 1),
        "shared_block_item_frac": (stats["shared_block_items"] - base["shared_block_items"]) / max(items, 1),
        "server": stats,
    }


def main(argv=None) -> int:
    """Replay quotes through the server over the resident serving workload
    (1,000,000 trials x Poisson(1000) events, 200 ELTs) and print one JSON
    line; by default 600 quotes all arriving at once (a saturating burst)."""
    import argparse
    import json

    import synth
    from . import EltTables, PreparedYet
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--rate", type=float, default=1e9, help="Poisson arrivals per second (1e9: all at once)")
    ap.add_argument("--seed", type=int, default=synth.SEED_BASE + 40)
    ap.add_argument("--plain-sample", type=int, default=1, help="quotes also timed through the batch entry points")
    ap.add_argument("--quotes-with-grad", type=int, default=16,
                    help="the server's arena is sized for this many gradient quotes at once")
    ap.add_argument("--max-slots", type=int, default=64, help="quotes active at once (1..256)")
    args = ap.parse_args(argv)
    w = synth.config(4)
    tables = EltTables.from_numpy(w.elts)
    yet = PreparedYet.from_numpy(w.yet)
    et = torch.tensor(w.elts.terms, dtype=torch.float64, device="cuda")
    reqs = synth.serving_requests(args.requests, w.yet.n_trials, n_elts=w.elts.n_elts, rate_per_s=args.rate,
                                  seed=args.seed)
    out = run_benchmark(tables, yet, et, reqs, p=0.99, quotes_with_grad=args.quotes_with_grad, max_slots=args.max_slots,
                        plain_sample=max(1, args.plain_sample))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
