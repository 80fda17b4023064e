"""Replay of a request trace against a ``Server`` (arrivals on schedule) and
the latency / throughput summary of the results.

A request is submitted at its arrival time on the server clock; its latency
runs from that scheduled arrival to the moment the server finished it, so a
late submission is charged to the server, not hidden.
"""
from __future__ import annotations

import time

import numpy as np

from . import Server


def replay(server: Server, requests, arrivals, tonal_iters: int = 30) -> list[dict]:
    """requests: list of (f uint8[side*side], mask int32[m]); arrivals: seconds
    from the start of the replay (ascending). Returns one result dict per
    request, in order, with ``arrival`` and ``latency`` (seconds) added."""
    arrivals = np.asarray(arrivals, dtype=np.float64)
    t0 = server.clock()
    tickets = []
    for (f, m), at in zip(requests, arrivals):
        wait = t0 + at - server.clock()
        if wait > 0:
            time.sleep(wait)
        tickets.append(server.submit(f, m, tonal_iters=tonal_iters))
    out = []
    for t, at, (f, _) in zip(tickets, arrivals, requests):
        r = server.poll(t, wait=True)
        r["arrival"] = t0 + at
        r["latency"] = r["t_done"] - r["arrival"]
        r["pixels"] = int(f.size)
        out.append(r)
    return out


def summarize(results: list[dict]) -> dict:
    """p50 / p99 / mean latency (ms), makespan from the first arrival to the
    last completion, and the throughput over it (Mpixel/s, requests/s)."""
    lat = np.array([r["latency"] for r in results]) * 1e3
    first = min(r["arrival"] for r in results)
    last = max(r["t_done"] for r in results)
    span = last - first
    pix = sum(r["pixels"] for r in results)
    return {
        "requests": len(results),
        "failed": int(sum(r["status"] != 0 for r in results)),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "makespan_s": span,
        "mpixel_per_s": pix / span / 1e6,
        "requests_per_s": len(results) / span,
        "inner_iterations": int(sum(r["inner_iterations"] for r in results)),
    }
