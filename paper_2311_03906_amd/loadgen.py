"""Open-loop load generator for the sampling server.

Requests arrive as a Poisson process of rate `rate` (requests/s); each picks
a model uniformly from a pool and a shot count log-uniform in
[shots_lo, shots_hi]; its seed is its request id.  A submitter thread sleeps
until each arrival time and submits; a consumer thread waits for requests in
submission order and releases their outputs.  Latency is the server's own
done - submit time (host steady clock).
"""

from __future__ import annotations

import math
import threading
import time

import numpy as np


def poisson_plan(n: int, rate: float, n_models: int, shots_lo: int, shots_hi: int, seed: int = 0):
    """(arrival offsets in s, model index, shots) for n requests."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    models = rng.integers(0, n_models, size=n)
    shots = np.round(np.exp(rng.uniform(math.log(shots_lo), math.log(shots_hi), size=n))).astype(np.int64)
    return arrivals, models, shots


def run(server, models: list, plan, first_id: int = 0, trim: float = 0.1) -> dict:
    """Drives `server` with `plan`; returns latencies and throughput over the
    whole run, and (`steady`) over its middle: the requests completing
    between the completions of the first and last `trim` fraction."""
    arrivals, midx, shots = plan
    n = len(arrivals)
    tickets = [None] * n
    ready = threading.Semaphore(0)
    results = [None] * n
    err = []

    def submitter():
        t0 = time.perf_counter()
        for i in range(n):
            delay = t0 + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            try:
                tickets[i] = server.submit(models[midx[i]], int(shots[i]), seed=first_id + i)
            except Exception as e:  # noqa: BLE001
                err.append(e)
                tickets[i] = None
            ready.release()

    def consumer():
        for i in range(n):
            ready.acquire()
            if tickets[i] is None:
                continue
            st = server.wait(tickets[i], timeout_ms=600_000)
            results[i] = st
            server.release(tickets[i])

    ts, tc = threading.Thread(target=submitter), threading.Thread(target=consumer)
    ts.start()
    tc.start()
    ts.join()
    tc.join()
    done = [(r, int(shots[i]), models[midx[i]].n_meas) for i, r in enumerate(results) if r is not None]
    lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r, _, _ in done])
    first = min(r["t_submit_ns"] for r, _, _ in done)
    last = max(r["t_done_ns"] for r, _, _ in done)
    bits = sum(s * m for _, s, m in done)
    span = (last - first) * 1e-9
    res = {"requests": len(done), "refused": len(err), "bits": bits, "span_s": span,
           "bits_per_s": bits / span if span > 0 else 0.0,
           "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
           "mean_ms": float(lat.mean()) if len(lat) else None}
    # steady part: completions between the k0-th and k1-th completion
    order = sorted(range(len(done)), key=lambda i: done[i][0]["t_done_ns"])
    k0, k1 = int(trim * len(order)), int((1.0 - trim) * len(order)) - 1
    if k1 > k0:
        t0 = done[order[k0]][0]["t_done_ns"]
        t1 = done[order[k1]][0]["t_done_ns"]
        mid = order[k0 + 1: k1 + 1]
        mbits = sum(done[i][1] * done[i][2] for i in mid)
        mlat = lat[mid]
        res["steady"] = {"requests": len(mid), "window_s": (t1 - t0) * 1e-9,
                         "bits_per_s": mbits / ((t1 - t0) * 1e-9) if t1 > t0 else 0.0,
                         "p50_ms": float(np.percentile(mlat, 50)), "p99_ms": float(np.percentile(mlat, 99))}
    return res
