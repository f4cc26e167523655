"""Serving workloads on the library's continuous-batching server: open-loop
Poisson arrivals of (transmitter, receiver set) queries, latency percentiles
and throughput.  Latency of a query = results on the host minus its submit
time, both taken by the library on the host monotonic clock."""
from __future__ import annotations

import queue
import threading
import time

import numpy as np


def _collect(server, tickets_q, n, out):
    for _ in range(n):
        t = tickets_q.get()
        if t is None:
            break
        _, _, info = server.poll(t, -1)
        out.append(info)


def run_open_loop(server, queries, rate: float) -> dict:
    """Submit queries at their arrival times (unit-rate gaps scaled by 1/rate)
    and wait for all of them.  Returns latency percentiles (ms) and rates."""
    tq: queue.Queue = queue.Queue()
    infos: list = []
    th = threading.Thread(target=_collect, args=(server, tq, len(queries), infos), daemon=True)
    th.start()
    t0 = time.perf_counter()
    at = 0.0
    nrx = 0
    for gap, tx, rx in queries:
        at += gap / rate
        while True:
            dt = t0 + at - time.perf_counter()
            if dt <= 0:
                break
            if dt > 2e-4:
                time.sleep(dt - 1e-4)
        tq.put(server.submit(tx, rx))
        nrx += rx.shape[0]
    th.join()
    return summarise(infos, nrx, offered=rate)


def run_burst(server, queries) -> dict:
    """Closed burst: every query submitted at once (saturation throughput)."""
    tq: queue.Queue = queue.Queue()
    infos: list = []
    th = threading.Thread(target=_collect, args=(server, tq, len(queries), infos), daemon=True)
    th.start()
    nrx = 0
    for _, tx, rx in queries:
        tq.put(server.submit(tx, rx))
        nrx += rx.shape[0]
    th.join()
    return summarise(infos, nrx, offered=None)


def summarise(infos, nrx, offered=None) -> dict:
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos]) * 1e3
    t_first = min(i["t_submit"] for i in infos)
    t_last = max(i["t_done"] for i in infos)
    span = max(t_last - t_first, 1e-9)
    bq = np.array([i["batch_queries"] for i in infos])
    return {
        "offered_qps": offered,
        "queries": len(infos),
        "achieved_qps": len(infos) / span,
        "rx_views_per_s": nrx / span,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "mean_batch_queries": float(bq.mean()),
    }
