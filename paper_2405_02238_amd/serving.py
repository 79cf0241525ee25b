"""Load generator for the serving loop: replays timed requests against a
Server and reports per-request latency.

A request is (arrival_s, m, l, n, a_words, b_words): the serialised operand
ciphertexts a client sends (hg_ct_export of hg_encrypt outputs).  One thread
submits each request at its arrival time (host clock, relative to the start
of the replay); the caller's thread collects results in submission order.
Latency is done - arrival, where done is when the server had the result back
in host memory, so it includes queueing, the host-to-device copy, the
product and the device-to-host copy.
"""
from __future__ import annotations

import threading
import time
from typing import List, Sequence, Tuple

import numpy as np

from . import Server


def replay(server: Server, requests: Sequence[Tuple[float, int, int, int, np.ndarray, np.ndarray]],
           time_scale: float = 1.0):
    """Submit every request at arrival_s * time_scale after the start; returns
    (results, latencies_s, makespan_s) with results[i] the result words."""
    n = len(requests)
    tickets: List[int] = [0] * n
    arrive = [0.0] * n        # on the server clock
    ready = [threading.Event() for _ in range(n)]
    errors: List[BaseException] = []
    # align the replay clock with the server clock
    base = server.stats()["clock"]
    t0 = time.perf_counter()

    def submitter():
        try:
            for i, (at, m, l, nn, a, b) in enumerate(requests):
                delay = at * time_scale - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                arrive[i] = base + at * time_scale
                tickets[i] = server.submit(a, b, m, l, nn)
                ready[i].set()
        except BaseException as e:  # surfaced to the caller below
            errors.append(e)
            for ev in ready:
                ev.set()

    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    results, lat, done_times = [], [], []
    for i in range(n):
        ready[i].wait()
        if errors:
            break
        words, (t_sub, t_start, t_done) = server.wait(tickets[i])
        results.append(words)
        lat.append(t_done - min(arrive[i], t_sub))
        done_times.append(t_done)
    th.join()
    if errors:
        raise errors[0]
    makespan = max(done_times) - base if done_times else 0.0
    return results, np.array(lat), makespan


def percentile_ms(lat: np.ndarray, q: float) -> float:
    return float(np.percentile(lat, q) * 1000.0) if len(lat) else 0.0
