"""Request driver for the serving loop: per-headset Poisson frame arrivals
in real time, gaze from each headset's seeded trace, completion polling and
latency statistics.  The loop itself (admission, continuous batching,
device work) runs in the native library's dispatcher thread."""
from __future__ import annotations

import time

import numpy as np


def arrival_times(n_headsets: int, rate_hz: float, duration_s: float, seed_base: int = 5):
    """Merged (time_s, headset, frame) arrivals: each headset's requests form
    a Poisson process of the given rate (seeded with seed_base + h)."""
    ev = []
    for h in range(n_headsets):
        rng = np.random.default_rng(seed_base + h)
        t, f = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            ev.append((t, h, f))
            f += 1
    ev.sort()
    return ev


def run(server, V, gazes, arrivals, deadline_ms=0.0, on_result=None, poll_every_s=0.0005):
    """Submit `arrivals` at their times (relative to the start), release each
    result after on_result(result) (if given), and return per-request
    records plus the wall time.  gazes[h][f] is the gaze of headset h's frame f."""
    recs = []
    refused = 0
    t0 = time.perf_counter()
    i = 0

    def drain():
        for r in server.poll():
            if on_result is not None:
                on_result(r)
            if r["status"] == 0:
                server.release(r["slot"])
            recs.append(r)

    while i < len(arrivals):
        now = time.perf_counter() - t0
        t, h, f = arrivals[i]
        if now >= t:
            g = gazes[h][f % len(gazes[h])]
            if not server.submit(h, f, V.gaze(float(g[0]), float(g[1])), deadline_ms, tag=i):
                refused += 1
            i += 1
            continue
        drain()
        time.sleep(min(poll_every_s, max(0.0, t - now)))
    # keep releasing results until nothing is queued or in flight (leased
    # buffers count against the budget, so waiting without draining could
    # starve admission)
    t_end = time.perf_counter() + 120.0
    while time.perf_counter() < t_end:
        drain()
        st = server.stats()
        if st["waiting"] == 0 and st["inflight"] == 0:
            break
        time.sleep(poll_every_s)
    drain()
    wall = time.perf_counter() - t0
    return recs, refused, wall


def latency_stats(recs):
    ok = [r for r in recs if r["status"] == 0]
    lat = np.array([r["done_ms"] - r["submit_ms"] for r in ok]) if ok else np.zeros(1)
    queue = np.array([r["launch_ms"] - r["submit_ms"] for r in ok]) if ok else np.zeros(1)
    return {"completed": len(ok), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "mean_queue_ms": float(queue.mean())}
