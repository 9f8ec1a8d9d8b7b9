"""Serving experiments: Poisson arrivals into the continuous-batching server,
against a plain sequential solver (rei_solve per request, first come first
served) on the same arrivals.

The request mix is 60% plain, 30% large and 10% single instances (the three
single-instance shapes), each searched up to its target's cost.  Large
requests get a 1 GiB language cache (the deepest of them end out of memory,
an outcome compared like any other), the others 64 MiB and 1 GiB.
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np

from . import instances as I


_large_memo = {}


def _large(seed: int):
    # drawing a large specification takes tens of milliseconds (its target's
    # language is enumerated over all ternary strings up to length 10); the
    # mix reuses 64 seeds, each drawn once per process
    if seed not in _large_memo:
        _large_memo[seed] = I.large_instance(seed)
    return _large_memo[seed]


def request_mix(seed: int, n: int):
    """n request specs: (kind, Instance, cache_bytes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = rng.choice(3, size=n, p=[0.6, 0.3, 0.1])
    out = []
    for k, kind in enumerate(kinds):
        sub = int(rng.integers(0, 1 << 30))
        if kind == 0:
            inst = I.plain_instance(sub)
            out.append(("plain", inst, 64 << 20))
        elif kind == 1:
            inst = _large(sub % 64)
            out.append(("large", inst, 1 << 30))
        else:
            costs = (1, 1, 1, 1, 1) if k % 2 == 0 else (1, 1, 5, 1, 2)
            inst = I.single_instance(sub % 256, costs)
            out.append(("single", inst, 1 << 30))
    return out


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def stage(rei, specs):
    return [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for _, i, cache in specs]


def percentiles(lat: Sequence[float]):
    a = np.sort(np.asarray(lat))
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3)}


def run_served(rei, handles, arrivals, budget: int, max_batch: int = 64, n_streams: int = 4,
               n_workers: int = 4, queue: bool = True):
    """Submits handles[i] at arrivals[i] seconds; returns results, latencies and
    instances per second (requests / time from first arrival to last completion).
    queue: the server's queue mode (persistent launches fed while they run)
    or its launch mode (one batched launch per admitted group)."""
    srv = rei.Server(budget, max_batch, n_streams, n_workers, queue=queue)
    t0 = time.perf_counter()
    tickets, submit_at = [], []
    for h, ta in zip(handles, arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        submit_at.append(time.perf_counter() - t0)
        tickets.append(srv.submit(h))
    results, lat = [], []
    for t in tickets:
        r, l = srv.wait(t)
        results.append(r)
        lat.append(l)
    srv.close()
    end = max(s + l for s, l in zip(submit_at, lat))
    return results, lat, len(handles) / (end - submit_at[0])


def run_sequential(rei, handles, arrivals, stream=None):
    """One request at a time in arrival order (rei_solve); a request waits
    for the previous one.  Service times are measured; waiting is computed."""
    results, lat = [], []
    finish = 0.0
    for h, ta in zip(handles, arrivals):
        t = time.perf_counter()
        r = h.solve(stream) if stream is not None else h.solve()
        d = time.perf_counter() - t
        start = max(float(ta), finish)
        finish = start + d
        results.append(r)
        lat.append(finish - float(ta))
    return results, lat, len(handles) / (finish - float(arrivals[0]))


def same(a, b) -> bool:
    return (a.status, a.cost, a.regex, a.unique, a.candidates) == (b.status, b.cost, b.regex, b.unique,
                                                                    b.candidates)


def sweep(rei, n: int, fractions=(0.25, 0.5, 0.75, 1.0), seed: int = 2024, budget: int = 0, stream=None):
    """Serving at fixed rates: ``n`` Poisson arrivals of the mix per point, the
    rate a fraction of the measured sequential capacity (requests per second
    of back-to-back rei_solve), the server against a first-come-first-served
    sequential solver on the same arrivals.  The server is warmed (one untimed
    pass of the whole mix, so each instance's buffers exist) before the timed
    points.  budget 0 = the free HBM less 8 GB at server creation."""
    specs = request_mix(seed, n)
    hs = stage(rei, specs)
    base = poisson_arrivals(seed, n, 1.0)
    seq_res, _, _ = run_sequential(rei, hs, base * 0.0, stream)  # warms the instances (allocations)
    t = time.perf_counter()
    for h in hs:
        h.solve(stream)
    capacity = n / (time.perf_counter() - t)
    run_served(rei, hs, base / (4 * capacity), budget)  # warm the server paths (untimed)
    run_served(rei, hs, base / (4 * capacity), budget, queue=False)
    points = []
    for f in fractions:
        qps = capacity * f
        arr = base / qps
        res, lat, ips = run_served(rei, hs, arr, budget)
        lres, llat, lips = run_served(rei, hs, arr, budget, queue=False)
        sres, slat, sips = run_sequential(rei, hs, arr, stream)
        points.append({"load": f, "qps": round(qps, 2),
                       "served": {"mode": "queue", "instances_per_sec": round(ips, 2),
                                  **{k: round(v, 3) for k, v in percentiles(lat).items()}},
                       "served_launch_mode": {"instances_per_sec": round(lips, 2),
                                              **{k: round(v, 3) for k, v in percentiles(llat).items()}},
                       "sequential": {"instances_per_sec": round(sips, 2),
                                      **{k: round(v, 3) for k, v in percentiles(slat).items()}},
                       "identical_results": all(same(a, b) and same(a, c) for a, b, c in zip(res, seq_res, lres))})
    kinds = {k: sum(1 for s in specs if s[0] == k) for k in ("plain", "large", "single")}
    # the last point's latencies by request kind
    for key, l in (("served", lat), ("served_launch_mode", llat), ("sequential", slat)):
        points[-1][key]["by_kind"] = {k: {q: round(v, 3) for q, v in
                                          percentiles([x for x, s in zip(l, specs) if s[0] == k]).items()}
                                      for k in kinds if kinds[k]}
    for h in hs:
        h.close()
    return {"arrivals_per_point": n, "mix": kinds, "sequential_capacity_per_sec": round(capacity, 2),
            "points": points}
