"""Serving experiments: Poisson arrivals into the continuous-batching server,
against a plain sequential solver (rei_solve per request, first come first
served) on the same arrivals.

The request mix is 60% plain, 30% large and 10% single instances (the three
single-instance shapes).  Large-instance requests search up to cost 10 with a
1 GiB cache so that one request stays in the milliseconds-to-seconds range.
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np

from . import instances as I


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
            inst = I.large_instance(sub % 64)
            inst.max_cost = min(inst.max_cost, 10)
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
               n_workers: int = 4):
    """Submits handles[i] at arrivals[i] seconds; returns results, latencies and
    instances per second (requests / time from first arrival to last completion)."""
    srv = rei.Server(budget, max_batch, n_streams, n_workers)
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
