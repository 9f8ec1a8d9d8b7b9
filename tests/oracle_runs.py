"""The CPU oracle on many specifications at once, for the GPU tests.

The oracle's C calls release the GIL, so a thread pool runs independent
specifications in parallel.  Results are kept per specification for the
session: several tests compare against the same searches.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import oracle
from paper_2305_18575_amd import instances

_memo = {}


def _key(alphabet, pos, neg, costs, max_cost, row_cap, max_errors):
    return (alphabet, tuple(pos), tuple(neg), tuple(costs), int(max_cost), int(row_cap), int(max_errors))


def oracle_cap(cache_bytes: int, alphabet: str, pos, neg) -> int:
    """The row cap the library derives from a cache budget (0 infixes is the
    trivial empty specification, which stores nothing)."""
    n = instances.n_infixes(list(pos) + list(neg))
    return instances.row_cap(cache_bytes, n) if n else 1 << 40


def solve_many(specs, workers: int = 4, threads: int = 4):
    """specs: (alphabet, pos, neg, costs, max_cost, cache_bytes[, max_errors]).
    Returns the oracle's results in the same order."""
    keys = []
    for sp in specs:
        alphabet, pos, neg, costs, max_cost, cache = sp[:6]
        err = sp[6] if len(sp) > 6 else 0
        keys.append(_key(alphabet, pos, neg, costs, max_cost, oracle_cap(cache, alphabet, pos, neg), err))
    todo = [k for k in dict.fromkeys(keys) if k not in _memo]

    def run(k):
        a, p, n, c, m, cap, e = k
        return k, oracle.solve(a, list(p), list(n), c, m, cap, e, threads)

    with ThreadPoolExecutor(workers) as ex:
        for k, r in ex.map(run, todo):
            _memo[k] = r
    return [_memo[k] for k in keys]


def mismatch(g, o, max_cost: int):
    """None when the GPU result g equals the oracle's o in every reported
    field (status, minimal cost, expression, per-level unique and candidate
    counts), else a description of the first difference."""
    if (g.status, g.cost, g.regex) != (o.status, o.cost, o.regex):
        return f"status/cost/regex {g.status} {g.cost} {g.regex!r} vs {o.status} {o.cost} {o.regex!r}"
    for c in range(0, max_cost + 1):
        if g.unique_at(c) != o.unique[c] or g.candidates_at(c) != o.candidates[c]:
            return f"level {c}: unique {g.unique_at(c)} vs {o.unique[c]}, candidates " \
                   f"{g.candidates_at(c)} vs {o.candidates[c]}"
    return None
