"""The oracle against brute force over expression trees and against invariants.

Brute force enumerates every tree up to a cost bound and decides each tree's
language on the strings with the relational semantics (tests/brute.py), so a
mistake in the oracle's constructors, its dedup or its level bookkeeping
changes a count here.
"""
import random

import pytest

import brute
from paper_2305_18575_amd import instances


def _compare(oracle_mod, sigma, P, N, costs, kmax, max_errors=0):
    counts, cstar = brute.brute_levels(sigma, P, N, costs, kmax, max_errors)
    r = oracle_mod.solve(sigma, P, N, costs=costs, max_cost=kmax, max_errors=max_errors)
    if cstar is None:
        assert r.status == "NOT_FOUND"
        for c in range(1, kmax + 1):
            assert r.unique[c] == counts.get(c, 0), (c, r.unique, counts)
    else:
        assert r.status == "OK" and r.cost == cstar
        for c in range(1, cstar):
            assert r.unique[c] == counts.get(c, 0), (c, r.unique, counts)
        # the answer's expression is precise and has the minimal cost
        lang = brute.language_on(r.regex, brute.ic_of(P + N))
        bad = sum(1 for w in P if w not in lang) + sum(1 for w in N if w in lang)
        assert bad <= max_errors
        assert brute.regex_cost(r.regex, costs) == cstar
    return r


@pytest.mark.parametrize("seed", range(12))
def test_plain_instances_vs_brute_force(oracle_mod, seed):
    inst = instances.plain_instance(seed)
    _compare(oracle_mod, "01", inst.pos, inst.neg, (1, 1, 1, 1, 1), 7)


@pytest.mark.parametrize("seed", range(6))
def test_unsolvable_levels_vs_brute_force(oracle_mod, seed):
    # random strings: usually no cheap precise expression, so every level up
    # to the bound is compared
    rng = random.Random(seed)
    words = instances.words("01", 0, 6)
    sample = rng.sample(words, 14)
    P, N = sample[:7], sample[7:]
    _compare(oracle_mod, "01", P, N, (1, 1, 1, 1, 1), 7)


@pytest.mark.parametrize("costs", [(1, 1, 5, 1, 2), (2, 1, 1, 3, 1), (1, 3, 1, 1, 4)])
def test_other_cost_functions_vs_brute_force(oracle_mod, costs):
    kmax = 9 if costs[0] == 1 else 11
    for seed in range(3):
        rng = random.Random(100 + seed)
        words = instances.words("01", 0, 5)
        sample = rng.sample(words, 10)
        _compare(oracle_mod, "01", sample[:5], sample[5:], costs, kmax)


def test_ternary_vs_brute_force(oracle_mod):
    for seed in range(3):
        rng = random.Random(7 + seed)
        words = instances.words("012", 0, 4)
        sample = rng.sample(words, 10)
        _compare(oracle_mod, "012", sample[:5], sample[5:], (1, 1, 1, 1, 1), 6)


def test_allowed_error_vs_brute_force(oracle_mod):
    rng = random.Random(3)
    words = instances.words("01", 0, 6)
    sample = rng.sample(words, 16)
    for k in (1, 2, 3, 5):
        _compare(oracle_mod, "01", sample[:8], sample[8:], (1, 1, 1, 1, 1), 7, k)


@pytest.mark.parametrize("seed", range(4))
def test_rows_print_their_language(oracle_mod, seed):
    """Every stored language's printed expression denotes exactly that
    language on ic (checked with ``re``); no language repeats; each level
    has the cost of its expressions."""
    inst = instances.plain_instance(seed + 50)
    o = oracle_mod.Oracle("01", inst.pos, inst.neg, max_cost=7)
    r = o.solve()
    ic = o.ic
    seen = set()
    for row in range(o.num_rows()):
        cs = o.row_cs(row)
        assert cs not in seen
        seen.add(cs)
        text = o.row_regex(row)
        lang = brute.language_on(text, ic)
        assert {w for w, b in zip(ic, cs) if b} == set(lang), text
        assert brute.regex_cost(text) == o.row_level(row)
    # no stored language below the answer's cost is precise
    for row in range(o.num_rows()):
        cs = o.row_cs(row)
        precise = all(cs[ic.index(p)] for p in inst.pos) and not any(cs[ic.index(n)] for n in inst.neg)
        assert not precise


def test_candidate_counts_follow_level_sizes(oracle_mod):
    """Below the answer's level, candidates per level = Q + S + C + U block sizes."""
    rng = random.Random(11)
    words = instances.words("01", 0, 6)
    sample = rng.sample(words, 16)
    costs = (1, 2, 1, 1, 3)
    o = oracle_mod.Oracle("01", sample[:8], sample[8:], costs=costs, max_cost=9)
    r = o.solve()
    n = {c: o.level_size(c) for c in range(0, 10)}
    last = 9 if r.status == "NOT_FOUND" else r.cost - 1
    for c in range(2, last + 1):
        q = n.get(c - costs[1], 0) if c - costs[1] >= 1 else 0
        s = n.get(c - costs[2], 0) if c - costs[2] >= 1 else 0
        cc = sum(n[L] * n[c - costs[3] - L] for L in range(1, c) if c - costs[3] - L >= 1)
        u = 0
        for L in range(1, c):
            R = c - costs[4] - L
            if R < L:
                break
            u += n[L] * n[R] if L < R else n[L] * (n[L] - 1) // 2
        assert r.candidates[c] == q + s + cc + u, c
    # cumulative counts never exceed the number of possible languages
    assert sum(r.unique) <= 2 ** len(o.ic)


def test_thread_count_does_not_change_results(oracle_mod):
    inst = instances.single_instance(6)
    a = oracle_mod.solve("01", inst.pos, inst.neg, threads=1)
    b = oracle_mod.solve("01", inst.pos, inst.neg, threads=5)
    assert a == b


def test_row_cap_out_of_memory(oracle_mod):
    inst = instances.single_instance(3)
    full = oracle_mod.solve("01", inst.pos, inst.neg)
    cap = sum(full.unique[: full.cost]) // 2
    r = oracle_mod.solve("01", inst.pos, inst.neg, row_cap=cap)
    assert r.status == "OUT_OF_MEMORY"
    assert sum(r.unique) == cap


@pytest.mark.parametrize("seed,sigma,char_costs,costs", [
    (0, "01", {"0": 1, "1": 2}, (1, 1, 1, 1, 1)),
    (1, "01", {"0": 3, "1": 1}, (1, 1, 1, 1, 1)),
    (2, "01", {"0": 2, "1": 2}, (1, 1, 2, 1, 1)),
    (3, "012", {"0": 1, "1": 2, "2": 3}, (1, 1, 1, 1, 1)),
    (4, "012", {"0": 2, "1": 1, "2": 1}, (1, 2, 1, 1, 2)),
])
def test_per_character_costs_vs_brute_force(oracle_mod, seed, sigma, char_costs, costs):
    """Per-character costs (the cost-homomorphism definition allows one cost
    per character): brute force gives every character its own leaf cost."""
    rng = random.Random(seed)
    words = ["".join(rng.choice(sigma) for _ in range(rng.randint(0, 4))) for _ in range(8)]
    words = list(dict.fromkeys(words))
    P, N = words[: len(words) // 2], words[len(words) // 2:]
    kmax = 8
    counts, cstar = brute.brute_levels(sigma, P, N, costs, kmax, 0, char_costs)
    r = oracle_mod.solve(sigma, P, N, costs=costs, max_cost=kmax,
                         char_costs=[char_costs[a] for a in sigma])
    lo = min(char_costs.values())
    if not P:
        assert (r.status, r.cost) == ("OK", lo)
        return
    if cstar is None:
        assert r.status == "NOT_FOUND"
        for c in range(1, kmax + 1):
            assert r.unique[c] == counts.get(c, 0), (c, r.unique, counts)
    else:
        assert r.status == "OK" and r.cost == cstar, (r, cstar)
        for c in range(1, cstar):
            assert r.unique[c] == counts.get(c, 0), (c, r.unique, counts)
        assert brute.regex_cost(r.regex, costs, char_costs) == cstar
