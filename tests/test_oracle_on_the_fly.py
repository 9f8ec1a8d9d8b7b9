"""OnTheFly mode of the oracle (Sec. 3, "OnTheFly mode").

Once the language cache is full the search goes on without storing and
without uniqueness checks, for as long as every block it enumerates draws on
complete (fully stored) levels.  Pinned against the unlimited search, which
brute force and the paper's printed answers pin in the other oracle tests:
when OnTheFly finds an expression it is the unlimited search's answer, with
the same candidate counts up to it; otherwise it reports out of memory.
"""
import brute
from paper_2305_18575_amd import instances

COSTS = [(1, 1, 1, 1, 1), (1, 1, 5, 1, 2), (1, 3, 3, 3, 3), (2, 5, 5, 5, 5)]


def _full_level(unique, cap):
    """The level at which a search capped at `cap` rows fills its cache."""
    acc = 0
    for c, u in enumerate(unique):
        acc += u
        if acc > cap:
            return c
    return None


def test_on_the_fly_finds_the_unlimited_answer(oracle_mod):
    beyond = 0
    checked = 0
    for seed in range(16):
        it = instances.single_instance(seed, (1, 1, 1, 1, 1))
        for costs in COSTS:
            full = oracle_mod.solve(it.alphabet, it.pos, it.neg, costs, 40, 1 << 40, 0, 4)
            assert full.status == "OK"
            total = sum(full.unique)
            for frac in (0.2, 0.5, 0.9):
                cap = max(1, int(total * frac))
                r = oracle_mod.solve(it.alphabet, it.pos, it.neg, costs, 40, cap, 0, 4, on_the_fly=True)
                plain = oracle_mod.solve(it.alphabet, it.pos, it.neg, costs, 40, cap, 0, 4)
                assert plain.status == "OUT_OF_MEMORY"
                lvl = _full_level(full.unique, cap)
                # levels before the full one are searched exactly as without a cap
                assert r.unique[:lvl] == full.unique[:lvl]
                assert r.candidates[:lvl] == full.candidates[:lvl]
                # nothing counts as new once the cache is full
                assert sum(r.unique) == cap
                if r.status == "OK":
                    assert (r.cost, r.regex) == (full.cost, full.regex), (seed, costs, cap)
                    assert r.candidates[: full.cost + 1] == full.candidates[: full.cost + 1]
                    assert brute.regex_cost(r.regex, costs) == full.cost
                    checked += 1
                    beyond += full.cost > lvl
                else:
                    assert r.status == "OUT_OF_MEMORY"
    assert checked > 50
    assert beyond > 10  # answers found several levels after the cache filled


def test_on_the_fly_stops_at_an_incomplete_level(oracle_mod):
    """Unit costs: level c+1 starts with r? over level c, so once level c
    filled the cache, level c is finished on the fly and the search stops
    before enumerating anything of level c+1."""
    stopped = 0
    for seed in range(16):
        it = instances.single_instance(seed, (1, 1, 1, 1, 1))
        full = oracle_mod.solve(it.alphabet, it.pos, it.neg, (1, 1, 1, 1, 1), 40, 1 << 40, 0, 4)
        cap = max(1, sum(full.unique) // 3)
        lvl = _full_level(full.unique, cap)
        r = oracle_mod.solve(it.alphabet, it.pos, it.neg, (1, 1, 1, 1, 1), 40, cap, 0, 4, on_the_fly=True)
        if full.cost > lvl:
            assert r.status == "OUT_OF_MEMORY"
            assert r.candidates[lvl] == full.candidates[lvl]  # the full level is finished
            assert r.candidates[lvl + 1] == 0
            stopped += 1
        else:
            assert (r.status, r.cost, r.regex) == ("OK", full.cost, full.regex)
    assert stopped > 5


def test_on_the_fly_brute_force(oracle_mod):
    """Tiny instances: the OnTheFly answer has brute force's minimal cost."""
    for seed in range(8):
        it = instances.plain_instance(seed)
        costs = (1, 2, 2, 2, 2)
        counts, cstar = brute.brute_levels("01", it.pos, it.neg, costs, 9)
        if cstar is None:
            continue
        total = sum(counts.get(c, 0) for c in range(1, cstar))
        r = oracle_mod.solve("01", it.pos, it.neg, costs, 9, max(1, total // 2), 0, 1, on_the_fly=True)
        assert r.status in ("OK", "OUT_OF_MEMORY")
        if r.status == "OK":
            assert r.cost == cstar
            assert brute.regex_cost(r.regex, costs) == cstar
