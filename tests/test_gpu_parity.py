"""GPU search (through the C ABI) against the CPU oracle, element by element.

Exact agreement is required on everything: status, minimal cost, the printed
expression (the enumeration order is fixed, so the first precise candidate is
unique), unique languages and candidates per level, and the stored rows
themselves.  All arithmetic is bitwise, so there is no tolerance.
"""
import pytest

import oracle
from paper_2305_18575_amd import instances

pytestmark = pytest.mark.gpu


def run_both(rei, alphabet, pos, neg, costs=(1, 1, 1, 1, 1), max_cost=30, cache_bytes=1 << 30,
             max_errors=0, chunk=0, rows=False, row_limit=None):
    print(f"\ncase: sigma={alphabet} |P|={len(pos)} |N|={len(neg)} costs={costs} "
          f"max_cost={max_cost} cache={cache_bytes} err={max_errors} chunk={chunk}", flush=True)
    inst = rei.Instance(alphabet, pos, neg, costs, max_cost, cache_bytes)
    if max_errors:
        inst.set_max_errors(max_errors)
    if chunk:
        inst.set_chunk(chunk)
    g = inst.solve()
    n_ic = g.ic_size
    cap = instances.row_cap(cache_bytes, n_ic) if n_ic else 1 << 40
    o_inst = oracle.Oracle(alphabet, pos, neg, costs, max_cost, cap, max_errors, threads=8)
    o = o_inst.solve()
    assert g.status == o.status, (g, o)
    assert g.cost == o.cost
    assert g.regex == o.regex
    assert g.ic_size == o.ic_size
    for c in range(0, max_cost + 1):
        assert g.unique_at(c) == o.unique[c], (c, g.unique, o.unique)
        assert g.candidates_at(c) == o.candidates[c], (c, g.candidates, o.candidates)
    if rows:
        compare_rows(inst, o_inst, g, row_limit)
    inst.close()
    return g, o


def words_of(cs_bytes, W):
    out = [0] * W
    for i, b in enumerate(cs_bytes):
        if b:
            out[i >> 6] |= 1 << (i & 63)
    return out


def compare_rows(inst, o_inst, g, limit=None):
    """Level c row i on the GPU is level c row i of the oracle (same bits)."""
    W = g.cs_words
    for k, c in enumerate(range(g.first_level, g.first_level + len(g.unique))):
        n = inst.level_size(c)
        assert n == o_inst.level_size(c), c
        idx = range(n) if limit is None else range(0, n, max(1, n // limit))
        for i in idx:
            got = inst.row_bits(c, i, W)
            want = words_of(o_inst.row_cs(o_inst.level_row(c, i)), W)
            assert got == want, (c, i)


@pytest.mark.parametrize("block", range(4))
def test_plain_config_all_seeds(rei, block):
    """Plain single instances (alphabet {0,1}, 4+4 strings of length 1..5)."""
    for seed in range(block * 50, block * 50 + 50):
        inst = instances.plain_instance(seed)
        run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost,
                 rows=(seed % 10 == 0))


@pytest.mark.parametrize("costs", [(1, 1, 1, 1, 1), (1, 1, 5, 1, 2)])
def test_single_config_all_seeds(rei, costs):
    """Single instances (10+10 strings of length 0..7, up to 255 infixes)."""
    for seed in range(32):
        inst = instances.single_instance(seed, costs)
        run_both(rei, inst.alphabet, inst.pos, inst.neg, costs, inst.max_cost,
                 rows=(seed % 8 == 0))


def test_batched_config_instances(rei):
    """Uneven small instances: alphabets of 2..4 symbols, 1..8 words per language."""
    for inst in instances.batched_instances(0, 48):
        run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost)


def test_large_config_partial(rei):
    """Ternary instances with hundreds of infixes (seed 0: 689 infixes, 16
    words per language; seed 1: 474, 8 words), levels up to cost 8 (the
    oracle is fast there).  Twenty plus twenty ternary strings of length at
    most 10 have at most 961 distinct infixes, so this configuration never
    needs 32 words; test_wide_spec_32_words covers that width."""
    for seed in (0, 1):
        inst = instances.large_instance(seed)
        run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, 8, rows=True)


@pytest.mark.parametrize("seed", range(4))
def test_large_config_full_size(rei, seed):
    """The large configuration at its full size: ternary alphabet, 20+20
    strings of length 0..10, 474-700 infixes (8-16 words per language),
    searched to the target's cost with a 64 GB cache, as bench.py's large
    instances run; all counts and the answer exact, and up to 64 rows of
    every level compared bit by bit."""
    inst = instances.large_instance(seed)
    run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, 64 << 30,
             rows=True, row_limit=64)


@pytest.mark.parametrize("chunk", [1, 7, 64, 1000])
def test_chunk_size_does_not_change_results(rei, chunk):
    inst = instances.single_instance(3, (1, 1, 5, 1, 2))
    run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, chunk=chunk,
             rows=True)


def test_repeated_solves_identical(rei):
    inst = instances.single_instance(6)
    h = rei.Instance(inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost)
    first = h.solve()
    for _ in range(3):
        again = h.solve()
        assert (again.status, again.cost, again.regex, again.unique, again.candidates) == \
            (first.status, first.cost, first.regex, first.unique, first.candidates)


def test_out_of_memory_parity(rei):
    inst = instances.single_instance(3, (1, 1, 5, 1, 2))
    for cache in (0, 16, 24 * 40, 1000 * 40, 50000 * 40):
        run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost,
                 cache_bytes=cache)


def test_not_found_parity(rei, golden):
    t = golden["table1_row1"]
    run_both(rei, t["alphabet"], t["pos"], t["neg"], (1, 1, 1, 1, 1), max_cost=12, rows=True)


def test_trivial_specifications(rei):
    g, _ = run_both(rei, "01", [], ["0", "1"])
    assert g.regex == "∅"
    g, _ = run_both(rei, "01", [""], ["0"], costs=(2, 1, 1, 1, 1))
    assert g.regex == "ε" and g.cost == 2
    g, _ = run_both(rei, "01", ["1"], ["0"])
    assert g.regex == "1"


@pytest.mark.parametrize("percent", [50, 45, 40, 35, 30, 25, 20, 15, 10])
def test_allowed_error_table_gpu(rei, golden, percent):
    """REI with error on the Table 1 row 1 specification: the GPU reproduces
    the expression and cost the paper prints, and the oracle's counts."""
    t = golden["table1_row1"]
    row = next(r for r in t["allowed_error"] if r["percent"] == percent)
    k = percent * (len(t["pos"]) + len(t["neg"])) // 100
    g, _ = run_both(rei, t["alphabet"], t["pos"], t["neg"], (1, 1, 1, 1, 1), 30, max_errors=k)
    assert (g.regex, g.cost) == (row["regex"], row["cost"])


def test_allowed_error_5_percent_gpu(rei, golden):
    """The 5% row (cost 22) against the paper's printed expression."""
    t = golden["table1_row1"]
    row = next(r for r in t["allowed_error"] if r["percent"] == 5)
    k = 5 * (len(t["pos"]) + len(t["neg"])) // 100
    g = rei.solve(t["alphabet"], t["pos"], t["neg"], max_cost=30, max_errors=k)
    assert (g.status, g.regex, g.cost) == ("OK", row["regex"], row["cost"])


def test_table1_row1_exact_answer_gpu(rei, golden):
    """Table 1 row 1 without error: minimal cost 28 (printed in the paper).
    The expression printed depends on the tie-break among equal-cost
    representatives; the language it denotes on ic must be the one of the
    paper's expression."""
    t = golden["table1_row1"]
    row = next(r for r in t["allowed_error"] if r["percent"] == 0)
    g = rei.solve(t["alphabet"], t["pos"], t["neg"], max_cost=30, cache_bytes=8 << 30)
    assert (g.status, g.cost) == ("OK", row["cost"])
    o = oracle.Oracle(t["alphabet"], t["pos"], t["neg"])
    assert o.cs_of_regex(g.regex) == o.cs_of_regex(row["regex"])
    import brute
    assert brute.regex_cost(g.regex) == 28


# ---- batched mode: many instances per call, one workgroup per instance ----

def check_against_oracle(res, spec, cache_bytes=1 << 30, max_errors=0):
    alphabet, pos, neg, costs, max_cost = spec
    cap = instances.row_cap(cache_bytes, res.ic_size) if res.ic_size else 1 << 40
    o = oracle.solve(alphabet, pos, neg, costs, max_cost, cap, max_errors, threads=8)
    assert (res.status, res.cost, res.regex) == (o.status, o.cost, o.regex), (res, o)
    for c in range(0, max_cost + 1):
        assert res.unique_at(c) == o.unique[c], (c, res.unique, o.unique)
        assert res.candidates_at(c) == o.candidates[c], (c, res.candidates, o.candidates)


def batch_specs():
    specs = []
    for seed in range(0, 200, 5):
        i = instances.plain_instance(seed)
        specs.append((i.alphabet, i.pos, i.neg, i.costs, i.max_cost))
    for costs in ((1, 1, 1, 1, 1), (1, 1, 5, 1, 2)):
        for seed in range(32):
            i = instances.single_instance(seed, costs)
            specs.append((i.alphabet, i.pos, i.neg, costs, i.max_cost))
    for i in instances.batched_instances(0, 48):
        specs.append((i.alphabet, i.pos, i.neg, i.costs, i.max_cost))
    # one instance with 16 words per language: solved on the per-chunk path
    i = instances.large_instance(0)
    specs.append((i.alphabet, i.pos, i.neg, i.costs, 8))
    return specs


@pytest.mark.parametrize("arena", [0, 1 << 16])
def test_batch_equals_oracle(rei, arena):
    """All results of one batched call equal the oracle's; arena 64 KiB
    forces most instances to outgrow their rows and take the per-chunk path."""
    specs = batch_specs()
    print(f"\nbatch of {len(specs)} instances, arena {arena}", flush=True)
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    res = rei.solve_batch(hs, arena_bytes=arena)
    for r, spec in zip(res, specs):
        check_against_oracle(r, spec)
    # rows of a few batched instances equal the oracle's rows
    for k in (0, 45, 80):
        a, p, n, c, m = specs[k]
        o_inst = oracle.Oracle(a, p, n, c, m, 1 << 40, 0, threads=8)
        o_inst.solve()
        compare_rows(hs[k], o_inst, res[k])
    for h in hs:
        h.close()


def test_batch_out_of_memory_and_errors(rei, golden):
    t = golden["table1_row1"]
    specs, hs, caps, errs = [], [], [], []
    inst = instances.single_instance(3, (1, 1, 5, 1, 2))
    for cache in (0, 16, 24 * 40, 1000 * 40, 50000 * 40):
        specs.append((inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost))
        caps.append(cache)
        errs.append(0)
    for percent in (50, 40, 25, 15, 10):
        k = percent * 22 // 100
        specs.append((t["alphabet"], t["pos"], t["neg"], (1, 1, 1, 1, 1), 30))
        caps.append(1 << 30)
        errs.append(k)
    for (a, p, n, c, m), cache, k in zip(specs, caps, errs):
        h = rei.Instance(a, p, n, c, m, cache)
        if k:
            h.set_max_errors(k)
        hs.append(h)
    res = rei.solve_batch(hs)
    for r, spec, cache, k in zip(res, specs, caps, errs):
        check_against_oracle(r, spec, cache, k)
    for h in hs:
        h.close()


def test_batch_repeat_and_single_agree(rei):
    specs = batch_specs()[40:104]
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    first = rei.solve_batch(hs)
    second = rei.solve_batch(hs)
    for h, a, b in zip(hs, first, second):
        s = h.solve()
        key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)
        assert key(a) == key(b) == key(s)
    for h in hs:
        h.close()


@pytest.mark.parametrize("seed", [3, 6])
def test_resolves_stay_exact(rei, seed):
    """Regression: re-solving one instance (all buffers already large, so no
    table rebuild between chunks) must stay exact.  These two instances
    exposed wrong second words of concatenations when the guide table was
    read from LDS through a generic pointer."""
    inst = instances.single_instance(seed, (1, 1, 5, 1, 2))
    spec = (inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost)
    o = oracle.solve(*spec, threads=8)
    h = rei.Instance(*spec)
    for rep in range(10):
        r = h.solve()
        assert (r.status, r.cost, r.regex) == (o.status, o.cost, o.regex), rep
        for c in range(0, inst.max_cost + 1):
            assert r.unique_at(c) == o.unique[c] and r.candidates_at(c) == o.candidates[c], (rep, c)
    h.close()


def test_batch_hands_large_levels_to_grid(rei, golden):
    """An instance whose levels outgrow one workgroup (Table 1 row 1, minimal
    cost 28) is handed to the per-chunk path inside a batched call; its
    result equals rei_solve's, and a small instance in the same call still
    equals the oracle."""
    t = golden["table1_row1"]
    small = instances.single_instance(0, (1, 1, 1, 1, 1))
    big = rei.Instance(t["alphabet"], t["pos"], t["neg"], (1, 1, 1, 1, 1), 30, 8 << 30)
    h = rei.Instance(small.alphabet, small.pos, small.neg, small.costs, small.max_cost)
    print("\nbatch: Table 1 row 1 + single seed 0", flush=True)
    rb, rs = rei.solve_batch([big, h])
    alone = big.solve()
    key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)
    assert key(rb) == key(alone)
    assert (rb.status, rb.cost) == ("OK", 28)
    check_against_oracle(rs, (small.alphabet, small.pos, small.neg, small.costs, small.max_cost))
    big.close()
    h.close()


@pytest.mark.parametrize("level_max", [1, 300, 5000])
def test_batch_handoff_resumes_exactly(rei, level_max):
    """Instances handed to the per-chunk path at a level boundary continue
    with the levels the workgroup stored (rows, back-pointers, table); the
    results equal the oracle's for every hand-off level, word width and
    table form."""
    specs = batch_specs()[::3]
    for seed in (3, 6):
        i = instances.single_instance(seed, (1, 1, 5, 1, 2))
        specs.append((i.alphabet, i.pos, i.neg, i.costs, i.max_cost))
    print(f"\nbatch of {len(specs)} instances, hand-off above {level_max} candidates", flush=True)
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    for h in hs:
        h.set_batch_level(level_max)
    res = rei.solve_batch(hs)
    for r, spec in zip(res, specs):
        check_against_oracle(r, spec)
    for h in hs:
        h.close()


@pytest.mark.parametrize("us", [0, 1, 200])
def test_batch_time_handoff_is_exact(rei, us):
    """Hand-off on time (rei_set_batch_time): 1 us moves every instance at its
    first level above 4096 candidates, 0 never on time, 200 wherever the
    clock says; the results equal the oracle's whatever the hand-off level."""
    specs = batch_specs()[::3]
    for seed in (3, 6, 9):
        i = instances.single_instance(seed, (1, 1, 5, 1, 2))
        specs.append((i.alphabet, i.pos, i.neg, i.costs, i.max_cost))
    print(f"\nbatch of {len(specs)} instances, hand-off after {us} us", flush=True)
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    for h in hs:
        h.set_batch_time(us)
    res = rei.solve_batch(hs)
    for r, spec in zip(res, specs):
        check_against_oracle(r, spec)
    for h in hs:
        h.close()


# ---- OnTheFly mode (Sec. 3) ----

def _otf_cases():
    cases = []
    for seed in (1, 3, 4, 6, 8):
        it = instances.single_instance(seed, (1, 1, 1, 1, 1))
        for costs in ((1, 1, 1, 1, 1), (1, 3, 3, 3, 3), (2, 5, 5, 5, 5), (1, 1, 5, 1, 2)):
            full = oracle.solve(it.alphabet, it.pos, it.neg, costs, 40, 1 << 40, 0, 8)
            total = sum(full.unique)
            for frac in (0.3, 0.8):
                cases.append((it, costs, max(1, int(total * frac))))
    return cases


@pytest.mark.parametrize("chunk", [0, 100])
def test_on_the_fly_parity(rei, chunk):
    """The cache fills mid-level (in a chunk of its own with chunk=100, inside
    one large chunk otherwise); the rest of that level and the later levels
    whose blocks use complete levels run on the fly.  Status, cost, regex and
    per-level counts equal the oracle's OnTheFly search."""
    n_ok = n_oom = 0
    for it, costs, cap in _otf_cases():
        h = rei.Instance(it.alphabet, it.pos, it.neg, costs, 40, 1 << 30)
        probe = h.solve()
        words = probe.cs_words
        h.close()
        cache = cap * (8 * words + 8)
        print(f"\nOnTheFly seed-instance costs {costs} cap {cap} rows chunk {chunk}", flush=True)
        h = rei.Instance(it.alphabet, it.pos, it.neg, costs, 40, cache)
        h.set_on_the_fly(True)
        if chunk:
            h.set_chunk(chunk)
        g = h.solve()
        o = oracle.solve(it.alphabet, it.pos, it.neg, costs, 40, cap, 0, 8, on_the_fly=True)
        assert (g.status, g.cost, g.regex) == (o.status, o.cost, o.regex), (costs, cap, g, o)
        for c in range(41):
            assert g.unique_at(c) == o.unique[c], (c, g.unique, o.unique)
            assert g.candidates_at(c) == o.candidates[c], (c, g.candidates, o.candidates)
        n_ok += g.status == "OK"
        n_oom += g.status == "OUT_OF_MEMORY"
        h.close()
    assert n_ok > 5 and n_oom > 5


def test_on_the_fly_in_a_batch_runs_on_the_grid(rei):
    it = instances.single_instance(3, (1, 1, 1, 1, 1))
    costs = (1, 3, 3, 3, 3)
    full = oracle.solve(it.alphabet, it.pos, it.neg, costs, 40, 1 << 40, 0, 8)
    cap = sum(full.unique) // 2
    h = rei.Instance(it.alphabet, it.pos, it.neg, costs, 40, cap * (8 * 2 + 8))
    h.set_on_the_fly(True)
    other = rei.Instance(it.alphabet, it.pos, it.neg, (1, 1, 1, 1, 1), it.max_cost)
    rb, _ = rei.solve_batch([h, other])
    o = oracle.solve(it.alphabet, it.pos, it.neg, costs, 40, cap, 0, 8, on_the_fly=True)
    assert (rb.status, rb.cost, rb.regex) == (o.status, o.cost, o.regex)
    h.close()
    other.close()


# ---- per-character costs ----

def _char_cost_cases():
    cases = []
    for seed in range(6):
        it = instances.single_instance(seed, (1, 1, 1, 1, 1))
        for cc in ((1, 2), (3, 1), (2, 2)):
            cases.append((it.alphabet, it.pos, it.neg, (1, 1, 1, 1, 1), cc))
    for it in instances.batched_instances(7, 12):
        k = len(it.alphabet)
        cc = tuple(1 + (i * 2) % 3 for i in range(k))
        cases.append((it.alphabet, it.pos, it.neg, (1, 1, 2, 1, 1), cc))
    return cases


def test_per_character_costs_parity(rei):
    """Characters enter at the level of their own cost; results (status,
    cost, regex, per-level counts) equal the oracle's, also inside a batched
    call (such instances run on the per-chunk path there)."""
    cases = _char_cost_cases()
    hs = []
    for a, p, n, costs, cc in cases:
        print(f"\nper-character costs {cc} alphabet {a!r}", flush=True)
        h = rei.Instance(a, p, n, costs, 30)
        h.set_char_costs(cc)
        hs.append(h)
    single = [h.solve() for h in hs]
    batched = rei.solve_batch(hs)
    for (a, p, n, costs, cc), g, b in zip(cases, single, batched):
        o = oracle.solve(a, p, n, costs, 30, 1 << 40, 0, 8, char_costs=list(cc))
        assert (g.status, g.cost, g.regex) == (o.status, o.cost, o.regex), (cc, g, o)
        assert g.first_level == min(cc)
        for c in range(31):
            assert g.unique_at(c) == o.unique[c], (c, g.unique, o.unique)
            assert g.candidates_at(c) == o.candidates[c], (c, g.candidates, o.candidates)
        assert (b.status, b.cost, b.regex, b.unique, b.candidates) == (g.status, g.cost, g.regex, g.unique,
                                                                        g.candidates)
    for h in hs:
        h.close()


# ---- the paper's benchmark generators under its twelve cost functions ----

def test_paper_generators_all_cost_functions(rei):
    """Small Type 1 and Type 2 instances (Sec. 4, Benchmark Construction)
    under each of the twelve cost functions: the GPU equals the oracle."""
    cases = [instances.type1_instance(s, p=5, n=5, le=4) for s in range(3)]
    cases += [instances.type2_instance(s, p=6, n=6, le=5) for s in range(2)]
    for it in cases:
        for costs in instances.PAPER_COST_FUNCTIONS:
            print(f"\n{it.kind} {it.meta} costs {costs}", flush=True)
            g = rei.solve(it.alphabet, it.pos, it.neg, costs, max_cost=1000)
            o = oracle.solve(it.alphabet, it.pos, it.neg, costs, 1000, 1 << 40, 0, 8)
            assert (g.status, g.cost, g.regex) == (o.status, o.cost, o.regex), (costs, g, o)
            for c in range(0, g.cost + 1):
                assert g.unique_at(c) == o.unique[c] and g.candidates_at(c) == o.candidates[c], c


def test_trim_frees_and_resolves(rei):
    """rei_trim frees the last search's device memory; the result stays, the
    rows are gone (inspection refuses), and the next solve is identical."""
    it = instances.single_instance(3, (1, 1, 5, 1, 2))
    h = rei.Instance(it.alphabet, it.pos, it.neg, it.costs, it.max_cost)
    a = h.solve()
    assert h.level_size(a.first_level) > 0
    h.trim()
    assert h.level_size(a.first_level) == 0
    with pytest.raises(rei.ReiError):
        h.row_bits(a.first_level, 0, a.cs_words)
    b = h.solve()
    assert (a.status, a.cost, a.regex, a.unique, a.candidates) == (b.status, b.cost, b.regex, b.unique,
                                                                    b.candidates)
    h.close()


def test_tuned_launch_shapes_give_identical_results(rei):
    """Every workgroup size the tuner tries gives the same results; the
    tuner returns one size per word-width group present."""
    specs = batch_specs()[::2]
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    before = rei.solve_batch(hs)
    tuned = rei.tune_batch(hs)
    shape = tuned["threads_per_instance"]
    assert shape and all(t in (256, 512, 1024) for t in shape.values())
    assert set(tuned["level_max"]) == set(shape)
    assert all(v in (0, 1 << 8, 1 << 10) or 1 << 12 <= v <= 1 << 19 for v in tuned["level_max"].values())
    assert len({v for v in tuned["level_max"].values() if v}) <= 1  # one size, or 0 for small groups
    after = rei.solve_batch(hs)
    key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)
    assert [key(r) for r in before] == [key(r) for r in after]
    for r, spec in zip(after, specs):
        check_against_oracle(r, spec)
    for h in hs:
        h.close()


def test_large_batch_equals_per_instance_solves(rei):
    """2500 instances: the groups are large enough that the launch gives each
    instance 256 or 512 threads; every result equals the instance's own
    rei_solve (the per-chunk path, parity-tested against the oracle)."""
    xs = instances.batched_instances(3, 2500)
    print(f"\nbatch of {len(xs)} instances", flush=True)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, 1 << 30) for i in xs]
    batched = rei.solve_batch(hs)
    key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)
    for h, b in zip(hs, batched):
        assert key(h.solve()) == key(b)
    for h in hs:
        h.close()


def test_kernel_statistics(rei):
    """Profiling level 1 times the generators (units = candidates, summing to
    the result's candidate counts); level 2 adds the other classes; enabling
    clears the statistics, disabling keeps them."""
    it = instances.single_instance(6, (1, 1, 1, 1, 1))
    h = rei.Instance(it.alphabet, it.pos, it.neg, it.costs, it.max_cost)
    classes = rei.KERNEL_CLASSES
    h.set_profiling(True, level=1)
    r = h.solve()
    h.set_profiling(False)
    stats = {c: h.kernel_stats(k) for k, c in enumerate(classes)}
    gen_units = sum(stats[c][2] for c in classes if c.startswith("gen_"))
    assert gen_units >= sum(r.candidates)  # chunks enqueued past the answer count too
    assert all(stats[c][1] > 0 for c in classes if c.startswith("gen_") and stats[c][0])
    assert stats["insert_survivors"][0] == 0 and stats["compact_winners"][0] == 0
    h.set_profiling(True, level=2)
    h.solve()
    stats2 = {c: h.kernel_stats(k) for k, c in enumerate(classes)}
    assert stats2["insert_survivors"][0] > 0 and stats2["compact_winners"][0] > 0
    assert sum(stats2[c][2] for c in classes if c.startswith("gen_")) == gen_units
    h.close()


def test_profiling_one_class(rei):
    """rei_set_profiling_class times the launches of one class only (the
    same count as level 2 gives that class); a batch's launches are
    counted on its first instance; results are unchanged; a class outside
    the enumeration is refused."""
    it = instances.single_instance(6, (1, 1, 1, 1, 1))
    h = rei.Instance(it.alphabet, it.pos, it.neg, it.costs, it.max_cost)
    classes = rei.KERNEL_CLASSES
    h.set_profiling(True, level=2)
    ref = h.solve()
    full = {c: h.kernel_stats(k) for k, c in enumerate(classes)}
    timed = [c for c in ("gen_concat", "gen_pieces", "insert_survivors") if full[c][0] > 0]
    assert len(timed) >= 2
    for c in timed:
        h.set_profiling_class(c)
        r = h.solve()
        h.set_profiling(False)
        got = {q: h.kernel_stats(k) for k, q in enumerate(classes)}
        assert got[c][0] == full[c][0] > 0
        assert all(got[q][0] == 0 for q in classes if q != c)
        assert (r.status, r.cost, r.regex, r.unique, r.candidates) == (ref.status, ref.cost, ref.regex,
                                                                        ref.unique, ref.candidates)
    with pytest.raises(rei.ReiError):
        h.set_profiling_class(len(classes))
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost) for i in instances.batched_instances(0, 16)]
    hs[0].set_profiling_class("solve_batch")
    rei.solve_batch(hs)
    n, ms, units = hs[0].kernel_stats(classes.index("solve_batch"))
    assert n >= 1 and ms > 0 and units > 0
    assert hs[0].kernel_stats(classes.index("gen_concat"))[0] == 0
    for x in hs + [h]:
        x.close()


def test_timing_overhead_is_measured(rei):
    us = rei.timing_overhead_us()
    assert 0.0 < us < 1000.0


@pytest.mark.parametrize("bits", [6, 12])
def test_weak_hash_gives_identical_results(rei, bits):
    """With only the low bits of the hash kept, languages collide in the
    table, every fingerprint is equal (each probe compares whole languages)
    and probe sequences grow long; the results still equal the oracle's on
    the per-chunk path, in the batched solver and with OnTheFly mode."""
    rei.set_hash_bits(bits)
    try:
        print(f"\nhash bits {bits}", flush=True)
        for seed in range(0, 200, 25):
            inst = instances.plain_instance(seed)
            run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, chunk=50)
        if bits >= 12:  # 124 K rows: with 64 start positions the probes would walk them all
            inst = instances.single_instance(6, (1, 1, 1, 1, 1))
            run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, rows=True, row_limit=32)
        specs = batch_specs()[:40]
        hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
        for r, spec in zip(rei.solve_batch(hs), specs):
            check_against_oracle(r, spec)
        for h in hs:
            h.close()
    finally:
        rei.set_hash_bits(0)


def test_caller_allocator_gives_identical_results(rei):
    """rei_set_allocator: with device memory from torch's caching allocator the
    per-chunk path, a batch and its hand-offs (allocating from worker threads)
    give the results of hipMalloc'd memory, and every allocation comes back."""
    import torch
    specs = batch_specs()[::4]
    key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)

    def run():
        hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
        single = [key(h.solve()) for h in hs]
        for h in hs:
            h.set_batch_level(300)
        batch = [key(r) for r in rei.solve_batch(hs)]
        for h in hs:
            h.close()
        return single, batch

    ref = run()
    live, calls = {}, [0, 0]

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n, 0)
        calls[0] += 1
        live[p] = n
        return p

    def free(p):
        calls[1] += 1
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    print(f"\n{len(specs)} instances, torch caching allocator", flush=True)
    rei.set_allocator(alloc, free)
    try:
        got = run()
    finally:
        rei.set_allocator(None, None)
    assert got == ref
    assert calls[0] > len(specs) and calls[0] == calls[1] and not live
    with pytest.raises(ValueError):
        rei.set_allocator(alloc, None)


def test_concurrent_batched_calls(rei):
    """Two threads call rei_solve_batch at once on disjoint instance sets
    whose instances hand off early: the calls share the process's hand-off
    workers and stream pools, and each gets the results of a call alone."""
    import threading
    specs = batch_specs()[::4]
    key = lambda r: (r.status, r.cost, r.regex, r.unique, r.candidates)
    sets = [[rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs] for _ in range(2)]
    for hs in sets:
        for h in hs:
            h.set_batch_level(300)
    alone = [[key(r) for r in rei.solve_batch(hs)] for hs in sets]
    assert alone[0] == alone[1]
    got = [None, None]
    errors = []

    def run(k):
        try:
            for _ in range(3):
                got[k] = [key(r) for r in rei.solve_batch(sets[k])]
        except Exception as e:  # reported below, on the test's thread
            errors.append(e)

    print(f"\ntwo threads x {len(specs)} instances", flush=True)
    ts = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    assert got[0] == alone[0] and got[1] == alone[1]
    for hs in sets:
        for h in hs:
            h.close()


def test_batch_all_4096_equal_oracle(rei):
    """The batched configuration at full size: all 4096 instances (master seed
    0) in one rei_solve_batch call, every result compared with the oracle's
    (the oracle runs across instances on host threads)."""
    from oracle_runs import mismatch, solve_many
    specs = instances.batched_instances(0, 4096)
    cache = 1 << 30
    want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs],
                      workers=8, threads=1)
    print("\ncase: 4096 batched instances, one rei_solve_batch call", flush=True)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs]
    got = rei.solve_batch(hs)
    bad = [(k, mismatch(g, o, specs[k].max_cost)) for k, (g, o) in enumerate(zip(got, want))
           if mismatch(g, o, specs[k].max_cost) is not None]
    assert not bad, bad[:5]
    for h in hs:
        h.close()


@pytest.mark.parametrize("seed,max_cost,row_limit", [(0, 11, 64), (1, 10, 64), (2, 9, None)])
def test_wide_spec_32_words(rei, seed, max_cost, row_limit):
    """32 words per language (1219-1234 infixes: twenty plus twenty ternary
    strings of length at most 12): every constructor kernel at its widest
    instantiation.  Counts and status against the oracle; rows of every level
    compared bit by bit (all of them for seed 2)."""
    inst = instances.wide_instance(seed, max_cost)
    g, _ = run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, max_cost, 4 << 30,
                    rows=True, row_limit=row_limit)
    assert g.cs_words == 32 and g.ic_size == inst.meta["n_ic"]


def test_wide_spec_32_words_chunked(rei):
    """The 32-word path with tiny chunks (every chunk boundary inside a
    concatenation block) gives the same results."""
    inst = instances.wide_instance(3, 8)
    g, _ = run_both(rei, inst.alphabet, inst.pos, inst.neg, inst.costs, 8, 4 << 30, chunk=777, rows=True)
    assert g.cs_words == 32


def _graph_specs():
    """Batched instances of every word width, plus one that cannot be batched
    (16 words) and the two trivial specifications."""
    specs = instances.batched_instances(5, 300)
    big = instances.large_instance(2)
    big.max_cost = 7
    specs.append(big)
    specs.append(instances.Instance("01", [], ["0"], kind="trivial", max_cost=12))
    specs.append(instances.Instance("012", [""], ["1", "22"], kind="trivial", max_cost=12))
    return specs


@pytest.mark.parametrize("arena", [0, 1 << 16])
def test_batch_graph_replays_equal_oracle(rei, arena):
    """A captured batch replayed three times, with eager work of the program
    between the replays (another batched solve, a synchronisation): every
    replay's results equal the oracle's.  With a 64 KiB arena many instances
    outgrow their rows on the first replay, finish on the per-chunk path and
    get an arena that fits before the next replay."""
    import torch
    from oracle_runs import mismatch, solve_many
    specs = _graph_specs()
    cache = 1 << 30
    want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs], workers=8, threads=1)
    print(f"\ncase: graph of {len(specs)} instances, arena {arena}", flush=True)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs]
    g = rei.BatchGraph(hs, arena)
    others = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache)
              for i in instances.batched_instances(6, 40)]
    for rep in range(3):
        print(f"replay {rep}", flush=True)
        got = g.run()
        bad = [(k, mismatch(a, o, specs[k].max_cost)) for k, (a, o) in enumerate(zip(got, want))
               if mismatch(a, o, specs[k].max_cost) is not None]
        assert not bad, (rep, bad[:5])
        rei.solve_batch(others)
        torch.cuda.synchronize()
    g.close()
    for h in hs + others:
        h.close()


def test_batch_graph_4096_equal_oracle(rei):
    """The batched configuration at full size through the captured graph: all
    4096 instances (master seed 0) per replay, two replays, every result
    equal to the oracle's."""
    from oracle_runs import mismatch, solve_many
    specs = instances.batched_instances(0, 4096)
    cache = 1 << 30
    want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs],
                      workers=8, threads=1)
    print("\ncase: 4096 batched instances through the graph", flush=True)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs]
    g = rei.BatchGraph(hs)
    for rep in range(2):
        got = g.run()
        bad = [(k, mismatch(a, o, specs[k].max_cost)) for k, (a, o) in enumerate(zip(got, want))
               if mismatch(a, o, specs[k].max_cost) is not None]
        assert not bad, (rep, bad[:5])
    g.close()
    for h in hs:
        h.close()


@pytest.mark.parametrize("level_max", [0, 1 << 12])
def test_batch_16_and_32_words_equal_oracle(rei, level_max):
    """The one-workgroup solver at its widest instantiations: the large
    configuration's seeds 0-3 (8-16 words) and three 32-word specifications,
    in one rei_solve_batch call (with the default hand-off, and with levels
    over 4096 candidates handed to the per-chunk path), against the oracle."""
    from oracle_runs import mismatch, solve_many
    specs = [instances.large_instance(s) for s in range(4)] + [instances.wide_instance(s, 9) for s in range(3)]
    cache = 64 << 30
    want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs], workers=4, threads=4)
    print(f"\ncase: large 0-3 + wide 0-2 batched, level_max {level_max}", flush=True)
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, cache) for i in specs]
    if level_max:
        for h in hs:
            h.set_batch_level(level_max)
    got = rei.solve_batch(hs)
    for k, (g, o) in enumerate(zip(got, want)):
        assert mismatch(g, o, specs[k].max_cost) is None, (k, mismatch(g, o, specs[k].max_cost))
    assert {g.cs_words for g in got} >= {16, 32}
    for h in hs:
        h.close()


@pytest.mark.parametrize("first,cmax,wg,xi", [(1 << 10, 1 << 12, 64, 4), (1 << 18, 1 << 20, 8192, 64),
                                              (3, 1000, 512, 1)])
def test_grid_tuning_parameters_give_identical_results(rei, first, cmax, wg, xi):
    """Every launch shape the grid tuner may pick (and odd ones) gives the
    oracle's results: a 4-word single instance and a 16-word large one."""
    for inst in (instances.single_instance(3, (1, 1, 5, 1, 2)), instances.large_instance(0)):
        print(f"\ncase: {inst.kind} seed {inst.seed} first {first} max {cmax} wg {wg} xi {xi}", flush=True)
        h = rei.Instance(inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, 64 << 30)
        h.set_grid_tuning(first, cmax, wg, xi)
        g = h.solve()
        from oracle_runs import mismatch, solve_many
        o = solve_many([(inst.alphabet, inst.pos, inst.neg, inst.costs, inst.max_cost, 64 << 30)])[0]
        assert mismatch(g, o, inst.max_cost) is None, mismatch(g, o, inst.max_cost)
        h.close()


def test_grid_tuner_runs_and_keeps_results(rei, tmp_path):
    """rei_tune_grid picks parameters per word width; solves afterwards (which
    use the table) still equal the oracle's; the table survives a save/load."""
    from oracle_runs import mismatch, solve_many
    specs = [instances.large_instance(s) for s in (0, 2)] + [instances.single_instance(s) for s in (3, 5)]
    hs = [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, 64 << 30) for i in specs]
    chosen = rei.tune_grid(hs)
    print(f"\ntuned: {chosen}", flush=True)
    assert set(chosen) == {f"W{h.solve().cs_words}" for h in hs}
    rei.tune_save(str(tmp_path / "t.json"))
    rei.tune_load(str(tmp_path / "t.json"))
    want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, 64 << 30) for i in specs])
    for k, (h, o) in enumerate(zip(hs, want)):
        g = h.solve()
        assert mismatch(g, o, specs[k].max_cost) is None, (k, mismatch(g, o, specs[k].max_cost))
        h.close()


def test_width_sent_to_per_chunk_path_equals_oracle(rei, tmp_path):
    """A word width whose tuned hand-off size is 0 skips the one-workgroup
    solver: rei_solve_batch and the server run its instances on the
    per-chunk path from the start (the tuning file sets it, as rei_tune_batch
    would); every result equals the oracle's.  The default sizes are put back
    afterwards."""
    from paper_2305_18575_amd import serving
    specs = batch_specs()[::3]
    hs = [rei.Instance(a, p, n, c, m) for (a, p, n, c, m) in specs]
    widths = sorted({h.solve().cs_words for h in hs})
    print(f"\nwidths {widths}, {len(hs)} instances", flush=True)
    groups = [0] + [w for w in widths]  # group 0: one word with keys in the table slots
    zero = tmp_path / "zero.json"
    zero.write_text('{"batch_level_max": [' + ", ".join(f'{{"group": {g}, "level_max": 0}}' for g in groups)
                    + ']}\n')
    back = tmp_path / "back.json"
    back.write_text('{"batch_level_max": [' + ", ".join(f'{{"group": {g}, "level_max": 65536}}' for g in groups)
                    + ']}\n')
    rei.tune_load(str(zero))
    try:
        got = rei.solve_batch(hs)
        for r, spec in zip(got, specs):
            check_against_oracle(r, spec)
        srv = rei.Server(64 << 30, 64, 2, 2)
        tickets = [srv.submit(h) for h in hs]
        served = [srv.wait(t)[0] for t in tickets]
        srv.close()
        for k, (a, b) in enumerate(zip(served, got)):
            assert serving.same(a, b), (k, a, b)
    finally:
        rei.tune_load(str(back))
    for h in hs:
        h.close()
