"""rei_solve_batch_noalloc: the batched search run in the library's static
device array (for callers that cannot allocate), against rei_solve_batch (the
entry point it is a variant of) and the oracle, exactly, on two calls in a
row, the second with fewer instances (larger shares, every arena moved)."""
import pytest

from oracle_runs import mismatch, solve_many
from paper_2305_18575_amd import instances

pytestmark = pytest.mark.gpu

CACHE = 1 << 30


def key(r):
    return (r.status, r.cost, r.regex, r.unique, r.candidates, r.ic_size, r.cs_words)


def handles(rei, specs):
    return [rei.Instance(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, CACHE) for i in specs]


def test_noalloc_equals_batched_entry_point(rei):
    wide16 = instances.large_instance(0)
    wide16.max_cost = 8
    wide32 = instances.wide_instance(3, 8)
    trivial = instances.Instance("01", [], ["0"], kind="trivial", max_cost=12)
    first = instances.batched_instances(0, 40) + [wide16, trivial]
    second = instances.batched_instances(0, 56)[40:] + [wide32]
    for name, specs in (("first", first), ("second", second)):
        print(f"\ncase: {name} call, {len(specs)} instances", flush=True)
        a, b = handles(rei, specs), handles(rei, specs)
        got = rei.solve_batch_noalloc(a)
        ref = rei.solve_batch(b)
        assert [key(x) for x in got] == [key(y) for y in ref]
        want = solve_many([(i.alphabet, i.pos, i.neg, i.costs, i.max_cost, CACHE) for i in specs],
                          workers=8, threads=1)
        for k, (g, o) in enumerate(zip(got, want)):
            assert mismatch(g, o, specs[k].max_cost) is None, (name, k, mismatch(g, o, specs[k].max_cost))
        assert {g.cs_words for g in got} >= ({16} if name == "first" else {32})
        # the rows lived in the shared array: not kept for inspection
        k = next(k for k, g in enumerate(got) if g.status == "OK" and g.unique)
        with pytest.raises(rei.ReiError):
            a[k].row_bits(got[k].first_level, 0, got[k].cs_words)
        # solved again another way, the instance holds its rows once more
        again = a[k].solve()
        assert key(again) == key(got[k])
        a[k].row_bits(got[k].first_level, 0, got[k].cs_words)
        for h in a + b:
            h.close()


def test_noalloc_rejects_what_does_not_fit(rei):
    specs = instances.batched_instances(0, 65)
    hs = handles(rei, specs)
    with pytest.raises(rei.ReiError) as e:
        rei.solve_batch_noalloc(hs)
    assert "64" in str(e.value)
    otf = hs[0]
    otf.set_on_the_fly(True)
    with pytest.raises(rei.ReiError):
        rei.solve_batch_noalloc([otf])
    for h in hs:
        h.close()
