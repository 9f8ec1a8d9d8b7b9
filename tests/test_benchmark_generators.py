"""The paper's benchmark generators (Sec. 4, Benchmark Construction)."""
import collections

from paper_2305_18575_amd import instances


def _check(inst, p, n, le):
    assert len(inst.pos) == p and len(inst.neg) == n
    assert len(set(inst.pos)) == p and len(set(inst.neg)) == n
    assert not set(inst.pos) & set(inst.neg)
    assert all(len(w) <= le and set(w) <= set(inst.alphabet) for w in inst.pos + inst.neg)


def test_type1_defaults_and_determinism():
    for seed in range(40):
        a = instances.type1_instance(seed)
        b = instances.type1_instance(seed)
        assert (a.pos, a.neg, a.meta) == (b.pos, b.neg, b.meta)
        m = a.meta
        assert 8 <= m["p"] <= 12 and 8 <= m["n"] <= 12 and 0 <= m["le"] <= 7
        assert 2 ** (m["le"] + 1) - 1 >= m["p"] + m["n"]
        _check(a, m["p"], m["n"], m["le"])


def test_type2_defaults_and_determinism():
    for seed in range(40):
        a = instances.type2_instance(seed)
        b = instances.type2_instance(seed)
        assert (a.pos, a.neg, a.meta) == (b.pos, b.neg, b.meta)
        m = a.meta
        assert 7 <= m["p"] <= 14 and 7 <= m["n"] <= 14 and 0 <= m["le"] <= 10
        _check(a, m["p"], m["n"], m["le"])


def test_type1_is_dominated_by_long_strings():
    """Uniform over all strings of length <= le: a length k string is drawn
    with probability 2^k / (2^(le+1) - 1)."""
    cnt = collections.Counter()
    for seed in range(300):
        a = instances.type1_instance(seed, p=5, n=5, le=6)
        cnt.update(len(w) for w in a.pos + a.neg)
    total = sum(cnt.values())
    for k in range(7):
        expect = total * 2 ** k / 127
        assert abs(cnt[k] - expect) <= 4 * expect ** 0.5 + 3, (k, cnt[k], expect)


def test_type2_gives_lengths_equal_chances():
    """Each length 0..le is drawn with equal probability (while it has unused
    strings): with le = 6 and 10 examples, lengths 2..6 never run out, so
    each gets about 1/7 of the draws; lengths 0 and 1 hold 1 and 2 strings
    and get fewer."""
    cnt = collections.Counter()
    for seed in range(300):
        a = instances.type2_instance(seed, p=5, n=5, le=6)
        cnt.update(len(w) for w in a.pos + a.neg)
    assert cnt[0] <= 300 and cnt[1] <= 600
    mids = [cnt[k] for k in range(2, 7)]
    assert max(mids) - min(mids) <= 0.2 * max(mids), cnt
    # the empty word is in most Type 2 specifications: 1 - (6/7)^10 = 0.79
    assert cnt[0] > 200


def test_paper_cost_functions():
    assert len(instances.PAPER_COST_FUNCTIONS) == 12
    assert len(set(instances.PAPER_COST_FUNCTIONS)) == 12
    assert all(len(c) == 5 and min(c) >= 1 for c in instances.PAPER_COST_FUNCTIONS)
