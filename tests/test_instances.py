"""Seeded input generators: determinism and the target-membership automaton."""
import re

import numpy as np

from paper_2305_18575_amd import instances as I
from paper_2305_18575_amd import serving


def test_generators_are_deterministic():
    assert I.plain_instance(5) == I.plain_instance(5)
    assert I.single_instance(3, (1, 1, 5, 1, 2)) == I.single_instance(3, (1, 1, 5, 1, 2))
    a, b = I.batched_instances(1, 6), I.batched_instances(1, 6)
    assert a == b


def test_membership_automaton_matches_re():
    # python's re on small, shallow targets agrees with the Thompson automaton
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(200):
        sigma = "012"[: int(rng.integers(2, 4))]
        ast = I.random_ast(rng, sigma, int(rng.integers(1, 8)))
        pat = re.compile(I.ast_to_pyre(ast))
        want = [w for w in I.words(sigma, 0, 5) if pat.fullmatch(w)]
        assert I.language_members(ast, sigma, 0, 5) == want


def test_instances_respect_their_shapes():
    for s in range(5):
        i = I.plain_instance(s)
        assert len(i.pos) == 4 and len(i.neg) == 4
        assert all(1 <= len(w) <= 5 for w in i.pos + i.neg)
        assert not set(i.pos) & set(i.neg)
        assert I.n_infixes(i.pos + i.neg) <= 63
        j = I.single_instance(s)
        assert len(j.pos) == 10 and len(j.neg) == 10 and I.n_infixes(j.pos + j.neg) <= 255
    k = I.large_instance(2)
    assert len(k.pos) == 20 and I.n_infixes(k.pos + k.neg) <= 2048
    for b in I.batched_instances(0, 10):
        assert 2 <= len(b.alphabet) <= 4 and I.n_infixes(b.pos + b.neg) <= 512


def test_serving_mix_and_arrivals():
    specs = serving.request_mix(0, 50)
    kinds = [k for k, _, _ in specs]
    assert set(kinds) <= {"plain", "large", "single"}
    arr = serving.poisson_arrivals(0, 1000, 100.0)
    assert np.all(np.diff(arr) > 0)
    assert abs(1000 / arr[-1] - 100.0) < 15.0
