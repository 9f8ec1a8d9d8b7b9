"""Algebraic laws of the constructors on characteristic sequences
(Definition of infix power series: union is idempotent, commutative and
associative; concatenation is associative and distributes over union; eps
is its unit; r* is the least fixed point of Y = eps + r Y), checked on the
oracle's constructors for random expressions, each CS also compared with
the relational matcher of tests/brute.py run directly on the words."""
import numpy as np

import brute
from paper_2305_18575_amd import instances


def _setup(oracle_mod, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    words = ["".join("01"[int(b)] for b in rng.integers(0, 2, size=int(rng.integers(0, 7))))
             for _ in range(6)]
    words = list(dict.fromkeys(words))
    o = oracle_mod.Oracle("01", words[:3], words[3:] or ["111111"])
    exprs = [instances.ast_to_text(instances.random_ast(rng, "01", int(rng.integers(1, 7))))
             for _ in range(3)]
    return o, exprs


def test_constructor_laws(oracle_mod):
    checked = 0
    for seed in range(40):
        o, (x, y, z) = _setup(oracle_mod, seed)
        cs = o.cs_of_regex
        ic = o.ic
        # every CS is the language on ic of an independent matcher
        for e in (x, y, z, f"({x})({y})", f"({x})*", f"({x}+{y})?"):
            got = cs(e)
            lang = brute.language_on(e, ic)
            assert got == bytes(1 if w in lang else 0 for w in ic), e
        laws = [
            (f"{x}+{y}", f"{y}+{x}"),
            (f"({x}+{y})+{z}", f"{x}+({y}+{z})"),
            (f"{x}+{x}", f"{x}"),
            (f"(({x})({y}))({z})", f"({x})(({y})({z}))"),
            (f"({x})({y}+{z})", f"({x})({y})+({x})({z})"),
            (f"({y}+{z})({x})", f"({y})({x})+({z})({x})"),
            (f"ε({x})", f"{x}"),
            (f"({x})ε", f"{x}"),
            (f"({x})*", f"ε+({x})({x})*"),
            (f"(({x})*)*", f"({x})*"),
            (f"({x})?", f"ε+{x}"),
            (f"({x})*({x})*", f"({x})*"),
        ]
        for a, b in laws:
            assert cs(a) == cs(b), (a, b)
            checked += 1
    assert checked == 40 * 12
