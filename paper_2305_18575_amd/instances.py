"""Seeded synthetic REI instances (specifications (P, N) over an alphabet).

This module holds no part of the inference method itself: it only draws
inputs.  Both the GPU path and the CPU oracle are fed from here, so it must
stay free of the language-cache / characteristic-sequence arithmetic.

Recipe (the paper's own instance files are not available; these stand in):

* A target regular expression is drawn uniformly among all expressions of a
  drawn cost, over the grammar  a | r? | r* | r.r | r+r  with unit costs
  (cost homomorphism (1,1,1,1,1), Definition of cost homomorphism, Sec. 3).
  Uniformity comes from a counting table over costs.
* Positive examples are drawn uniformly without replacement from the target's
  language restricted to the length window; negative examples from the
  complement in the same window.  Membership is decided by a Thompson
  automaton of the target, determinised on the fly while walking all strings
  of the window (a textbook construction, independent of both
  implementations under test, with no backtracking).
* If either side is too small, or the instance breaks a size bound, the
  target is redrawn from the same random stream.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import itertools
import re
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# AST nodes are tuples: ('c', ch) | ('?', x) | ('*', x) | ('.', x, y) | ('+', x, y)


def _ast_counts(nsym: int, kmax: int) -> List[int]:
    """Number of ASTs of each exact cost 0..kmax under unit costs."""
    cnt = [0] * (kmax + 1)
    for k in range(1, kmax + 1):
        if k == 1:
            cnt[k] = nsym
            continue
        pair = sum(cnt[a] * cnt[k - 1 - a] for a in range(1, k - 1))
        cnt[k] = 2 * cnt[k - 1] + 2 * pair
    return cnt


def random_ast(rng: np.random.Generator, sigma: str, cost: int):
    """Uniformly random AST of exactly ``cost`` under unit costs."""
    cnt = _ast_counts(len(sigma), cost)

    def draw(k):
        if k == 1:
            return ('c', sigma[int(rng.integers(len(sigma)))])
        total = cnt[k]
        r = int(rng.integers(total))
        # unary: '?' then '*'
        if r < cnt[k - 1]:
            return ('?', draw(k - 1))
        r -= cnt[k - 1]
        if r < cnt[k - 1]:
            return ('*', draw(k - 1))
        r -= cnt[k - 1]
        for op in ('.', '+'):
            for a in range(1, k - 1):
                b = k - 1 - a
                block = cnt[a] * cnt[b]
                if r < block:
                    return (op, draw(a), draw(b))
                r -= block
        raise AssertionError("unreachable")

    return draw(cost)


def ast_to_pyre(ast) -> str:
    """Translate an AST into Python ``re`` syntax (non-capturing groups)."""
    t = ast[0]
    if t == 'c':
        return re.escape(ast[1])
    if t == '?':
        return '(?:' + ast_to_pyre(ast[1]) + ')?'
    if t == '*':
        return '(?:' + ast_to_pyre(ast[1]) + ')*'
    if t == '.':
        return '(?:' + ast_to_pyre(ast[1]) + ')(?:' + ast_to_pyre(ast[2]) + ')'
    if t == '+':
        return '(?:' + ast_to_pyre(ast[1]) + '|' + ast_to_pyre(ast[2]) + ')'
    raise ValueError(t)


def ast_to_text(ast) -> str:
    t = ast[0]
    if t == 'c':
        return ast[1]
    if t in '?*':
        return '(' + ast_to_text(ast[1]) + ')' + t
    if t == '.':
        return '(' + ast_to_text(ast[1]) + ast_to_text(ast[2]) + ')'
    return '(' + ast_to_text(ast[1]) + '+' + ast_to_text(ast[2]) + ')'


class _Nfa:
    """Thompson automaton of an AST: epsilon moves and character moves."""

    def __init__(self, ast):
        self.eps: List[List[int]] = []
        self.move: List[dict] = []
        self.start, self.accept = self._build(ast)

    def _state(self) -> int:
        self.eps.append([])
        self.move.append({})
        return len(self.eps) - 1

    def _build(self, ast):
        t = ast[0]
        if t == 'c':
            a, b = self._state(), self._state()
            self.move[a][ast[1]] = b
            return a, b
        if t in '?*':
            rs, ra = self._build(ast[1])
            a, b = self._state(), self._state()
            self.eps[a] += [rs, b]
            self.eps[ra].append(b)
            if t == '*':
                self.eps[ra].append(rs)
            return a, b
        ls, la = self._build(ast[1])
        rs, ra = self._build(ast[2])
        if t == '.':
            self.eps[la].append(rs)
            return ls, ra
        a, b = self._state(), self._state()
        self.eps[a] += [ls, rs]
        self.eps[la].append(b)
        self.eps[ra].append(b)
        return a, b

    def closure(self, states) -> frozenset:
        out, stack = set(states), list(states)
        while stack:
            q = stack.pop()
            for r in self.eps[q]:
                if r not in out:
                    out.add(r)
                    stack.append(r)
        return frozenset(out)


def language_members(ast, sigma: str, lo: int, hi: int) -> List[str]:
    """Strings of length lo..hi (length-major, alphabet order) in the
    target's language."""
    nfa = _Nfa(ast)
    trans = {}

    def step(S, a):
        k = (S, a)
        if k not in trans:
            trans[k] = nfa.closure({nfa.move[q][a] for q in S if a in nfa.move[q]})
        return trans[k]

    level = {"": nfa.closure({nfa.start})}
    out = []
    for n in range(0, hi + 1):
        if n >= lo:
            out.extend(w for w in level if nfa.accept in level[w])
        if n == hi:
            break
        nxt = {}
        for w, S in level.items():
            for a in sigma:
                nxt[w + a] = step(S, a)
        level = nxt
    return out


def words(sigma: str, lo: int, hi: int) -> List[str]:
    """All strings over ``sigma`` with length in [lo, hi], length-major order."""
    out = []
    for n in range(lo, hi + 1):
        out.extend(''.join(p) for p in itertools.product(sigma, repeat=n))
    return out


def n_infixes(strings) -> int:
    """Size of the set of all substrings (used only as a rejection bound)."""
    s = set()
    for w in strings:
        for i in range(len(w) + 1):
            for j in range(i, len(w) + 1):
                s.add(w[i:j])
    return len(s)


@dataclass
class Instance:
    alphabet: str
    pos: List[str]
    neg: List[str]
    target: str = ""              # target regex in readable form (provenance only)
    target_cost: int = 0
    seed: int = 0
    kind: str = ""
    costs: Tuple[int, int, int, int, int] = (1, 1, 1, 1, 1)
    max_cost: int = 30
    meta: dict = field(default_factory=dict)


def _draw_spec(rng, sigma, cost_lo, cost_hi, npos, nneg, len_lo, len_hi,
               max_ic: Optional[int], universe=None):
    universe = universe if universe is not None else words(sigma, len_lo, len_hi)
    while True:
        cost = int(rng.integers(cost_lo, cost_hi + 1))
        ast = random_ast(rng, sigma, cost)
        members = set(language_members(ast, sigma, len_lo, len_hi))
        inl = [w for w in universe if w in members]
        outl = [w for w in universe if w not in members]
        if len(inl) < npos or len(outl) < nneg:
            continue
        pi = rng.choice(len(inl), size=npos, replace=False)
        ni = rng.choice(len(outl), size=nneg, replace=False)
        pos = sorted(inl[int(i)] for i in pi)
        neg = sorted(outl[int(i)] for i in ni)
        if max_ic is not None and n_infixes(pos + neg) > max_ic:
            continue
        return ast, cost, pos, neg


def plain_instance(seed: int) -> Instance:
    """Small single instance: Sigma={0,1}, target cost 1..8, 4+4 strings of
    length 1..5 (at most 63 distinct infixes, one 64-bit word per language)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ast, cost, pos, neg = _draw_spec(rng, "01", 1, 8, 4, 4, 1, 5, 63)
    return Instance("01", pos, neg, ast_to_text(ast), cost, seed, "plain",
                    (1, 1, 1, 1, 1), 30)


def single_instance(seed: int, costs=(1, 1, 1, 1, 1)) -> Instance:
    """Single instance: Sigma={0,1}, target cost 10..14 (unit costs), 10+10
    strings of length 0..7 (at most 255 distinct infixes, four 64-bit words).
    ``max_cost`` is the target's cost under ``costs``: the target is precise,
    so the answer never costs more."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ast, cost, pos, neg = _draw_spec(rng, "01", 10, 14, 10, 10, 0, 7, 255)
    return Instance("01", pos, neg, ast_to_text(ast), cost, seed, "single",
                    tuple(costs), ast_cost(ast, costs))


def large_instance(seed: int) -> Instance:
    """Large single instance: Sigma={0,1,2}, target cost 14..18, 20+20 strings
    of length 0..10, at most 2048 distinct infixes (32 words)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ast, cost, pos, neg = _draw_spec(rng, "012", 14, 18, 20, 20, 0, 10, 2048)
    return Instance("012", pos, neg, ast_to_text(ast), cost, seed, "large",
                    (1, 1, 1, 1, 1), cost)


def wide_instance(seed: int, max_cost: int = 11) -> Instance:
    """A specification wide enough for 32 words per language (1025..2048
    infixes): twenty positive and twenty negative ternary strings drawn as the
    paper's Type 1 benchmarks are (distinct strings uniform among all strings
    of length at most 12, the first twenty positive).  Twenty plus twenty
    ternary strings of length at most 10 (the large configuration) have at
    most 961 distinct infixes, so that configuration never reaches this
    width.  Seeds 0..3 give 1219..1234 infixes.  Random strings share little
    structure, so the minimal expression is expensive: ``max_cost`` bounds
    the search (NOT_FOUND below the answer's cost)."""
    it = type1_instance(seed, p=20, n=20, le=12, sigma="012", max_cost=max_cost)
    n = n_infixes(it.pos + it.neg)
    if not 1024 < n <= 2048:
        raise ValueError(f"seed {seed}: {n} infixes, not a 32-word specification")
    it.kind = "wide"
    it.meta["n_ic"] = n
    return it


def batched_instances(master_seed: int, count: int) -> List[Instance]:
    """Many small uneven instances: |Sigma| in {2,3,4}, 2..16 positive and
    2..16 negative strings of length 0..6, target cost 4..12, at most 512
    distinct infixes."""
    mrng = np.random.Generator(np.random.PCG64(master_seed))
    seeds = mrng.integers(0, 2**63 - 1, size=count)
    out = []
    universes = {}
    for s in seeds:
        rng = np.random.Generator(np.random.PCG64(int(s)))
        k = int(rng.integers(2, 5))
        sigma = "0123"[:k]
        npos = int(rng.integers(2, 17))
        nneg = int(rng.integers(2, 17))
        if sigma not in universes:
            universes[sigma] = words(sigma, 0, 6)
        ast, cost, pos, neg = _draw_spec(rng, sigma, 4, 12, npos, nneg, 0, 6,
                                         512, universes[sigma])
        out.append(Instance(sigma, pos, neg, ast_to_text(ast), cost, int(s),
                            "batched", (1, 1, 1, 1, 1), cost))
    return out


# The twelve cost functions (c1..c5) of the paper's measurements (Table 1 and
# the cost-function comparison of Sec. 4).
PAPER_COST_FUNCTIONS = [
    (1, 1, 1, 1, 1), (10, 1, 1, 1, 1), (1, 10, 1, 1, 1), (1, 1, 10, 1, 1),
    (1, 1, 1, 10, 1), (1, 1, 1, 1, 10), (10, 10, 10, 10, 1), (10, 10, 10, 1, 10),
    (10, 10, 1, 10, 10), (10, 1, 10, 10, 10), (1, 10, 10, 10, 10), (20, 20, 20, 5, 30),
]


def type1_instance(seed: int, p: Optional[int] = None, n: Optional[int] = None,
                   le: Optional[int] = None, sigma: str = "01",
                   costs=(1, 1, 1, 1, 1), max_cost: int = 1000) -> Instance:
    """Type 1 benchmark (Sec. 4, Benchmark Construction): P and N are drawn
    uniformly among pairs of disjoint sets of p and n strings of length at
    most le, i.e. p + n distinct strings drawn uniformly without replacement
    from all such strings, the first p positive.  Most strings are long.
    Unset parameters are drawn as in the paper's main benchmarks: p and n in
    8..12, le in 0..7 (le is drawn again while fewer than p + n strings of
    length <= le exist)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = int(rng.integers(8, 13)) if p is None else p
    n = int(rng.integers(8, 13)) if n is None else n
    fixed_le = le is not None
    while True:
        le_v = le if fixed_le else int(rng.integers(0, 8))
        universe = words(sigma, 0, le_v)
        if len(universe) >= p + n:
            break
        if fixed_le:
            raise ValueError(f"only {len(universe)} strings of length <= {le_v}")
    idx = rng.choice(len(universe), size=p + n, replace=False)
    chosen = [universe[int(i)] for i in idx]
    return Instance(sigma, sorted(chosen[:p]), sorted(chosen[p:]), "", 0, seed, "type1",
                    tuple(costs), max_cost, {"p": p, "n": n, "le": le_v})


def type2_instance(seed: int, p: Optional[int] = None, n: Optional[int] = None,
                   le: Optional[int] = None, sigma: str = "01",
                   costs=(1, 1, 1, 1, 1), max_cost: int = 1000) -> Instance:
    """Type 2 benchmark (Sec. 4, Benchmark Construction): every length
    0..le has the same chance of occurring.  Each example's length is drawn
    uniformly from 0..le, then the string uniformly among the strings of that
    length not drawn yet (a length with none left is drawn again); the p
    positive examples first, then the n negative ones.  Short strings such as
    the empty word are therefore common.  Unset parameters are drawn as in
    the paper's main benchmarks: p and n in 7..14, le in 0..10 (le is drawn
    again while fewer than p + n strings of length <= le exist)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = int(rng.integers(7, 15)) if p is None else p
    n = int(rng.integers(7, 15)) if n is None else n
    fixed_le = le is not None
    while True:
        le_v = le if fixed_le else int(rng.integers(0, 11))
        if (len(sigma) ** (le_v + 1) - 1) // max(1, len(sigma) - 1) >= p + n or (
                len(sigma) == 1 and le_v + 1 >= p + n):
            break
        if fixed_le:
            raise ValueError(f"fewer than {p + n} strings of length <= {le_v}")
    by_len = [words(sigma, k, k) for k in range(le_v + 1)]
    used = set()
    chosen = []
    while len(chosen) < p + n:
        k = int(rng.integers(0, le_v + 1))
        free = [w for w in by_len[k] if w not in used]
        if not free:
            continue
        w = free[int(rng.integers(len(free)))]
        used.add(w)
        chosen.append(w)
    return Instance(sigma, sorted(chosen[:p]), sorted(chosen[p:]), "", 0, seed, "type2",
                    tuple(costs), max_cost, {"p": p, "n": n, "le": le_v})


def ast_cost(ast, costs) -> int:
    c1, c2, c3, c4, c5 = costs
    t = ast[0]
    if t == 'c':
        return c1
    if t == '?':
        return ast_cost(ast[1], costs) + c2
    if t == '*':
        return ast_cost(ast[1], costs) + c3
    if t == '.':
        return ast_cost(ast[1], costs) + ast_cost(ast[2], costs) + c4
    return ast_cost(ast[1], costs) + ast_cost(ast[2], costs) + c5


def row_cap(cache_bytes: int, n_ic: int) -> int:
    """Rows that fit ``cache_bytes``: each row is one language bitvector of
    W 64-bit words (W = smallest power of two with 64*W >= n_ic) plus one
    64-bit back-pointer word."""
    w = 1
    while 64 * w < n_ic:
        w *= 2
    return cache_bytes // (8 * w + 8)
