"""Independent checkers for the oracle: brute force over expression trees.

Nothing here shares code with the oracle or the GPU library.  A tree's
language is decided on the strings themselves with the relational semantics
of regular expressions: for a string s, an expression denotes the relation
M(i, j) = "s[i:j] is in the language" between positions 0..|s|, with
  char a   M(i, i+1) = [s[i] == a]
  x?       M_x or identity
  x*       reflexive-transitive closure of M_x
  x.y      boolean product M_x M_y
  x+y      M_x or M_y
and s is accepted iff M(0, |s|).  All strings are handled at once as a batch
of (L+1) x (L+1) boolean matrices; numpy's matmul is the product.
"""
from __future__ import annotations

import re
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def ic_of(strings: Sequence[str]) -> List[str]:
    """All substrings of the given strings."""
    out = set()
    for w in strings:
        for i in range(len(w) + 1):
            for j in range(i, len(w) + 1):
                out.add(w[i:j])
    return sorted(out, key=lambda s: (len(s), s))


class Matcher:
    """Relational-semantics evaluator over a fixed list of strings."""

    def __init__(self, words: Sequence[str]):
        self.words = list(words)
        self.n = len(self.words)
        self.L = max([len(w) for w in self.words] + [0])
        P = self.L + 1
        self.lens = np.array([len(w) for w in self.words], dtype=np.int64)
        self.eye = np.broadcast_to(np.eye(P, dtype=bool), (self.n, P, P)).copy()
        self._chars: Dict[str, np.ndarray] = {}

    def char(self, a: str) -> np.ndarray:
        if a not in self._chars:
            P = self.L + 1
            m = np.zeros((self.n, P, P), dtype=bool)
            for s, w in enumerate(self.words):
                for i, ch in enumerate(w):
                    if ch == a:
                        m[s, i, i + 1] = True
            self._chars[a] = m
        return self._chars[a]

    @staticmethod
    def prod(x: np.ndarray, y: np.ndarray) -> np.ndarray:
        return np.matmul(x.astype(np.uint8), y.astype(np.uint8)) > 0

    def question(self, x):
        return x | self.eye

    def star(self, x):
        t = x | self.eye
        while True:
            t2 = self.prod(t, t)
            if np.array_equal(t2, t):
                return t
            t = t2

    def concat(self, x, y):
        return self.prod(x, y)

    @staticmethod
    def union(x, y):
        return x | y

    def accepted(self, m) -> np.ndarray:
        return m[np.arange(self.n), 0, self.lens]

    # printed syntax: union '+', juxtaposition, postfix ? and *, parentheses
    def parse(self, printed: str):
        s, pos = printed, 0

        def union():
            nonlocal pos
            v = concat()
            while pos < len(s) and s[pos] == '+':
                pos += 1
                v = self.union(v, concat())
            return v

        def concat():
            nonlocal pos
            v = post()
            while pos < len(s) and s[pos] not in '+)?*':
                v = self.concat(v, post())
            return v

        def post():
            nonlocal pos
            v = atom()
            while pos < len(s) and s[pos] in '?*':
                v = self.question(v) if s[pos] == '?' else self.star(v)
                pos += 1
            return v

        def atom():
            nonlocal pos
            ch = s[pos]
            pos += 1
            if ch == '(':
                v = union()
                assert s[pos] == ')'
                pos += 1
                return v
            if ch == 'ε':
                return self.eye.copy()
            if ch == '∅':
                return np.zeros_like(self.eye)
            return self.char(ch)

        v = union()
        assert pos == len(s), printed
        return v


def language_on(printed: str, words: Sequence[str]) -> frozenset:
    """The words (from ``words``) that the printed expression accepts."""
    m = Matcher(words)
    acc = m.accepted(m.parse(printed))
    return frozenset(w for w, a in zip(words, acc) if a)


def to_pyre(printed: str) -> str:
    """Printed syntax to Python ``re`` syntax (for cross-checks on small,
    non-degenerate expressions)."""
    out = []
    for ch in printed:
        if ch == '(':
            out.append('(?:')
        elif ch == ')':
            out.append(')')
        elif ch == '+':
            out.append('|')
        elif ch in '?*':
            out.append(ch)
        elif ch == 'ε':
            out.append('(?:)')
        elif ch == '∅':
            out.append('(?!)')
        else:
            out.append(re.escape(ch))
    return ''.join(out)


def regex_cost(printed: str, costs=(1, 1, 1, 1, 1), char_costs=None) -> int:
    """Cost of a printed expression under the cost homomorphism (c1..c5);
    ``char_costs`` maps characters to their own costs (default c1)."""
    c1, c2, c3, c4, c5 = costs
    s = printed
    pos = 0

    def union():
        nonlocal pos
        v = concat()
        while pos < len(s) and s[pos] == '+':
            pos += 1
            v = v + concat() + c5
        return v

    def concat():
        nonlocal pos
        v = post()
        while pos < len(s) and s[pos] not in '+)?*':
            v = v + post() + c4
        return v

    def post():
        nonlocal pos
        v = atom()
        while pos < len(s) and s[pos] in '?*':
            v += c2 if s[pos] == '?' else c3
            pos += 1
        return v

    def atom():
        nonlocal pos
        if s[pos] == '(':
            pos += 1
            v = union()
            assert s[pos] == ')'
            pos += 1
            return v
        pos += 1
        return char_costs.get(s[pos - 1], c1) if char_costs else c1

    v = union()
    assert pos == len(s), printed
    return v


def brute_levels(sigma: str, pos: Sequence[str], neg: Sequence[str], costs, kmax: int,
                 max_errors: int = 0, char_costs=None):
    """Enumerate every expression tree of cost <= kmax over sigma with ?, *,
    concatenation and union, evaluate it on the substrings of the examples,
    and return (number of distinct languages whose cheapest tree costs c, for
    each c; minimal cost of a tree that misclassifies at most ``max_errors``
    examples, or None)."""
    c1, c2, c3, c4, c5 = costs
    words = ic_of(list(pos) + list(neg))
    m = Matcher(words)
    widx = {w: i for i, w in enumerate(words)}
    pi = np.array([widx[w] for w in pos], dtype=np.int64)
    ni = np.array([widx[w] for w in neg], dtype=np.int64)
    by: Dict[int, List[np.ndarray]] = {k: [] for k in range(kmax + 1)}
    first: Dict[bytes, int] = {}
    cstar: Optional[int] = None
    for k in range(1, kmax + 1):
        lst = by[k]
        lst.extend(m.char(a) for a in sigma if (char_costs[a] if char_costs else c1) == k)
        if k - c2 >= 1:
            lst.extend(m.question(x) for x in by[k - c2])
        if k - c3 >= 1:
            lst.extend(m.star(x) for x in by[k - c3])
        for a in range(1, k - c4):
            for x in by[a]:
                for y in by[k - c4 - a]:
                    lst.append(m.concat(x, y))
        for a in range(1, k - c5):
            for x in by[a]:
                for y in by[k - c5 - a]:
                    lst.append(m.union(x, y))
        for t in lst:
            acc = m.accepted(t)
            key = np.packbits(acc).tobytes()
            if key not in first:
                first[key] = k
            if cstar is None:
                bad = int((~acc[pi]).sum() + acc[ni].sum()) if len(pi) + len(ni) else 0
                if bad <= max_errors:
                    cstar = k
    counts: Dict[int, int] = {}
    for k in first.values():
        counts[k] = counts.get(k, 0) + 1
    return counts, cstar
