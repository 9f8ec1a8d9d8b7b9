"""CPU oracle for search-based regular expression inference.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never calls into it and shares no code with it.

The computation lives in ``rei_oracle.cpp`` (plain C++17, one byte per word of
the infix closure, definitional split matcher on strings); this module only
compiles it with g++ and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rei_oracle.cpp")
_LIB = os.path.join(_HERE, "librei_oracle.so")

STATUS = {0: "OK", 1: "NOT_FOUND", 2: "OUT_OF_MEMORY", -1: "INVALID_ARG",
          -2: "INCONSISTENT", -3: "BAD_CHAR"}


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/librei_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, ip, cp = ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p
    ll, ull_p = ctypes.c_longlong, ctypes.POINTER(ctypes.c_ulonglong)
    strarr = ctypes.POINTER(ctypes.c_char_p)
    lib.oracle_create.restype = vp
    lib.oracle_create.argtypes = [cp, strarr, ip, strarr, ip, ctypes.POINTER(ip), ip,
                                  ll, ip, ip, ctypes.POINTER(ip)]
    lib.oracle_solve.argtypes = [vp]
    lib.oracle_set_on_the_fly.argtypes = [vp, ip]
    lib.oracle_set_on_the_fly.restype = None
    lib.oracle_set_char_costs.argtypes = [vp, ctypes.POINTER(ip), ip]
    lib.oracle_set_char_costs.restype = ip
    lib.oracle_destroy.argtypes = [vp]
    for name in ("oracle_status", "oracle_cost", "oracle_ic_size", "oracle_max_cost"):
        getattr(lib, name).argtypes = [vp]
    lib.oracle_regex.argtypes = [vp]
    lib.oracle_regex.restype = cp
    lib.oracle_ic_word.argtypes = [vp, ip]
    lib.oracle_ic_word.restype = cp
    lib.oracle_level_counts.argtypes = [vp, ull_p, ull_p]
    lib.oracle_num_rows.argtypes = [vp]
    lib.oracle_num_rows.restype = ll
    lib.oracle_row_level.argtypes = [vp, ll]
    lib.oracle_level_size.argtypes = [vp, ip]
    lib.oracle_level_size.restype = ll
    lib.oracle_level_row.argtypes = [vp, ip, ll]
    lib.oracle_level_row.restype = ll
    lib.oracle_row_cs.argtypes = [vp, ll, ctypes.c_char_p]
    lib.oracle_row_regex.argtypes = [vp, ll]
    lib.oracle_row_regex.restype = cp
    lib.oracle_cs_of_regex.argtypes = [vp, cp, ctypes.c_char_p]
    lib.oracle_last_error.argtypes = [vp]
    lib.oracle_last_error.restype = cp
    _lib = lib
    return lib


def _strarr(items: Sequence[str]):
    arr = (ctypes.c_char_p * max(1, len(items)))()
    for i, s in enumerate(items):
        arr[i] = s.encode("latin-1")
    return arr


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{STATUS.get(status, status)} {msg}")
        self.status = status


@dataclass
class OracleResult:
    status: str
    cost: int
    regex: str
    unique: List[int]        # index = cost level, 0..max_cost
    candidates: List[int]
    ic_size: int


class Oracle:
    """One specification, staged.  ``solve()`` runs the bottom-up search."""

    def __init__(self, alphabet: str, pos: Sequence[str], neg: Sequence[str],
                 costs=(1, 1, 1, 1, 1), max_cost: int = 30,
                 row_cap: int = 1 << 40, max_errors: int = 0, threads: int = 1,
                 on_the_fly: bool = False, char_costs: Optional[Sequence[int]] = None):
        lib = _load()
        st = ctypes.c_int(0)
        c = (ctypes.c_int * 5)(*costs)
        self._h = lib.oracle_create(alphabet.encode("latin-1"), _strarr(pos), len(pos),
                                    _strarr(neg), len(neg), c, int(max_cost), int(row_cap),
                                    int(max_errors), int(threads), ctypes.byref(st))
        if not self._h:
            raise OracleError(st.value)
        lib.oracle_set_on_the_fly(self._h, 1 if on_the_fly else 0)
        self._lib = lib
        if char_costs is not None:
            arr = (ctypes.c_int * max(1, len(char_costs)))(*char_costs)
            if lib.oracle_set_char_costs(self._h, arr, len(char_costs)) != 0:
                raise OracleError(-1, "bad per-character costs")
        self.max_cost = int(max_cost)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_destroy(h)
            self._h = None

    @property
    def ic(self) -> List[str]:
        n = self._lib.oracle_ic_size(self._h)
        return [self._lib.oracle_ic_word(self._h, i).decode("latin-1") for i in range(n)]

    def solve(self) -> OracleResult:
        lib = self._lib
        st = lib.oracle_solve(self._h)
        m = self.max_cost + 1
        u = (ctypes.c_ulonglong * m)()
        cd = (ctypes.c_ulonglong * m)()
        lib.oracle_level_counts(self._h, u, cd)
        return OracleResult(STATUS[st], lib.oracle_cost(self._h),
                            lib.oracle_regex(self._h).decode("utf-8"),
                            list(u), list(cd), lib.oracle_ic_size(self._h))

    # --- cache inspection (after solve) ---
    def num_rows(self) -> int:
        return self._lib.oracle_num_rows(self._h)

    def level_size(self, c: int) -> int:
        return self._lib.oracle_level_size(self._h, c)

    def level_row(self, c: int, i: int) -> int:
        return self._lib.oracle_level_row(self._h, c, i)

    def row_level(self, r: int) -> int:
        return self._lib.oracle_row_level(self._h, r)

    def row_cs(self, r: int) -> bytes:
        n = self._lib.oracle_ic_size(self._h)
        buf = ctypes.create_string_buffer(max(1, n))
        self._lib.oracle_row_cs(self._h, r, buf)
        return buf.raw[:n]

    def row_regex(self, r: int) -> str:
        return self._lib.oracle_row_regex(self._h, r).decode("utf-8")

    def cs_of_regex(self, text: str) -> Optional[bytes]:
        n = self._lib.oracle_ic_size(self._h)
        buf = ctypes.create_string_buffer(max(1, n))
        rc = self._lib.oracle_cs_of_regex(self._h, text.encode("utf-8"), buf)
        return None if rc != 0 else buf.raw[:n]


def solve(alphabet, pos, neg, costs=(1, 1, 1, 1, 1), max_cost=30, row_cap=1 << 40,
          max_errors=0, threads=1, on_the_fly=False, char_costs=None) -> OracleResult:
    return Oracle(alphabet, pos, neg, costs, max_cost, row_cap, max_errors, threads,
                  on_the_fly, char_costs).solve()
