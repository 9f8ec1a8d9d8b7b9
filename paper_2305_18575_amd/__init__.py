"""Python binding of the MI355X regular-expression-inference library.

Argument marshalling only: every step of the search runs in ``librei.so``
(host staging in C++, the search in HIP kernels).  The names follow the C ABI
declared in ``include/rei.h``.  PyTorch, when present, only supplies the HIP
stream the search is launched on.

If the library has not been built this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librei.so")

STATUS = {0: "OK", 1: "NOT_FOUND", 2: "OUT_OF_MEMORY", -1: "INVALID_ARG",
          -2: "INCONSISTENT", -3: "BAD_CHAR", -4: "TOO_LARGE", -5: "DEVICE",
          -6: "HOST_ALLOC"}

KERNEL_CLASSES = ["gen_char", "gen_question", "gen_star", "gen_concat", "gen_union",
                  "insert_survivors", "compact_winners", "other", "solve_batch", "gen_pieces"]

# exported symbols, as declared in include/rei.h
EXPORTS = ["rei_create", "rei_solve", "rei_solve_batch", "rei_tune_batch", "rei_server_create", "rei_server_submit",
           "rei_server_poll", "rei_server_destroy", "rei_set_allocator", "rei_trim", "rei_destroy", "rei_status_str", "rei_last_error",
           "rei_create_error", "rei_ic_word", "rei_level_size", "rei_row_bits",
           "rei_row_regex", "rei_set_chunk", "rei_set_batch_level", "rei_set_batch_time", "rei_set_on_the_fly", "rei_set_char_costs", "rei_set_max_errors", "rei_set_profiling", "rei_set_profiling_class",
           "rei_kernel_stats", "rei_timing_overhead", "rei_set_hash_bits", "rei_kernel_name",
           "rei_measure_peak", "rei_batch_graph_create", "rei_batch_graph_launch", "rei_batch_graph_results",
           "rei_batch_graph_error", "rei_batch_graph_destroy", "rei_tune_grid", "rei_set_grid_tuning",
           "rei_tune_save", "rei_tune_load", "rei_solve_batch_noalloc", "rei_server_set_queue_mode",
           "rei_batch_graph_outside"]


class ReiError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.status_name = STATUS.get(status, str(status))


class _Costs(ctypes.Structure):
    _fields_ = [("c_char", ctypes.c_uint32), ("c_question", ctypes.c_uint32),
                ("c_star", ctypes.c_uint32), ("c_concat", ctypes.c_uint32),
                ("c_union", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cost", ctypes.c_uint32),
                ("regex", ctypes.c_char_p), ("first_level", ctypes.c_uint32),
                ("n_levels", ctypes.c_uint32),
                ("unique_per_level", ctypes.POINTER(ctypes.c_uint64)),
                ("candidates_per_level", ctypes.POINTER(ctypes.c_uint64)),
                ("total_unique", ctypes.c_uint64), ("ic_size", ctypes.c_uint32),
                ("cs_words", ctypes.c_uint32), ("seconds_stage", ctypes.c_double),
                ("seconds_solve", ctypes.c_double)]


_lib = None


def load_library():
    """Load ``librei.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2305_18575_amd._build")
    # torch ships its own HIP runtime with the same soname; loading it first
    # makes librei.so bind to that one, so the process has a single runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, cp = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_char_p
    strarr = ctypes.POINTER(ctypes.c_char_p)
    lib.rei_create.restype = ctypes.c_int
    lib.rei_create.argtypes = [cp, strarr, ctypes.c_size_t, strarr, ctypes.c_size_t, _Costs,
                               u32, u64, ctypes.POINTER(vp)]
    lib.rei_solve.restype = ctypes.c_int
    lib.rei_solve.argtypes = [vp, vp, ctypes.POINTER(_Result)]
    lib.rei_solve_batch.restype = ctypes.c_int
    lib.rei_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, vp, u64,
                                    ctypes.POINTER(_Result)]
    lib.rei_tune_batch.restype = ctypes.c_int
    lib.rei_solve_batch_noalloc.restype = ctypes.c_int
    lib.rei_solve_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, vp, ctypes.POINTER(_Result)]
    lib.rei_tune_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, vp, u64, ctypes.POINTER(u32),
                                   ctypes.POINTER(u64)]
    lib.rei_server_create.restype = ctypes.c_int
    lib.rei_server_create.argtypes = [u64, u32, u32, u32, ctypes.POINTER(vp)]
    lib.rei_server_submit.restype = ctypes.c_int
    lib.rei_server_submit.argtypes = [vp, vp, ctypes.POINTER(u64)]
    lib.rei_server_poll.restype = ctypes.c_int
    lib.rei_server_poll.argtypes = [vp, u64, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(_Result), ctypes.POINTER(ctypes.c_double)]
    lib.rei_server_destroy.restype = None
    lib.rei_server_destroy.argtypes = [vp]
    lib.rei_batch_graph_outside.restype = ctypes.c_size_t
    lib.rei_batch_graph_outside.argtypes = [vp]
    lib.rei_server_set_queue_mode.restype = ctypes.c_int
    lib.rei_server_set_queue_mode.argtypes = [vp, ctypes.c_int]
    lib.rei_destroy.restype = None
    lib.rei_destroy.argtypes = [vp]
    lib.rei_trim.restype = ctypes.c_int
    lib.rei_trim.argtypes = [vp]
    lib.rei_status_str.restype = cp
    lib.rei_status_str.argtypes = [ctypes.c_int]
    lib.rei_last_error.restype = cp
    lib.rei_last_error.argtypes = [vp]
    lib.rei_create_error.restype = cp
    lib.rei_create_error.argtypes = []
    lib.rei_ic_word.restype = ctypes.c_int
    lib.rei_ic_word.argtypes = [vp, u32, cp, ctypes.c_size_t]
    lib.rei_level_size.restype = ctypes.c_int
    lib.rei_level_size.argtypes = [vp, u32, ctypes.POINTER(u64)]
    lib.rei_row_bits.restype = ctypes.c_int
    lib.rei_row_bits.argtypes = [vp, u32, u64, ctypes.POINTER(u64)]
    lib.rei_row_regex.restype = ctypes.c_int
    lib.rei_row_regex.argtypes = [vp, u32, u64, cp, ctypes.c_size_t]
    lib.rei_set_chunk.restype = ctypes.c_int
    lib.rei_set_chunk.argtypes = [vp, u64]
    lib.rei_set_batch_level.restype = ctypes.c_int
    lib.rei_set_batch_level.argtypes = [vp, u64]
    lib.rei_set_on_the_fly.restype = ctypes.c_int
    lib.rei_set_on_the_fly.argtypes = [vp, ctypes.c_int]
    lib.rei_set_char_costs.restype = ctypes.c_int
    lib.rei_set_char_costs.argtypes = [vp, ctypes.POINTER(u32), ctypes.c_size_t]
    lib.rei_set_max_errors.restype = ctypes.c_int
    lib.rei_set_max_errors.argtypes = [vp, u32]
    lib.rei_set_profiling.restype = ctypes.c_int
    lib.rei_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.rei_kernel_stats.restype = ctypes.c_int
    lib.rei_kernel_stats.argtypes = [vp, ctypes.c_int, ctypes.POINTER(u64),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]
    lib.rei_set_hash_bits.restype = ctypes.c_int
    lib.rei_set_hash_bits.argtypes = [u32]
    lib.rei_timing_overhead.restype = ctypes.c_int
    lib.rei_timing_overhead.argtypes = [ctypes.POINTER(ctypes.c_double)]
    lib.rei_kernel_name.restype = cp
    lib.rei_set_profiling_class.restype = ctypes.c_int
    lib.rei_set_profiling_class.argtypes = [vp, ctypes.c_int]
    lib.rei_set_batch_time.restype = ctypes.c_int
    lib.rei_set_batch_time.argtypes = [vp, ctypes.c_int64]
    lib.rei_set_allocator.restype = ctypes.c_int
    lib.rei_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    lib.rei_kernel_name.argtypes = [ctypes.c_int]
    lib.rei_batch_graph_create.restype = ctypes.c_int
    lib.rei_batch_graph_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, u64, ctypes.POINTER(vp)]
    lib.rei_batch_graph_launch.restype = ctypes.c_int
    lib.rei_batch_graph_launch.argtypes = [vp, vp]
    lib.rei_batch_graph_results.restype = ctypes.c_int
    lib.rei_batch_graph_results.argtypes = [vp, ctypes.POINTER(_Result)]
    lib.rei_batch_graph_error.restype = cp
    lib.rei_batch_graph_error.argtypes = [vp]
    lib.rei_batch_graph_destroy.restype = None
    lib.rei_batch_graph_destroy.argtypes = [vp]
    lib.rei_tune_grid.restype = ctypes.c_int
    lib.rei_tune_grid.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, vp, ctypes.POINTER(u64)]
    lib.rei_set_grid_tuning.restype = ctypes.c_int
    lib.rei_set_grid_tuning.argtypes = [vp, u64, u64, u32, u32]
    lib.rei_tune_save.restype = ctypes.c_int
    lib.rei_tune_save.argtypes = [cp]
    lib.rei_tune_load.restype = ctypes.c_int
    lib.rei_tune_load.argtypes = [cp]
    lib.rei_measure_peak.restype = ctypes.c_int
    lib.rei_measure_peak.argtypes = [ctypes.c_int, u64, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def _strarr(items: Sequence[str]):
    arr = (ctypes.c_char_p * max(1, len(items)))()
    for i, s in enumerate(items):
        arr[i] = s.encode("latin-1")
    return arr


def current_stream_handle() -> Optional[int]:
    """hipStream_t of torch's current stream (None = null stream)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # torch absent or not built with HIP
        pass
    return None


@dataclass
class Result:
    status: str
    cost: int
    regex: str
    first_level: int
    unique: List[int]          # per level, first_level .. first_level + n_levels - 1
    candidates: List[int]
    total_unique: int
    ic_size: int
    cs_words: int
    seconds_stage: float
    seconds_solve: float

    def unique_at(self, cost: int) -> int:
        i = cost - self.first_level
        return self.unique[i] if 0 <= i < len(self.unique) else 0

    def candidates_at(self, cost: int) -> int:
        i = cost - self.first_level
        return self.candidates[i] if 0 <= i < len(self.candidates) else 0


class Instance:
    """One staged specification (``rei_create``); ``solve`` runs ``rei_solve``."""

    def __init__(self, alphabet: str, pos: Sequence[str], neg: Sequence[str],
                 costs=(1, 1, 1, 1, 1), max_cost: int = 30, cache_bytes: int = 1 << 30):
        lib = load_library()
        self._lib = lib
        self._h = None
        # memory from a Python allocator is given back through Python: not
        # possible while the interpreter shuts down (the process frees it)
        self._py_alloc = _py_allocator_active
        h = ctypes.c_void_p()
        st = lib.rei_create(alphabet.encode("latin-1"), _strarr(pos), len(pos),
                            _strarr(neg), len(neg), _Costs(*costs), int(max_cost),
                            int(cache_bytes), ctypes.byref(h))
        if st != 0:
            raise ReiError(st, lib.rei_create_error().decode())
        self._h = h
        self.costs = tuple(costs)
        self.max_cost = int(max_cost)

    def close(self):
        if self._h:
            self._lib.rei_destroy(self._h)
            self._h = None

    def __del__(self):
        if getattr(self, "_py_alloc", False) and sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _result(self, r) -> "Result":
        n = r.n_levels
        return Result(STATUS[r.status], r.cost, (r.regex or b"").decode("utf-8"), r.first_level,
                      r.unique_per_level[:n] if n else [], r.candidates_per_level[:n] if n else [],
                      r.total_unique, r.ic_size, r.cs_words, r.seconds_stage, r.seconds_solve)

    def _check(self, st):
        if st != 0:
            raise ReiError(st, self._lib.rei_last_error(self._h).decode())

    def solve(self, stream: Optional[int] = -1) -> Result:
        """Run the search on ``stream`` (-1 = torch's current stream)."""
        if stream == -1:
            stream = current_stream_handle()
        r = _Result()
        self._check(self._lib.rei_solve(self._h, ctypes.c_void_p(stream or 0), ctypes.byref(r)))
        return self._result(r)

    # ---- tuning / measurement ----
    def set_chunk(self, max_candidates: int):
        self._check(self._lib.rei_set_chunk(self._h, int(max_candidates)))

    def trim(self):
        """Free the device memory of the last search (``rei_trim``)."""
        self._check(self._lib.rei_trim(self._h))

    def set_char_costs(self, costs: Sequence[int]):
        """Per-character costs, one per alphabet character in alphabet order."""
        arr = (ctypes.c_uint32 * max(1, len(costs)))(*costs)
        self._check(self._lib.rei_set_char_costs(self._h, arr, len(costs)))

    def set_on_the_fly(self, enable: bool = True):
        """OnTheFly mode: keep searching, precision only, once the cache is full."""
        self._check(self._lib.rei_set_on_the_fly(self._h, 1 if enable else 0))

    def set_batch_level(self, max_candidates: int):
        """Largest level the batched solver keeps on one workgroup (0 = default)."""
        self._check(self._lib.rei_set_batch_level(self._h, int(max_candidates)))

    def set_batch_time(self, microseconds: int):
        """Workgroup time after which larger levels move to the per-chunk path
        (-1 = default, 0 = never on time)."""
        self._check(self._lib.rei_set_batch_time(self._h, int(microseconds)))

    def set_grid_tuning(self, first_chunk: int = 0, chunk_max: int = 0, concat_wg: int = 0, concat_xi: int = 0):
        """Per-chunk path launch parameters of this instance (0 = tuned or default)."""
        self._check(self._lib.rei_set_grid_tuning(self._h, int(first_chunk), int(chunk_max), int(concat_wg),
                                                  int(concat_xi)))

    def set_max_errors(self, k: int):
        self._check(self._lib.rei_set_max_errors(self._h, int(k)))

    def set_profiling(self, on, level: int = 1):
        """Kernel timing: level 1 = generators and batched solver, 2 = all."""
        self._check(self._lib.rei_set_profiling(self._h, level if on else 0))

    def set_profiling_class(self, k):
        """Kernel timing for one class only (index or name in KERNEL_CLASSES)."""
        k = KERNEL_CLASSES.index(k) if isinstance(k, str) else int(k)
        self._check(self._lib.rei_set_profiling_class(self._h, k))

    def kernel_stats(self, k: int):
        n, u = ctypes.c_uint64(), ctypes.c_uint64()
        ms = ctypes.c_double()
        self._check(self._lib.rei_kernel_stats(self._h, int(k), ctypes.byref(n), ctypes.byref(ms),
                                               ctypes.byref(u)))
        return n.value, ms.value, u.value

    # ---- inspection ----
    def ic_word(self, i: int) -> str:
        buf = ctypes.create_string_buffer(4096)
        self._check(self._lib.rei_ic_word(self._h, int(i), buf, 4096))
        return buf.value.decode("latin-1")

    def level_size(self, cost: int) -> int:
        v = ctypes.c_uint64()
        self._check(self._lib.rei_level_size(self._h, int(cost), ctypes.byref(v)))
        return v.value

    def row_bits(self, cost: int, i: int, words: int) -> List[int]:
        buf = (ctypes.c_uint64 * words)()
        self._check(self._lib.rei_row_bits(self._h, int(cost), int(i), buf))
        return list(buf)

    def row_regex(self, cost: int, i: int) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self._lib.rei_row_regex(self._h, int(cost), int(i), buf, 1 << 16))
        return buf.value.decode("utf-8")


def solve_batch(instances: Sequence["Instance"], stream: Optional[int] = -1,
                arena_bytes: int = 0) -> List[Result]:
    """``rei_solve_batch`` over staged instances (results in the same order)."""
    if not instances:
        return []
    lib = load_library()
    if stream == -1:
        stream = current_stream_handle()
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i._h for i in instances])
    rs = (_Result * n)()
    st = lib.rei_solve_batch(hs, n, ctypes.c_void_p(stream or 0), int(arena_bytes), rs)
    if st != 0:
        msg = "; ".join(sorted({lib.rei_last_error(i._h).decode() for i in instances} - {""}))
        raise ReiError(st, msg)
    return [inst._result(rs[k]) for k, inst in enumerate(instances)]


def solve_batch_noalloc(instances: Sequence["Instance"], stream: Optional[int] = -1) -> List[Result]:
    """``rei_solve_batch_noalloc``: the batched search in the library's static
    device array, with no device allocation (at most 64 instances)."""
    if not instances:
        return []
    lib = load_library()
    if stream == -1:
        stream = current_stream_handle()
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i._h for i in instances])
    rs = (_Result * n)()
    st = lib.rei_solve_batch_noalloc(hs, n, ctypes.c_void_p(stream or 0), rs)
    if st != 0:
        msg = "; ".join(sorted({lib.rei_last_error(i._h).decode() for i in instances} - {""}))
        raise ReiError(st, msg)
    return [inst._result(rs[k]) for k, inst in enumerate(instances)]


def tune_batch(instances: Sequence["Instance"], stream: Optional[int] = -1,
               arena_bytes: int = 0) -> dict:
    """``rei_tune_batch``: pick and remember the fastest workgroup size per
    word-width group for batches like this one, then each group's hand-off
    level size (0: rei_solve's path from the start); returns
    {"threads_per_instance": {group: threads}, "level_max": {group: n}}."""
    lib = load_library()
    if stream == -1:
        stream = current_stream_handle()
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i._h for i in instances])
    out = (ctypes.c_uint32 * 7)()
    lm = (ctypes.c_uint64 * 7)()
    st = lib.rei_tune_batch(hs, n, ctypes.c_void_p(stream or 0), int(arena_bytes), out, lm)
    if st != 0:
        msg = "; ".join(sorted({lib.rei_last_error(i._h).decode() for i in instances} - {""}))
        raise ReiError(st, msg)
    names = ["W1-inline", "W1", "W2", "W4", "W8", "W16", "W32"]
    shape = {names[k]: int(out[k]) for k in range(7) if out[k]}
    levels = {names[k]: int(lm[k]) for k in range(7) if lm[k] != (1 << 64) - 1}
    return {"threads_per_instance": shape, "level_max": levels}


def tune_grid(instances: Sequence["Instance"], stream: Optional[int] = -1) -> dict:
    """``rei_tune_grid``: per word width of the instances, the per-chunk
    path's launch parameters chosen by timing rei_solve; returns
    {"W<k>": {"first_chunk", "chunk_max", "concat_wg", "concat_xi"}}."""
    lib = load_library()
    if stream == -1:
        stream = current_stream_handle()
    n = len(instances)
    hs = (ctypes.c_void_p * n)(*[i._h for i in instances])
    out = (ctypes.c_uint64 * 24)()
    st = lib.rei_tune_grid(hs, n, ctypes.c_void_p(stream or 0), out)
    if st != 0:
        msg = "; ".join(sorted({lib.rei_last_error(i._h).decode() for i in instances} - {""}))
        raise ReiError(st, msg)
    names = ("first_chunk", "chunk_max", "concat_wg", "concat_xi")
    return {f"W{1 << k}": {names[j]: int(out[4 * k + j]) for j in range(4)} for k in range(6) if out[4 * k]}


def tune_save(path: str):
    """``rei_tune_save``: the process's tuning tables to a JSON file."""
    st = load_library().rei_tune_save(path.encode())
    if st != 0:
        raise ReiError(st, f"rei_tune_save({path})")


def tune_load(path: str):
    """``rei_tune_load``: tuning tables from a JSON file."""
    st = load_library().rei_tune_load(path.encode())
    if st != 0:
        raise ReiError(st, f"rei_tune_load({path})")


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = []  # every pair ever registered: instances keep theirs until destroyed
_py_allocator_active = False


def set_allocator(alloc: Optional[Callable[[int], int]], free: Optional[Callable[[int], None]]):
    """``rei_set_allocator``: instances created from now on take their device
    memory from ``alloc(bytes) -> address`` (0 on failure) and give it back
    with ``free(address)``; ``None, None`` restores hipMalloc / hipFree."""
    global _py_allocator_active
    lib = load_library()
    if alloc is None and free is None:
        st = lib.rei_set_allocator(_ALLOC_FN(), _FREE_FN(), None)
    elif alloc is None or free is None:
        raise ValueError("set_allocator needs both functions or neither")
    else:
        def c_alloc(nbytes, _ctx):
            try:
                return int(alloc(int(nbytes))) or None
            except Exception:  # an exception cannot cross the C boundary: report failure
                return None

        def c_free(ptr, _ctx):
            try:
                free(int(ptr))
            except Exception:
                pass

        pair = (_ALLOC_FN(c_alloc), _FREE_FN(c_free))
        _allocator_refs.append(pair)
        st = lib.rei_set_allocator(pair[0], pair[1], None)
    if st != 0:
        raise ReiError(st, "rei_set_allocator")
    _py_allocator_active = alloc is not None


def use_torch_allocator(device: Optional[int] = None):
    """Route the device memory of new instances through torch's caching
    allocator on ``device`` (default: the current device)."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev),
                  torch.cuda.caching_allocator_delete)


def set_hash_bits(bits: int):
    """``rei_set_hash_bits`` (testing): keep only the low bits of the hash."""
    st = load_library().rei_set_hash_bits(int(bits))
    if st != 0:
        raise ReiError(st, "rei_set_hash_bits")


def timing_overhead_us() -> float:
    """``rei_timing_overhead``: what the timing events read for an empty kernel."""
    lib = load_library()
    v = ctypes.c_double()
    st = lib.rei_timing_overhead(ctypes.byref(v))
    if st != 0:
        raise ReiError(st, "rei_timing_overhead")
    return v.value


class BatchGraph:
    """``rei_batch_graph_*``: a fixed set of staged instances whose batched
    solve is captured once as a graph; ``launch`` enqueues a replay,
    ``results`` waits for it and returns the results in the instances' order."""

    def __init__(self, instances: Sequence["Instance"], arena_bytes: int = 0):
        lib = load_library()
        self._lib = lib
        self._insts = list(instances)
        n = len(self._insts)
        hs = (ctypes.c_void_p * max(1, n))(*[i._h for i in self._insts])
        h = ctypes.c_void_p()
        st = lib.rei_batch_graph_create(hs, n, int(arena_bytes), ctypes.byref(h))
        if st != 0:
            msg = "; ".join(sorted({lib.rei_last_error(i._h).decode() for i in self._insts} - {""}))
            raise ReiError(st, msg or "rei_batch_graph_create")
        self._h = h

    def _check(self, st):
        if st != 0:
            raise ReiError(st, self._lib.rei_batch_graph_error(self._h).decode())

    def launch(self, stream: Optional[int] = -1):
        if stream == -1:
            stream = current_stream_handle()
        self._check(self._lib.rei_batch_graph_launch(self._h, ctypes.c_void_p(stream or 0)))

    def results(self) -> List[Result]:
        n = len(self._insts)
        rs = (_Result * max(1, n))()
        self._check(self._lib.rei_batch_graph_results(self._h, rs))
        return [inst._result(rs[k]) for k, inst in enumerate(self._insts)]

    def run(self, stream: Optional[int] = -1) -> List[Result]:
        self.launch(stream)
        return self.results()

    def outside(self) -> int:
        """Instances solved beside each replay on rei_solve's path (not
        batchable, or too heavy for one workgroup)."""
        return int(self._lib.rei_batch_graph_outside(self._h))

    def close(self):
        if self._h:
            self._lib.rei_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PEAK_KINDS = {"copy": 0, "probe": 1, "probe_atomic": 2, "bitwise": 3}


def measure_peak(kind: str, size: int = 0):
    """``rei_measure_peak``: (rate, seconds) of one achievable-peak kernel:
    copy (bytes read + written / s), probe / probe_atomic (random table probes
    / s over a table of ``size`` bytes), bitwise (32-bit bitwise ops / s)."""
    lib = load_library()
    rate, sec = ctypes.c_double(), ctypes.c_double()
    st = lib.rei_measure_peak(PEAK_KINDS[kind], int(size), ctypes.byref(rate), ctypes.byref(sec))
    if st != 0:
        raise ReiError(st, f"rei_measure_peak({kind})")
    return rate.value, sec.value


class Server:
    """Continuous-batching server (``rei_server_*``): submit staged instances,
    poll or wait for their results."""

    def __init__(self, hbm_budget: int = 0, max_batch: int = 64, n_streams: int = 4, n_workers: int = 4,
                 queue: bool = True):
        """hbm_budget: device bytes the requests in flight may hold (0 = the
        free device memory at creation less 8 GB).  queue: persistent
        launches fed from a ring while they run (True) or one batched launch
        per admitted group (False)."""
        lib = load_library()
        self._lib = lib
        h = ctypes.c_void_p()
        st = lib.rei_server_create(int(hbm_budget), int(max_batch), int(n_streams), int(n_workers),
                                   ctypes.byref(h))
        if st != 0:
            raise ReiError(st, "rei_server_create")
        self._h = h
        self._inst = {}
        st = lib.rei_server_set_queue_mode(h, 1 if queue else 0)
        if st != 0:
            raise ReiError(st, "rei_server_set_queue_mode")

    def submit(self, inst: "Instance") -> int:
        t = ctypes.c_uint64()
        st = self._lib.rei_server_submit(self._h, inst._h, ctypes.byref(t))
        if st != 0:
            raise ReiError(st, "rei_server_submit")
        self._inst[t.value] = inst
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """(done, Result or None, latency seconds or None)."""
        done = ctypes.c_int()
        r = _Result()
        lat = ctypes.c_double()
        st = self._lib.rei_server_poll(self._h, int(ticket), 1 if wait else 0, ctypes.byref(done),
                                       ctypes.byref(r), ctypes.byref(lat))
        if not done.value:
            return False, None, None
        inst = self._inst.pop(ticket)
        if st != 0:
            raise ReiError(st, inst._lib.rei_last_error(inst._h).decode())
        return True, inst._result(r), lat.value

    def wait(self, ticket: int):
        _, res, lat = self.poll(ticket, wait=True)
        return res, lat

    def close(self):
        if self._h:
            self._lib.rei_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(alphabet, pos, neg, costs=(1, 1, 1, 1, 1), max_cost=30, cache_bytes=1 << 30,
          max_errors=0, chunk=0, stream=-1, on_the_fly=False, char_costs=None) -> Result:
    inst = Instance(alphabet, pos, neg, costs, max_cost, cache_bytes)
    try:
        if char_costs is not None:
            inst.set_char_costs(char_costs)
        if max_errors:
            inst.set_max_errors(max_errors)
        if on_the_fly:
            inst.set_on_the_fly(True)
        if chunk:
            inst.set_chunk(chunk)
        return inst.solve(stream)
    finally:
        inst.close()
