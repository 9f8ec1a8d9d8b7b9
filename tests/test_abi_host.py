"""The C-ABI library without a GPU: it loads, exports what include/rei.h
declares, and rejects bad specifications on the host before any device work."""
import ctypes
import os
import re

import pytest

import paper_2305_18575_amd as rei

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rei.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rei_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rei.load_library()
    names = declared_functions()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(rei.EXPORTS) == names


def test_status_strings():
    lib = rei.load_library()
    for code, name in rei.STATUS.items():
        expect = "REI_" + name if code >= 0 else "REI_ERR_" + name
        assert lib.rei_status_str(code).decode() == expect


@pytest.mark.parametrize("alphabet,pos,neg,costs,status", [
    ("01", ["2"], [], (1, 1, 1, 1, 1), "BAD_CHAR"),
    ("01", ["01"], ["01"], (1, 1, 1, 1, 1), "INCONSISTENT"),
    ("01", ["0"], ["1"], (1, 0, 1, 1, 1), "INVALID_ARG"),
    ("", ["0"], ["1"], (1, 1, 1, 1, 1), "INVALID_ARG"),
    ("0*", ["0"], [], (1, 1, 1, 1, 1), "INVALID_ARG"),
    ("00", ["0"], [], (1, 1, 1, 1, 1), "INVALID_ARG"),
])
def test_create_rejects_bad_specifications(alphabet, pos, neg, costs, status):
    with pytest.raises(rei.ReiError) as ei:
        rei.Instance(alphabet, pos, neg, costs=costs)
    assert ei.value.status_name == status


def test_create_rejects_too_large_infix_closure():
    # 3 strings of length 40 over 3 letters: far more than 2048 distinct infixes
    import random
    rng = random.Random(0)
    strings = ["".join(rng.choice("012") for _ in range(40)) for _ in range(3)]
    with pytest.raises(rei.ReiError) as ei:
        rei.Instance("012", strings, [])
    assert ei.value.status_name == "TOO_LARGE"


def test_row_cap_formula_matches_header():
    # the header documents floor(cache_bytes / (8W + 8)) with W the smallest
    # power of two with 64W >= |ic|
    from paper_2305_18575_amd import instances
    assert instances.row_cap(1 << 20, 63) == (1 << 20) // 16
    assert instances.row_cap(1 << 20, 65) == (1 << 20) // 24
    assert instances.row_cap(1 << 20, 200) == (1 << 20) // 40
    assert instances.row_cap(1 << 20, 2048) == (1 << 20) // 264


def test_set_allocator_argument_checks():
    """rei_set_allocator takes both functions or neither; it touches no device."""
    lib = rei.load_library()
    alloc = rei._ALLOC_FN(lambda n, ctx: None)
    free = rei._FREE_FN(lambda p, ctx: None)
    assert lib.rei_set_allocator(alloc, rei._FREE_FN(), None) == -1
    assert lib.rei_set_allocator(rei._ALLOC_FN(), free, None) == -1
    assert lib.rei_set_allocator(alloc, free, None) == 0
    assert lib.rei_set_allocator(rei._ALLOC_FN(), rei._FREE_FN(), None) == 0
    with pytest.raises(ValueError):
        rei.set_allocator(None, lambda p: None)


def test_measure_peak_argument_checks():
    """rei_measure_peak rejects an unknown kind and too small a buffer before
    any device work."""
    lib = rei.load_library()
    rate, sec = ctypes.c_double(), ctypes.c_double()
    assert lib.rei_measure_peak(7, 1 << 20, ctypes.byref(rate), ctypes.byref(sec)) == -1
    assert lib.rei_measure_peak(-1, 1 << 20, ctypes.byref(rate), ctypes.byref(sec)) == -1
    assert lib.rei_measure_peak(0, 100, ctypes.byref(rate), ctypes.byref(sec)) == -1
    assert lib.rei_measure_peak(0, 1 << 20, None, ctypes.byref(sec)) == -1


def test_batch_graph_argument_checks():
    """The graph calls reject null handles and outputs before any device work."""
    lib = rei.load_library()
    out = ctypes.c_void_p()
    assert lib.rei_batch_graph_create(None, 0, 0, None) == -1
    assert lib.rei_batch_graph_create(None, 3, 0, ctypes.byref(out)) == -1
    assert lib.rei_batch_graph_launch(None, None) == -1
    assert lib.rei_batch_graph_results(None, None) == -1
    assert lib.rei_batch_graph_error(None) == b""
    lib.rei_batch_graph_destroy(None)


def test_tuning_file_round_trip(tmp_path):
    """rei_tune_load reads what rei_tune_save writes (host tables only, no
    device work); a file with an entry out of range is rejected whole."""
    good = tmp_path / "tune.json"
    good.write_text('{"batch_threads": [{"group": 16, "size_class": 2, "threads": 512}],\n'
                    ' "batch_level_max": [{"group": 16, "level_max": 32768}, {"group": 2, "level_max": 0}],\n'
                    ' "grid": [{"words": 16, "first_chunk": 16384, "chunk_max": 4194304, '
                    '"concat_wg": 4096, "concat_xi": 8}]}\n')
    rei.tune_load(str(good))
    out = tmp_path / "saved.json"
    rei.tune_save(str(out))
    import json
    saved = json.loads(out.read_text())
    assert {"group": 16, "size_class": 2, "threads": 512} in saved["batch_threads"]
    assert {"group": 16, "level_max": 32768} in saved["batch_level_max"]
    assert {"group": 2, "level_max": 0} in saved["batch_level_max"]
    assert {"words": 16, "first_chunk": 16384, "chunk_max": 4194304, "concat_wg": 4096,
            "concat_xi": 8} in saved["grid"]
    bad = tmp_path / "bad.json"
    bad.write_text('{"grid": [{"words": 3, "first_chunk": 1, "chunk_max": 1, "concat_wg": 1, "concat_xi": 1}]}')
    with pytest.raises(rei.ReiError):
        rei.tune_load(str(bad))
    bad.write_text('{"batch_threads": [{"group": 32, "size_class": 1, "threads": 1024}]}')
    with pytest.raises(rei.ReiError):
        rei.tune_load(str(bad))
    bad.write_text('{"batch_level_max": [{"group": 3, "level_max": 4096}]}')
    with pytest.raises(rei.ReiError):
        rei.tune_load(str(bad))
    with pytest.raises(rei.ReiError):
        rei.tune_load(str(tmp_path / "missing.json"))
