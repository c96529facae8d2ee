"""Host-side checks of the tuning table (no GPU): entries set, looked up by
nearest size class, saved and loaded as JSON; malformed entries and files are
rejected. Runs in its own process-wide table, so every entry it adds is
removed again."""
import ctypes
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1907_09575_amd", "libtc.so")
P = ctypes.c_char_p


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtc.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB)
    L.tc_tuning_set.argtypes = [P, P]
    L.tc_tuning_get.argtypes = [P, P, ctypes.c_size_t]
    L.tc_tuning_load.argtypes = [P]
    L.tc_tuning_save.argtypes = [P]
    L.tc_last_error.restype = P
    return L


def get(lib, key):
    buf = ctypes.create_string_buffer(1024)
    assert lib.tc_tuning_get(key.encode(), buf, len(buf)) == 0
    return json.loads(buf.value.decode()) if buf.value else None


KEYS = ["testarch/7cu/graph_e20", "testarch/7cu/graph_e24", "testarch/7cu/batch_e28", "testarch/9cu/graph_e20"]


@pytest.fixture
def clean(lib):
    yield
    for k in KEYS:
        lib.tc_tuning_set(k.encode(), None)


def test_set_get_nearest_class(lib, clean):
    assert get(lib, "testarch/7cu/graph_e20") is None
    assert lib.tc_tuning_set(b"testarch/7cu/graph_e20", b'{"heavy_min": 8192}') == 0
    assert lib.tc_tuning_set(b"testarch/7cu/graph_e24", b'{"wave_chunk": 4096, "ms": 1.5}') == 0
    assert get(lib, "testarch/7cu/graph_e20") == {"heavy_min": 8192}
    # nearest class within two: e21, e22 -> e20 (a tie at e22 goes to the smaller class)
    assert get(lib, "testarch/7cu/graph_e21") == {"heavy_min": 8192}
    assert get(lib, "testarch/7cu/graph_e22") == {"heavy_min": 8192}
    assert get(lib, "testarch/7cu/graph_e23") == {"wave_chunk": 4096, "ms": 1.5}
    assert get(lib, "testarch/7cu/graph_e26") == {"wave_chunk": 4096, "ms": 1.5}
    assert get(lib, "testarch/7cu/graph_e27") is None  # three classes away
    assert get(lib, "testarch/7cu/graph_e17") is None
    # other kind, other CU count: no match
    assert get(lib, "testarch/7cu/batch_e20") is None
    assert get(lib, "testarch/8cu/graph_e20") is None
    # removal
    assert lib.tc_tuning_set(b"testarch/7cu/graph_e20", None) == 0
    assert get(lib, "testarch/7cu/graph_e20") is None


def test_bad_entries_rejected(lib, clean):
    for bad in [b"not json", b'{"a": }', b'{"a": 1,}', b'{"a": 1} trailing', b"[1, 2]",
                b'{"wave_chunk": 999999}', b'{"pack_slots": 12}', b'{"heavy_min": "x"}']:
        assert lib.tc_tuning_set(b"testarch/7cu/graph_e20", bad) == 1, bad
    assert get(lib, "testarch/7cu/graph_e20") is None
    assert lib.tc_tuning_set(b"", b"{}") == 1


def test_save_load_roundtrip(lib, clean, tmp_path):
    assert lib.tc_tuning_set(b"testarch/7cu/graph_e20", b'{"heavy_min": 8192, "pack_slots": 2048}') == 0
    assert lib.tc_tuning_set(b"testarch/7cu/batch_e28", b'{"blocks_per_cu": 4, "order": "input"}') == 0
    path = str(tmp_path / "tune.json")
    assert lib.tc_tuning_save(path.encode()) == 0
    saved = json.load(open(path))
    assert saved["testarch/7cu/graph_e20"] == {"heavy_min": 8192, "pack_slots": 2048}
    assert saved["testarch/7cu/batch_e28"] == {"blocks_per_cu": 4, "order": "input"}
    for k in KEYS:
        lib.tc_tuning_set(k.encode(), None)
    assert get(lib, "testarch/7cu/batch_e28") is None
    assert lib.tc_tuning_load(path.encode()) == 0
    assert get(lib, "testarch/7cu/batch_e28") == {"blocks_per_cu": 4, "order": "input"}
    # a file written by hand: merged entry by entry
    other = tmp_path / "other.json"
    other.write_text(json.dumps({"testarch/9cu/graph_e20": {"wave_chunk": 8192}}))
    assert lib.tc_tuning_load(str(other).encode()) == 0
    assert get(lib, "testarch/9cu/graph_e20") == {"wave_chunk": 8192}
    assert get(lib, "testarch/7cu/graph_e20") == {"heavy_min": 8192, "pack_slots": 2048}


def test_bad_files_rejected(lib, clean, tmp_path):
    assert lib.tc_tuning_load(str(tmp_path / "missing.json").encode()) == 1
    for text in ["", "[]", '{"k": 1}', '{"k": {"a": 1}', '{"testarch/7cu/graph_e20": {"a": }}',
                 '{"testarch/7cu/graph_e20": {"min_groups": -5}}']:
        f = tmp_path / "bad.json"
        f.write_text(text)
        assert lib.tc_tuning_load(str(f).encode()) == 1, text
    assert get(lib, "testarch/7cu/graph_e20") is None  # nothing merged
