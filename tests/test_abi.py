"""Host-side checks of the C ABI (no GPU): the library loads and exports every
symbol include/tc.h declares; argument validation that happens before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")
LIB = os.path.join(ROOT, "paper_1907_09575_amd", "libtc.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtc.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_core_entry_points():
    syms = declared_symbols()
    for name in ("tc_preprocess", "tc_count", "tc_edge_support", "tc_block_count", "tc_count_batched",
                 "tc_graph_info", "tc_graph_export", "tc_graph_free", "tc_status_string"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings(lib):
    lib.tc_status_string.restype = ctypes.c_char_p
    lib.tc_status_string.argtypes = [ctypes.c_int]
    for s in range(7):
        assert lib.tc_status_string(s)
    lib.tc_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.tc_version()


def test_argument_validation_without_device(lib):
    # rejected before any HIP call: null out pointer, n < 1, m_raw < 0
    P = ctypes.c_void_p
    lib.tc_preprocess.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P, ctypes.POINTER(P)]
    lib.tc_preprocess.restype = ctypes.c_int
    out = P()
    assert lib.tc_preprocess(None, None, 0, 10, None, None) == 1
    assert lib.tc_preprocess(None, None, 0, 0, None, ctypes.byref(out)) == 1
    assert lib.tc_preprocess(None, None, -5, 10, None, ctypes.byref(out)) == 1
    assert lib.tc_preprocess(None, None, 5, 10, None, ctypes.byref(out)) == 1
    assert out.value is None
    lib.tc_count.argtypes = [P, P, P]
    assert lib.tc_count(None, None, None) == 1
    lib.tc_edge_support.argtypes = [P, ctypes.c_int, P, P, P]
    assert lib.tc_edge_support(None, 0, None, None, None) == 1
    lib.tc_last_error.restype = ctypes.c_char_p
    assert b"null" in lib.tc_last_error()
    I32 = ctypes.c_int32
    lib.tc_block_count.argtypes = [P, I32, I32, I32, P, P, P]
    assert lib.tc_block_count(None, 2, 0, 0, None, None, None) == 1
    # the grid is checked before the handle is touched (a dummy handle is
    # never dereferenced on these paths)
    dummy = P(16)
    for q, x, y in [(0, 0, 0), (65, 0, 0), (13, 13, 0), (13, 0, -1)]:
        assert lib.tc_block_count(dummy, q, x, y, dummy, None, None) == 1
    assert b"grid" in lib.tc_last_error() or b"q must" in lib.tc_last_error()
    # batch and server entry points validate before touching the device
    lib.tc_batch_create.argtypes = [P, I32, ctypes.c_char_p, P, ctypes.POINTER(P)]
    assert lib.tc_batch_create(None, -1, None, None, ctypes.byref(out)) == 1
    assert lib.tc_batch_create(None, 2, None, None, ctypes.byref(out)) == 1
    assert lib.tc_batch_create(None, 0, b'{"order": "fifo"}', None, ctypes.byref(out)) == 1
    assert b"order" in lib.tc_last_error()
    lib.tc_server_create.argtypes = [ctypes.c_int64, I32, ctypes.c_char_p, ctypes.POINTER(P)]
    assert lib.tc_server_create(0, 4, None, ctypes.byref(out)) == 1
    assert lib.tc_server_create(1 << 30, 0, None, ctypes.byref(out)) == 1
    assert lib.tc_server_create(1 << 30, 4, b'{"prep_threads": 0}', ctypes.byref(out)) == 1
    lib.tc_server_submit.argtypes = [P, P, P]
    assert lib.tc_server_submit(None, None, None) == 1
    lib.tc_server_poll.argtypes = [P, ctypes.c_int64, I32, P]
    assert lib.tc_server_poll(None, 1, 0, None) == 1
    lib.tc_server_destroy.argtypes = [P]
    lib.tc_server_destroy(None)  # no-op
    lib.tc_graph_free.argtypes = [P]
    lib.tc_graph_free(None)  # no-op


def test_package_refuses_missing_library(tmp_path):
    # the binding must fail loudly rather than fall back to anything
    import subprocess
    import sys
    code = ("import importlib.util, sys; "
            "spec = importlib.util.spec_from_file_location('pkg', %r, "
            "submodule_search_locations=[]); "
            "m = importlib.util.module_from_spec(spec); "
            "m.__file__ = %r; spec.loader.exec_module(m)") % (
        os.path.join(ROOT, "paper_1907_09575_amd", "__init__.py"), str(tmp_path / "__init__.py"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode != 0
    assert "libtc.so is not built" in r.stderr
