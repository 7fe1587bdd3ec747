"""CPU checks of the C ABI library: it loads, exports every function that
include/lcd.h declares, and rejects malformed graphs on the host before any
device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcd.h")
LIB = os.path.join(ROOT, "paper_1301_0955_amd", "liblcd.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1301_0955_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "lcd_sweep" in names and "lcd_graph_upload" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_params(lib):
    lib.lcd_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.lcd_version()


def _upload(lib, n, rp, col, w=None):
    lib.lcd_graph_upload.restype = ctypes.c_int
    lib.lcd_graph_upload.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.uint8)
        wp = w.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    st = lib.lcd_graph_upload(n, col.size, rp.ctypes.data_as(ctypes.c_void_p),
                              col.ctypes.data_as(ctypes.c_void_p), wp, 0, None, ctypes.byref(h))
    lib.lcd_last_error.restype = ctypes.c_char_p
    return st, lib.lcd_last_error().decode()


@pytest.mark.parametrize("case", ["asymmetric", "self_loop", "unsorted", "range", "bad_ptr",
                                  "zero_weight", "weight_mismatch"])
def test_graph_validation_rejects(lib, case):
    # path 0-1-2 is the valid base
    n, rp, col, w = 3, [0, 1, 3, 4], [1, 0, 2, 1], None
    if case == "asymmetric":
        rp, col = [0, 1, 2, 2], [1, 2]
    elif case == "self_loop":
        rp, col = [0, 2, 4, 5], [0, 1, 0, 2, 1]
    elif case == "unsorted":
        rp, col = [0, 1, 3, 4], [1, 2, 0, 1]
    elif case == "range":
        rp, col = [0, 1, 3, 4], [1, 0, 3, 1]
    elif case == "bad_ptr":
        rp = [0, 2, 1, 4]
    elif case == "zero_weight":
        w = [1, 1, 0, 0]
    elif case == "weight_mismatch":
        w = [1, 2, 3, 3]
    st, msg = _upload(lib, n, rp, col, w)
    assert st == 1, (case, st, msg)     # LCD_EINVAL
    assert msg


def test_server_rejects_null_arguments(lib):
    """Argument checks of the server entry points that run before any device
    call."""
    P = ctypes.c_void_p
    lib.lcd_server_create.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.POINTER(P)]
    lib.lcd_server_submit.argtypes = [P, P, ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.lcd_server_poll.argtypes = [P, ctypes.c_uint64, P, ctypes.c_int32, P]
    lib.lcd_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.c_int32]
    lib.lcd_server_destroy.argtypes = [P]
    h = P()
    assert lib.lcd_server_create(None, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.lcd_server_create(None, 0, 0, None, None) == 1
    t = ctypes.c_uint64()
    seeds = np.array([0], np.int32)
    assert lib.lcd_server_submit(None, seeds.ctypes.data_as(P), 1, 0.5, ctypes.byref(t)) == 1
    assert lib.lcd_server_poll(None, 1, None, 0, None) == 1
    assert lib.lcd_server_wait(None, 1, 0) == 1
    assert lib.lcd_server_destroy(None) == 0


@pytest.mark.parametrize("case", ["local_range", "row_end", "offsets"])
def test_batch_upload_rejects(lib, case):
    """Batch upload validates each member graph in its local ids on the host."""
    P = ctypes.c_void_p
    lib.lcd_graph_upload_batch.restype = ctypes.c_int
    lib.lcd_graph_upload_batch.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P,
                                           ctypes.POINTER(P)]
    # two paths 0-1-2 (local ids)
    node_off = np.array([0, 3, 6], np.int64)
    edge_off = np.array([0, 4, 8], np.int64)
    rp = np.array([0, 1, 3, 4, 0, 1, 3, 4], np.int32)
    col = np.array([1, 0, 2, 1, 1, 0, 2, 1], np.int32)
    if case == "local_range":
        col[5] = 3            # a batch id, not a local one
    elif case == "row_end":
        rp[7] = 3
    elif case == "offsets":
        edge_off[1] = 5
    h = P()
    st = lib.lcd_graph_upload_batch(2, node_off.ctypes.data_as(P), edge_off.ctypes.data_as(P),
                                    rp.ctypes.data_as(P), col.ctypes.data_as(P), None, 0, None,
                                    ctypes.byref(h))
    assert st == 1, (case, st)
