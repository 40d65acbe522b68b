"""The C ABI library loads without a GPU and exports every function that
include/gg.h declares; calls that need a GPU fail cleanly with GG_EDEVICE."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gg_index_build", "gg_search", "gg_search_batch", "gg_serve_submit",
                 "gg_serve_poll", "gg_server_create", "gg_server_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1507_02987_amd import gg

    lib = ctypes.CDLL(gg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(gg.SYMBOLS) == set(declared_functions())


def test_strerror_and_no_gpu_paths():
    from paper_1507_02987_amd import gg

    L = gg.lib()
    assert L.gg_strerror(gg.GG_EBUDGET) == b"query exceeds the hit-buffer budget"
    assert L.gg_strerror(99) == b"unknown status"
    # argument checks that need no device
    out = ctypes.c_void_p()
    assert L.gg_index_build(None, None, 0, 0, 0, ctypes.byref(out)) == gg.GG_EINVAL
    assert L.gg_index_build(None, None, 0, 17, 0, ctypes.byref(out)) == gg.GG_EINVAL
    assert L.gg_search(None, None, 0, None, None, 0, None) == gg.GG_EINVAL
    assert L.gg_server_create(None, None, 0, 1, ctypes.byref(out)) == gg.GG_EINVAL
    try:
        gg.Index(np.frombuffer(b"ACGTACGT", np.uint8), np.array([0, 8]), 4)
    except gg.GGError as e:
        assert e.status == gg.GG_EDEVICE  # no GPU here: a clean error, no CPU fallback
    else:
        pytest.skip("a GPU is present")
