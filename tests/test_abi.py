"""The C ABI: libbbs loads and exports every function include/bbs.h declares.
No device work is started here (the tests run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2310_10023_amd as bbs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bbs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbs_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(bbs.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(bbs.library_path())
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version_defaults_and_error_text():
    L = bbs.lib()
    assert L.bbs_abi_version() == 1
    opt = bbs.Options()
    L.bbs_default_options(C.byref(opt))
    assert opt.batch_size == 10000 and opt.translation_only == 0 and opt.profile == 0 and not opt.stream
    assert isinstance(L.bbs_last_error(), bytes)


def test_argument_validation_before_any_device_call():
    L = bbs.lib()
    h = C.c_void_p()
    pts = np.zeros((4, 3), np.float32)
    assert L.bbs_build_map(pts.ctypes.data, 0, 0, 1.0, 3, 1, None, C.byref(h)) == -1
    assert b"n must be" in L.bbs_last_error()
    assert L.bbs_build_map(pts.ctypes.data, 4, 0, -1.0, 3, 1, None, C.byref(h)) == -1
    assert L.bbs_build_map(pts.ctypes.data, 4, 0, 1.0, 16, 1, None, C.byref(h)) == -1
    assert L.bbs_build_map(None, 4, 0, 1.0, 3, 1, None, C.byref(h)) == -1
    res = bbs.Result()
    assert L.bbs_localize(None, None, pts.ctypes.data, 4, 0, None, 0, None, C.byref(res)) == -1
    assert L.bbs_map_info(None, None, None, None, None, None) == -1
    L.bbs_free_map(None)
    L.bbs_workspace_free(None)


def test_struct_layouts():
    # field offsets the binding relies on
    assert C.sizeof(bbs.SearchRange) == 48
    assert bbs.Options.stream.offset == 16 and bbs.Options.prior.offset == 24 and bbs.Options.graph.offset == 40
    assert C.sizeof(bbs.Options) == 64
    assert bbs.Query.arrival_s.offset == 72 and bbs.Query.prior.offset == 80 and C.sizeof(bbs.Query) == 88
    assert bbs.Result.nodes_expanded.offset == 56
    assert C.sizeof(bbs.Result) == 56 + 6 * 8 + 8 + 8 + 8 + 8 + 4 * 8 + 24 + 32 + 16 * 8 + 8 + 8 + 4 + 4
