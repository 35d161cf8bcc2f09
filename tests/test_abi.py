"""The C ABI library loads and exports every entry point include/fctl1.h
declares; argument checks that need no device return FCT_ERR_BAD_ARG (CPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, ensure_built

HEADER = os.path.join(ROOT, "include", "fctl1.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:int|void|const char|void)\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text)
    return sorted(set(n for n in names if n.startswith(("fct_", "fct2_", "l1_"))))


def test_header_declares_the_four_paths():
    names = declared_functions()
    for n in ("fct_sketch", "l1_sample_probs", "l1_coreset", "l1_regress"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ensure_built())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_bad_arguments_rejected_without_device():
    lib = ctypes.CDLL(ensure_built())
    lib.fct_sketch.restype = ctypes.c_int
    lib.fct_sketch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                               ctypes.c_void_p]
    assert lib.fct_sketch(None, None, 10, 2, 10, 0, None, 4, 8, 0, 0, None, None) == -1
    lib.fct_strerror.restype = ctypes.c_char_p
    assert lib.fct_strerror(-4) == b"rank deficient"
    assert lib.fct_strerror(0) == b"ok"
    lib.fct_create.restype = ctypes.c_int
    lib.fct_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert lib.fct_create(None, 0, None) == -1
    lib.fct_sync.argtypes = [ctypes.c_void_p]
    assert lib.fct_sync(None) == -1
    lib.fct_destroy.argtypes = [ctypes.c_void_p]
    lib.fct_destroy(None)


def test_binding_names_match_abi():
    ensure_built()
    from paper_1207_4684_amd import fctl1
    assert set(fctl1.EXPORTED) == set(declared_functions())
    for n in ("fct_sketch", "l1_sample_probs", "l1_coreset", "l1_regress"):
        assert callable(getattr(fctl1, n))


def test_new_entry_points_reject_bad_arguments_without_device():
    """fct_sketch_window, l1_regress_batched, l1_solve and l1_select check
    their arguments before any device work: a null context or an empty batch
    is FCT_ERR_BAD_ARG."""
    lib = ctypes.CDLL(ensure_built())
    from paper_1207_4684_amd import fctl1
    lib.fct_sketch_window.restype = ctypes.c_int
    lib.fct_sketch_window.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_void_p]
    assert lib.fct_sketch_window(None, None, 512, 2, 512, 0, None, 64, 8, 0, 0, 0, None) == -1
    lib.l1_regress_batched.restype = ctypes.c_int
    lib.l1_regress_batched.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
    inst = (fctl1.fct_instance * 1)()
    x = (ctypes.c_double * 8)()
    status = (ctypes.c_int32 * 1)()
    assert lib.l1_regress_batched(None, inst, 1, 0, 0.05, x, None, None, None, status) == -1
    assert lib.l1_regress_batched(None, inst, 0, 0, 0.05, x, None, None, None, status) == -1
    lib.l1_solve.restype = ctypes.c_int
    lib.l1_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.l1_solve(None, None, None, None, 100, 4, 100, 0, 0, x, None) == -1
    lib.l1_select.restype = ctypes.c_int
    lib.l1_select.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p]
    S = ctypes.c_int64()
    assert lib.l1_select(None, None, None, 100, 10, 0, 50, None, None, ctypes.byref(S)) == -1
