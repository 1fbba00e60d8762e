"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1011_0468_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", text))
    # function-pointer typedef names are not exports
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_expected_entry_points():
    syms = _header_symbols()
    for name in ("tc_build_csr", "tc_sample", "tc_count_exact", "tc_estimate", "tc_rp_trace"):
        assert name in syms
    assert set(syms) == set(_native.EXPORTS)


def test_library_exports_every_header_symbol():
    L = _native.load()
    for name in _header_symbols():
        assert hasattr(L, name), name


def _status(call):
    return call


def test_invalid_arguments_fail_before_device_work():
    L = _native.load()
    out = ctypes.c_void_p(0)
    # null output
    assert L.tc_build_csr(4, 0, None, None, 0, None, None) == _native.TC_ERR_INVALID
    assert b"NULL" in L.tc_last_error()
    # negative sizes
    assert L.tc_build_csr(-1, 0, None, None, 0, None, ctypes.byref(out)) == _native.TC_ERR_INVALID
    # n and pair-count limits of the int32 CSR
    assert L.tc_build_csr(1 << 31, 0, None, None, 0, None, ctypes.byref(out)) == _native.TC_ERR_OVERFLOW
    assert L.tc_build_csr(10, 1 << 30, ctypes.c_void_p(8), ctypes.c_void_p(8), 0, None,
                          ctypes.byref(out)) == _native.TC_ERR_OVERFLOW
    # null graph handles
    c = _native.TcCounts()
    assert L.tc_count_exact(None, None, None, ctypes.byref(c)) == _native.TC_ERR_INVALID
    assert L.tc_sample(None, 0.5, 0, None, ctypes.byref(out)) == _native.TC_ERR_INVALID
    q = (ctypes.c_int64 * 4)()
    assert L.tc_rp_trace(None, 4, 0, None, q, None) == _native.TC_ERR_INVALID
    n = ctypes.c_int64()
    assert L.tc_graph_info(None, ctypes.byref(n), None, None) == _native.TC_ERR_INVALID
    L.tc_graph_free(None)  # ignored


def test_allocator_pairing_rule():
    L = _native.load()
    f = _native.ALLOC_FN(lambda b, s, c: None)
    assert L.tc_set_allocator(f, ctypes.cast(None, _native.FREE_FN), None) == _native.TC_ERR_INVALID
    assert L.tc_set_allocator(ctypes.cast(None, _native.ALLOC_FN), ctypes.cast(None, _native.FREE_FN),
                              None) == _native.TC_OK


def test_profile_hooks_without_device():
    L = _native.load()
    ms, cnt = ctypes.c_double(1.0), ctypes.c_int64(5)
    assert L.tc_profile_reset() == 0
    assert L.tc_profile_read(b"light_small", ctypes.byref(ms), ctypes.byref(cnt)) == 0
    assert ms.value == 0.0 and cnt.value == 0
    assert L.tc_profile_read(None, None, None) == _native.TC_ERR_INVALID


def test_heavy_multiplier_terms_are_capped():
    # heavy_num and heavy_den above 2^15 are refused before any device work:
    # the handle below is never dereferenced, because argument validation
    # precedes every use of it
    L = _native.load()
    dummy = ctypes.c_void_p(16)
    c = _native.TcCounts()
    for num, den in ((1 << 15, 1 << 16), (1 << 20, 1), (1, (1 << 15) + 1), (-1, 1), (1, 0)):
        prm = _native.TcParams(num, den, 0)
        assert L.tc_count_exact(dummy, ctypes.byref(prm), None, ctypes.byref(c)) == _native.TC_ERR_INVALID
        t = _native.TcTuning(num, den, 128, 1024, 8)
        assert L.tc_tune_set(dummy, ctypes.c_double(0.5), ctypes.byref(t)) == _native.TC_ERR_INVALID
    assert b"32768" in L.tc_last_error() or b">= 1" in L.tc_last_error()
