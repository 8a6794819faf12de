"""The C-ABI library loads and exports every entry point include/mcc.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2408_11331_amd as mcc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(mcc_\w+)\s*\(", txt, re.M))
    return names


def test_header_matches_binding():
    assert declared() == set(mcc.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    L = ctypes.CDLL(mcc.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name


def test_strerror_is_static_text():
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    L = mcc.lib()
    for code in (0, -1, -2, -3, -5, 7):
        assert isinstance(L.mcc_strerror(code), bytes)
