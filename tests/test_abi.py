"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1105_2769_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mb_[a-z0-9_]+)\s*\(", txt))
    return names


def test_every_declared_symbol_exported():
    lib = _lib.lib()
    names = declared_symbols()
    assert "mb_eval_direct" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    assert declared_symbols() == set(_lib.SIGNATURES)


def test_invalid_arguments_no_device():
    lib = _lib.lib()
    assert lib.mb_eval_direct(None, -1, 0, None, None) == 1
    assert lib.mb_eval_direct(None, 5, 0, None, None) == 1
    assert lib.mb_eval_direct(None, 5, 7, None, None) == 1
    assert b"precision" in lib.mb_last_error() or b"null" in lib.mb_last_error()
    assert lib.mb_eval_direct(None, 0, 0, None, None) == 0
    assert lib.mb_version() >= 100
