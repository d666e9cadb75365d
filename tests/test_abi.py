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
    assert lib.mb_eval_direct_deterministic(None, -1, None, 0, None) == 1
    assert lib.mb_eval_direct_deterministic(None, 5, None, 0, None) == 1
    assert lib.mb_eval_direct_deterministic(None, 0, None, 0, None) == 0
    assert lib.mb_version() >= 100


def test_normal_quantile_matches_python():
    # z_{alpha/2} of the Monte Carlo stop rule (host code, no device needed)
    from statistics import NormalDist

    import paper_1105_2769_amd as mb

    for a in (0.5, 0.2, 0.1, 0.05, 0.01, 0.001):
        assert mb.normal_quantile(a / 2) == pytest.approx(NormalDist().inv_cdf(1 - a / 2), rel=1e-12)
    assert mb.normal_quantile(0.0) == 0.0


def test_multitree_bad_params_no_device():
    import ctypes

    lib = _lib.lib()
    p = _lib.MtParams()
    lib.mb_mt_params_default(ctypes.byref(p))
    assert p.m_limit == 128 and p.m_min == 30 and p.zeta == 128.0 and p.bound == 0
    for field, bad in (("eps_rel", -1.0), ("alpha", 1.0), ("alpha", -0.1), ("m_limit", 1),
                       ("base_prec", 9), ("chunk", 0), ("bound", 7)):
        q = _lib.MtParams()
        lib.mb_mt_params_default(ctypes.byref(q))
        setattr(q, field, bad)
        assert lib.mb_eval_multitree(None, 10, 8, ctypes.byref(q), None, None, None, None,
                                     None) == 1, field
    out = ctypes.c_void_p()
    assert lib.mb_build_kdtree(None, 10, 0, None, ctypes.byref(out)) == 1
    assert lib.mb_build_kdtree(None, 10, 64, None, ctypes.byref(out)) in (1, 5)


def test_server_bad_arguments_no_device():
    import ctypes

    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.mb_server_create(0, 4, None, ctypes.byref(h)) == 1
    assert lib.mb_server_create(1 << 20, 0, None, ctypes.byref(h)) == 1
    assert lib.mb_server_create(1 << 20, 4, None, None) == 1
    assert not h.value
    rid = ctypes.c_int64()
    assert lib.mb_server_submit(None, None, 3, 1, ctypes.byref(rid)) == 1
    done = ctypes.c_int32()
    assert lib.mb_server_poll(None, 0, None, ctypes.byref(done)) == 1
    assert lib.mb_server_wait(None, 0, 0, None) == 1
    assert lib.mb_server_set_slice_units(None, 4) == 1
    assert lib.mb_server_cancel(None, 0) == 1
    assert lib.mb_server_set_timeout(None, 10) == 1
    assert lib.mb_server_destroy(None) == 0


def test_struct_layouts_match_the_library():
    import ctypes

    lib = _lib.lib()
    for name, cls in (("mb_mt_params", _lib.MtParams), ("mb_mt_stats", _lib.MtStats),
                      ("mb_factor_stats", _lib.FactorStats), ("mb_server_stats", _lib.ServerStats)):
        assert lib.mb_struct_size(name.encode()) == ctypes.sizeof(cls), name
    assert lib.mb_struct_size(b"nope") == -1
