"""CPU checks of the C ABI: the library loads and exports every entry point
that include/qdta.h declares; host-only calls behave.  No compute calls."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qdta.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qdta_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_2104_12911_amd import qdta
    if not os.path.exists(qdta.LIB_PATH):
        from paper_2104_12911_amd import build
        build.build()
    return qdta


def test_header_declares_entry_points():
    names = _declared()
    assert "qdta_solve" in names and "qdta_aon" in names and len(names) >= 20


def test_library_exports_every_declared_symbol():
    q = _lib()
    L = ctypes.CDLL(q.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert missing == []
    assert sorted(q.EXPORTS) == _declared()


def test_default_opts_are_the_papers():
    q = _lib()
    o = q.default_opts()
    assert (o.alpha, o.beta, o.K, o.passes) == (0.15, 4, 32, 3)
    assert (o.T1, o.T2, o.dx, o.tol) == (1e-4, 1e-4, 1e-4, 1e-4)
    assert o.trunc_rule == q.RULE_CEIL and o.ls_mode == q.LS_KSECTION
    assert ctypes.sizeof(q.Opts) == 136 and ctypes.sizeof(q.Stats) == 48


def test_strerror_covers_codes():
    q = _lib()
    L = q.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1):
        s = L.qdta_strerror(code).decode()
        assert s and s != "unknown code"
    assert L.qdta_strerror(-99).decode() == "unknown code"


def test_create_rejects_bad_device():
    q = _lib()
    h = ctypes.c_void_p()
    assert q.lib().qdta_create(ctypes.byref(h), -1, None) == q.EARG
    assert q.lib().qdta_create(None, 0, None) == q.EARG
