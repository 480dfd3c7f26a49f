"""The C-ABI library loads and exports every symbol that include/rtsn.h
declares; host-side argument validation (no GPU needed: calls that would
launch kernels are not made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsn.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("rt_problem_create", "rt_apply_operator", "rt_solve", "rt_batch_submit"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2602_21958_amd import rt
    lib = C.CDLL(rt.lib_path())
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared_symbols()) <= set(rt.EXPORTED)


def test_version_and_defaults():
    from paper_2602_21958_amd import rt
    assert rt.version() == 1
    o = rt.default_opts()
    assert o.restart == 30 and o.rtol == 1e-8 and o.precision == 0 and o.krylov == 0


def test_null_arguments_are_rejected():
    from paper_2602_21958_amd import rt
    lib = rt.raw_lib()
    h = C.c_void_p()
    assert lib.rt_problem_create(None, 0, C.byref(h)) == rt.RT_E_INVALID
    assert h.value is None
    assert lib.rt_apply_operator(None, 0, None, None, None) == rt.RT_E_INVALID
    assert b"null" in lib.rt_last_error()
    assert lib.rt_solve(None, None, None, None, 0, None, None) == rt.RT_E_INVALID
