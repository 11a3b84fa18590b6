"""The C ABI library loads and exports every symbol include/hh.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hh.h")
LIB = os.path.join(ROOT, "paper_2408_11929_amd", "libhh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hh_assemble", "hh_factor_sweeps", "hh_mpgmres", "hh_submit", "hh_poll"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhh.so not built")
def test_binding_prototypes_cover_the_header():
    from paper_2408_11929_amd import _lib
    assert set(_lib.PROTOTYPES) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhh.so not built")
def test_argument_errors_without_device_work():
    # argument validation happens before any device call
    from paper_2408_11929_amd import _lib
    lib = _lib.load()
    out = ctypes.c_void_p()
    c = (ctypes.c_double * 1)(1.0)
    assert lib.hh_assemble(-1.0, 1, c, 33, ctypes.byref(out)) == _lib.HH_EINVAL
    assert b"omega" in lib.hh_last_error()
    assert lib.hh_assemble(1.0, 1, c, 2, ctypes.byref(out)) == _lib.HH_EINVAL
    bad = (ctypes.c_double * 1)(0.0)
    assert lib.hh_assemble(1.0, 1, bad, 33, ctypes.byref(out)) == _lib.HH_EINVAL
    assert lib.hh_factor_sweeps(None, 3, 4, 0) == _lib.HH_EINVAL
    assert lib.hh_free(None) == _lib.HH_OK
