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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhh.so not built")
def test_tune_choices_round_trip_through_json(tmp_path):
    # the autotuner's JSON file: loading and saving again keeps every entry
    import json
    from paper_2408_11929_amd import _lib
    lib = _lib.load()
    src = tmp_path / "tune_in.json"
    entries = [{"precision": 1, "KP": 10, "P": 8, "kmax": 24, "n": 321, "N": 16, "chains": 128,
                "plan": 2, "ms": [5.4, 0.0, 3.5, 5.9]},
               {"precision": 1, "KP": 12, "P": 8, "kmax": 29, "n": 801, "N": 32, "chains": 16,
                "plan": 1, "ms": [37.0, 5.1, 21.6, 30.2]}]
    src.write_text(json.dumps({"entries": entries}))
    assert lib.hh_tune_clear() == 0
    assert lib.hh_tune_load(str(src).encode()) == 0
    out = tmp_path / "tune_out.json"
    assert lib.hh_tune_save(str(out).encode()) == 0
    got = json.loads(out.read_text())["entries"]
    key = lambda e: (e["n"], e["chains"])
    assert sorted(got, key=key) == sorted(entries, key=key)
    assert lib.hh_tune_load(str(tmp_path / "missing.json").encode()) == -1
    assert lib.hh_tune_clear() == 0
