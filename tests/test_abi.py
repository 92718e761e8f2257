"""The C-ABI library loads and exports every function include/mobius.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mobius.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mobius_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mobius_dslash", "mobius_dslash_dag", "mobius_m5inv", "mobius_cg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1206_5214_amd import mobius
    if not os.path.exists(mobius.LIB_PATH):
        pytest.fail("libmobius.so is not built (python -m paper_1206_5214_amd.build)")
    lib = ctypes.CDLL(mobius.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(mobius.EXPORTS)


def test_binding_rejects_missing_library(tmp_path, monkeypatch):
    from paper_1206_5214_amd import mobius
    monkeypatch.setattr(mobius, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(mobius, "_lib", None)
    with pytest.raises(mobius.MobiusError):
        mobius.lib()


def test_error_paths_without_gpu():
    """Argument validation happens before any device work."""
    from paper_1206_5214_amd import mobius
    L = mobius.lib()
    h = ctypes.c_void_p()
    # odd extent
    p = mobius._Params((ctypes.c_int32 * 4)(4, 3, 4, 4), 8, 1.8, 0.01, 1.0, 0.0)
    assert L.mobius_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(1), None) == -22
    assert b"even" in L.mobius_last_error()
    # Ls out of range
    p = mobius._Params((ctypes.c_int32 * 4)(4, 4, 4, 4), 65, 1.8, 0.01, 1.0, 0.0)
    assert L.mobius_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(1), None) == -22
    # non-finite chemical potential
    p = mobius._Params((ctypes.c_int32 * 4)(4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0, float("nan"))
    assert L.mobius_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(1), None) == -22
    assert b"chemical" in L.mobius_last_error()
    # null links
    p = mobius._Params((ctypes.c_int32 * 4)(4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0)
    assert L.mobius_create(ctypes.byref(h), ctypes.byref(p), None, None) == -22
    # null context
    assert L.mobius_dslash(None, 0, 0, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, None) == -22
    assert L.mobius_field_bytes(None, 0) == -1


def test_brick_validation_without_gpu():
    """A site-order brick with a side outside 1..L is rejected before any device
    work, by mobius_create and by the layout tuner's own checks."""
    from paper_1206_5214_amd import mobius
    L = mobius.lib()
    h = ctypes.c_void_p()
    for brick in ((0, 2, 2), (2, 2, 5), (-2, 2, 2)):
        p, _ = mobius._make_params((4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0, brick=brick)
        assert L.mobius_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(1), None) == -22
        assert b"brick" in L.mobius_last_error()
    p, _ = mobius._make_params((4, 3, 4, 4), 8, 1.8, 0.01, 1.0, 0.0)
    b = (ctypes.c_int32 * 3)()
    assert L.mobius_tune_brick(ctypes.byref(p), ctypes.c_void_p(1), 2, 1, None, 0, None, b, None, None) == -22
    p, _ = mobius._make_params((4, 4, 4, 4), 8, 1.8, 0.01, 1.0, 0.0)
    assert L.mobius_tune_brick(ctypes.byref(p), ctypes.c_void_p(1), 7, 1, None, 0, None, b, None, None) == -22
    assert L.mobius_tune_brick(ctypes.byref(p), None, 2, 1, None, 0, None, b, None, None) == -22
