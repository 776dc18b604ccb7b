"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/fl.h, and rejects invalid arguments before any GPU work."""
import ctypes
import os
import re

import pytest

from paper_1804_02718_amd import fl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fl_coeffs", "fl_apply", "fl_poisson_solve", "fl_allen_cahn_step", "fl_op_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = fl.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_declared()) == sorted(fl.EXPORTED)


@pytest.mark.parametrize("args,status", [
    ((0, 1.0, 0.1, 8), fl.FL_E_INVAL),
    ((4, 1.0, 0.1, 8), fl.FL_E_INVAL),
    ((1, 1.0, 0.1, 1), fl.FL_E_INVAL),
    ((1, 1.0, 0.1, 1026), fl.FL_E_UNSUPPORTED),
    ((2, 0.0, 0.1, 8), fl.FL_E_INVAL),
    ((2, 2.0, 0.1, 8), fl.FL_E_INVAL),
    ((2, float("nan"), 0.1, 8), fl.FL_E_INVAL),
    ((2, 1.0, 0.0, 8), fl.FL_E_INVAL),
    ((2, 1.0, -1.0, 8), fl.FL_E_INVAL),
    ((2, 1.0, float("inf"), 8), fl.FL_E_INVAL),
    ((2, 1.0, 0.1, 1), fl.FL_E_INVAL),
    ((2, 1.0, 0.1, 8194), fl.FL_E_UNSUPPORTED),
    ((3, 1.0, 0.1, 1000), fl.FL_E_UNSUPPORTED),
])
def test_coeffs_rejects_invalid_arguments(args, status):
    lib = fl.load()
    op = ctypes.c_void_p()
    assert lib.fl_coeffs(*args, ctypes.byref(op)) == status
    assert op.value is None
    assert lib.fl_last_error()


def test_null_handles_rejected():
    lib = fl.load()
    assert lib.fl_apply(None, None, None, 0, None) == fl.FL_E_INVAL
    assert lib.fl_poisson_solve(None, None, 1e-8, None, None, None) == fl.FL_E_INVAL
    assert lib.fl_allen_cahn_step(None, None, 1e-3, 0.05, None, None) == fl.FL_E_INVAL
    assert lib.fl_op_destroy(None) == fl.FL_OK
    assert lib.fl_status_string(fl.FL_E_BREAKDOWN) == b"FL_E_BREAKDOWN"


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(fl, "_LIB", None)
    with pytest.raises(fl.FlLibraryMissing):
        fl.load(str(tmp_path / "missing.so"))
