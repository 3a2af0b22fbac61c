"""C-ABI checks that need no GPU: the library loads, exports every function
include/mlsdisp.h declares, and rejects bad parameters before touching the
device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1308_4005_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlsdisp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mls_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmlsdisp.so is not built: run `python -m paper_1308_4005_amd.build`")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mls_plan_create", "mls_evaluate", "mls_plan_destroy", "mls_batch_create",
                     "mls_batch_evaluate", "mls_status_string", "mls_last_error"):
        assert required in names
    assert set(names) == set(_lib.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(mls_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_status_strings(lib):
    assert lib.mls_status_string(0).decode() == "success"
    for code in (-1, -2, -3, -4, -5):
        assert lib.mls_status_string(code).decode() not in ("", "unknown status")
    assert lib.mls_status_string(42).decode() == "unknown status"


def _params(**kw):
    p = _lib.MLSParams()
    box = kw.get("box", (10.0, 10.0, 10.0))
    for d in range(3):
        p.box[d] = box[d]
        p.grid[d] = kw.get("grid", (0, 0, 0))[d]
    p.cutoff = kw.get("cutoff", 3.0)
    p.h = kw.get("h", 1.0)
    p.order = kw.get("order", 4)
    p.levels = kw.get("levels", 2)
    p.precision = kw.get("precision", 0)
    p.continuity = kw.get("continuity", 0)
    p.mixing = kw.get("mixing", 0)
    return p


@pytest.mark.parametrize("bad", [
    dict(box=(10.0, -1.0, 10.0)), dict(box=(10.0, float("nan"), 10.0)), dict(cutoff=0.0),
    dict(cutoff=float("inf")), dict(h=-1.0), dict(order=5), dict(order=3), dict(levels=-1),
    dict(levels=17), dict(precision=7), dict(grid=(10, 10, 9), levels=2),
    dict(grid=(8, 8, 8), levels=0), dict(continuity=5), dict(continuity=-1), dict(mixing=2),
])
def test_plan_create_rejects_bad_parameters(lib, bad):
    p = _params(**bad)
    out = ctypes.c_void_p()
    st = lib.mls_plan_create(ctypes.byref(p), 100, ctypes.byref(out))
    assert st == _lib.MLS_ERR_INVALID_ARG
    assert out.value is None
    assert lib.mls_last_error().decode() != ""


def test_null_arguments_are_rejected(lib):
    out = ctypes.c_void_p()
    assert lib.mls_plan_create(None, 10, ctypes.byref(out)) == _lib.MLS_ERR_INVALID_ARG
    p = _params()
    assert lib.mls_plan_create(ctypes.byref(p), -5, ctypes.byref(out)) == _lib.MLS_ERR_INVALID_ARG
    assert lib.mls_evaluate(None, 0, None, None, None, None, None, None, None) == _lib.MLS_ERR_INVALID_ARG
    assert lib.mls_plan_destroy(None) == _lib.MLS_OK
    info = _lib.MLSPlanInfo()
    assert lib.mls_plan_get_info(None, ctypes.byref(info)) == _lib.MLS_ERR_INVALID_ARG


def test_md_entry_points_reject_bad_arguments(lib):
    # rejected on the host before any device work: null plan
    assert lib.mls_evaluate_md(None, 0, None, None, None, ctypes.c_double(1.0), None, None,
                               None) == _lib.MLS_ERR_INVALID_ARG
    assert lib.mls_md_run(None, 0, None, None, None, None, ctypes.c_double(1.0), None, ctypes.c_double(0.001), 1,
                          None, None, None, None) == _lib.MLS_ERR_INVALID_ARG
    assert "null plan" in lib.mls_last_error().decode()
