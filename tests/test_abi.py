"""CPU checks of the C ABI: the library loads, exports every symbol that
include/lbrr.h declares with the binding's signatures, and rejects invalid
arguments before touching a GPU.  No compute calls are made here."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbrr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(lb_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for n in ("lb_create", "lb_init_fields", "lb_step", "lb_moments", "lb_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported_and_bound(lbrr):
    import ctypes

    lib = ctypes.CDLL(lbrr._lib.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in lbrr._lib.SIGNATURES, n
        assert getattr(lbrr, n) is not None
    assert set(lbrr._lib.SIGNATURES) == set(declared_functions())


@pytest.mark.parametrize("args,msg", [
    ((7, 8, 8, 1, 0.7, 4), "unknown lattice"),
    ((0, 8, 8, 2, 0.7, 4), "nz == 1"),
    ((0, 0, 8, 1, 0.7, 4), "dims"),
    ((2, 8, 8, 70000, 0.7, 4), "dims"),
    ((2, 2048, 2048, 1024, 0.7, 4), "2^31"),
    ((0, 8, 8, 1, 0.5, 4), "tau"),
    ((0, 8, 8, 1, float("nan"), 4), "tau"),
    ((0, 8, 8, 1, 0.7, 5), "order"),
    ((1, 8, 8, 8, 0.7, 5), "order"),
    ((2, 8, 8, 8, 0.7, 7), "order"),
    ((2, 8, 8, 8, 0.7, 1), "order"),
])
def test_invalid_create_arguments_are_rejected(lbrr, args, msg):
    h = lbrr.lb_create(*args)
    assert not h
    assert msg in lbrr.lb_last_error().decode()


def test_null_handle_calls_fail_cleanly(lbrr):
    assert lbrr.lb_step(None, 1) == lbrr.LB_ERR_INVALID_ARG
    assert lbrr.lb_config(None, 1, 1.0) == lbrr.LB_ERR_INVALID_ARG
    assert lbrr.lb_step_count(None) == -1
    assert lbrr.lb_bytes_per_update(None) == 0.0
    lbrr.lb_destroy(None)  # NULL-safe
    assert lbrr.lb_probe_copy(None, None, 16, None) == lbrr.LB_ERR_INVALID_ARG


def test_header_enums_match_the_binding(lbrr):
    """Every LB_* enumerator of the header has the value the Python binding uses."""
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "lbrr.h")).read(), flags=re.S)
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(LB_[A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    assert {"LB_STORE_MOM_FP64", "LB_STORE_MOM_FP32", "LB_ERR_UNSUPPORTED"} <= set(vals)
    for k, v in vals.items():
        assert getattr(lbrr, k) == v, k


@pytest.mark.parametrize("args,code,msg", [
    ((7, 1, 8, 8, 1, 1.0), "INVALID_ARG", "unknown lattice"),
    ((2, 4, 8, 8, 8, 1.0), "UNSUPPORTED", "population storage"),
    ((0, 1, 8, 8, 2, 1.0), "INVALID_ARG", "dims"),
    ((2, 1, 2048, 2048, 1024, 1.0), "INVALID_ARG", "2^31"),
    ((2, 1, 8, 8, 8, 0.0), "INVALID_ARG", "rho0"),
])
def test_reduce_static_rejects_bad_arguments_before_any_device_call(lbrr, args, code, msg):
    import ctypes

    r = lbrr.lb_reduce_static(*args, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert r == getattr(lbrr, "LB_ERR_" + code)
    assert msg in lbrr.lb_last_error().decode()
