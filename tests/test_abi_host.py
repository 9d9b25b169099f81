"""The C-ABI library on the CPU (no GPU calls): it loads, exports every
function include/hj.h declares, and rejects invalid descriptors before
touching the device."""

import ctypes
import os
import re

import pytest

from paper_2012_04011_amd import hj
from paper_2012_04011_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hj.LIB_PATH):
        pytest.fail("libhj.so not built: run __graft_entry__.build()")
    return hj.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hj_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for core in ("hj_grid_create", "hj_set_target", "hj_solve_brt", "hj_step"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hj.EXPORTED)


def test_struct_sizes_match_the_header_layout():
    # int32[4] + pad to 8 + double[4] * 2 + uint32 (+ pad) = 88
    assert ctypes.sizeof(hj.hj_grid_desc) == 88
    assert ctypes.sizeof(hj.hj_scheme_desc) == 32
    assert ctypes.sizeof(hj.hj_solve_info) == 32
    assert ctypes.sizeof(hj.hj_dynamics_desc) == 112
    assert ctypes.sizeof(hj.hj_launch_info) == 48


def _create(grid=None, dyn=None, sch=None, precision="f32"):
    return hj.hj_grid_create(grid or W.car_grid(10, 10, 5, 8), dyn or W.car_dynamics(),
                             sch or W.scheme("eno2", "rk2"), precision)


@pytest.mark.parametrize("case", [
    "few_nodes", "lo_ge_hi", "nan_range", "bad_mask", "neg_bound", "nan_drift", "bad_kind", "bad_deriv",
    "bad_integ", "bad_prec", "cfl_zero", "cfl_big", "bad_norm", "too_many_points",
])
def test_invalid_descriptors_rejected(lib, case):
    grid = W.car_grid(10, 10, 5, 8)
    grid["n"] = list(grid["n"])
    grid["lo"] = list(grid["lo"])
    dyn = dict(W.car_dynamics())
    sch = dict(W.scheme("eno2", "rk2"))
    prec = "f32"
    if case == "few_nodes":
        grid["n"][2] = 2
    elif case == "lo_ge_hi":
        grid["lo"][1] = 5.0
    elif case == "nan_range":
        grid["lo"][0] = float("nan")
    elif case == "bad_mask":
        grid["periodic_mask"] = 1 << 5
    elif case == "neg_bound":
        dyn["a_max"] = -1.0
    elif case == "nan_drift":
        dyn = {"kind": "drift_input", "drift": (0.0, float("nan"), 0.0, 0.0)}
    elif case == "bad_kind":
        dyn["kind"] = "drift_input"
        dyn["in_axes"] = (7,)
    elif case == "cfl_zero":
        sch["cfl"] = 0.0
    elif case == "cfl_big":
        sch["cfl"] = 1.5
    elif case == "bad_norm":
        dyn = {"kind": "drift_input", "in_norm": "ball", "in_speed": float("inf")}
    elif case == "too_many_points":
        grid["n"] = [2000, 2000, 1000, 10]
    if case in ("bad_deriv", "bad_integ", "bad_prec"):
        # out-of-range enum values straight through the C structs
        g, d, s = hj.grid_desc(grid), hj.dynamics_desc(dyn), hj.scheme_desc(sch, prec)
        if case == "bad_deriv":
            s.deriv = 7
        elif case == "bad_integ":
            s.integrator = -1
        else:
            s.precision = 3
        out = ctypes.c_void_p()
        st = lib.hj_grid_create(ctypes.byref(g), ctypes.byref(d), ctypes.byref(s), None, ctypes.byref(out))
        assert st == hj.HJ_ERR_INVALID_ARG
        assert out.value is None
        assert hj.hj_last_error()
        return
    with pytest.raises(hj.HJError) as e:
        hj.hj_grid_create(grid, dyn, sch, prec)
    assert e.value.status == hj.HJ_ERR_INVALID_ARG, str(e.value)


def test_null_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.hj_grid_create(None, None, None, None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    g, d, s = hj.grid_desc(W.car_grid(10, 10, 5, 8)), hj.dynamics_desc(W.car_dynamics()), \
        hj.scheme_desc(W.scheme("eno2", "rk2"), "f32")
    assert lib.hj_grid_create(ctypes.byref(g), ctypes.byref(d), ctypes.byref(s), None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_solve_brt(None, 1.0, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_step(None, 0.0, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_set_target(None, None, 0, 0) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_grid_destroy(None) == hj.HJ_OK
    assert "null" in hj.hj_last_error()


def test_batch_null_and_range_arguments(lib):
    """Batch calls validate their arguments before touching the device."""
    out = ctypes.c_void_p()
    assert lib.hj_batch_create(None, 1, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.hj_batch_create(arr, 1, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_create(arr, 0, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_create(arr, 257, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_create(arr, 1, None) == hj.HJ_ERR_INVALID_ARG
    h = (ctypes.c_double * 1)(1.0)
    assert lib.hj_batch_solve(None, h, 0, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_set_tile(None, 8) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_set_spin_limit(None, 8) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_autotune(None, h, 0, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_get_info(None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_batch_destroy(None) == hj.HJ_OK


def test_batch_info_layout():
    assert ctypes.sizeof(hj.hj_batch_info) == 48


def test_server_null_and_range_arguments(lib):
    out = ctypes.c_void_p()
    assert lib.hj_server_create(None, None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    d = hj.hj_server_desc()
    d.scheme = hj.scheme_desc(W.scheme("eno2", "rk2"), "f32")
    d.max_inflight = 0
    assert lib.hj_server_create(ctypes.byref(d), None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    d.max_inflight = 300
    assert lib.hj_server_create(ctypes.byref(d), None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    d.max_inflight = 4
    d.hbm_budget = -1
    assert lib.hj_server_create(ctypes.byref(d), None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    d.hbm_budget = 0
    d.policy = 7  # neither small-first nor sharing
    assert lib.hj_server_create(ctypes.byref(d), None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    d.policy = hj.HJ_SERVE_SHARE
    d.scheme.cfl = 0.0
    assert lib.hj_server_create(ctypes.byref(d), None, ctypes.byref(out)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_create(ctypes.byref(d), None, None) == hj.HJ_ERR_INVALID_ARG
    i64 = ctypes.c_int64()
    assert lib.hj_server_submit(None, None, None, None, None, None, 1, 1.0, ctypes.byref(i64)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_tick(None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_poll(None, None, 0, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_take(None, 1, None, 0, 0) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_get_stats(None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_server_destroy(None) == hj.HJ_OK


def test_server_struct_layouts():
    assert ctypes.sizeof(hj.hj_server_desc) == 64
    assert ctypes.sizeof(hj.hj_server_stats) == 56
