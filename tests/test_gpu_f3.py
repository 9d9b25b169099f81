"""The steering car of the paper's experiment (eq (6)), the convergence-mode
solve and the optimal-control query (eq (9)) through the C ABI, against the
oracle."""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import assert_f32_close, assert_f64_close, check_f32_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


# --------------------------------------------------------- steering car ---


@pytest.mark.parametrize("kernel", ["plane", "stream", "generic"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_steering_car_solve_matches_oracle(monkeypatch, kernel, precision):
    """ENO2 + TVD-RK2 solve of the steering car (the paper's limits, with a
    disturbance) on every stage kernel: the CFL step is the oracle's bit for
    bit, V within the parity bars."""
    from paper_2012_04011_amd import hj

    if kernel != "plane":
        monkeypatch.setenv("HJ_STAGE_KERNEL", kernel)
    grid = W.car_grid(30, 28, 12, 20)
    dyn = W.steer_dynamics(d_max=0.05)
    sch = W.scheme("eno2", "rk2")
    cyl = W.cylinders(13, 4)
    V0 = oracle.target_cylinders(grid, *cyl)
    ref, oinfo = oracle.solve(grid, dyn, sch, V0, 0.5)
    with hj.Grid(grid, dyn, sch, precision) as g:
        g.set_target_cylinders(*cyl)
        assert g.cfl_dt() == oracle.cfl_dt(grid, dyn, 0.8, 0.5)
        np.testing.assert_array_equal(g.alpha_max(), oracle.alpha_max(grid, dyn))
        info = g.solve_brt(0.5)
        assert g.launch_info()["kernel"] == kernel
        V = g.value(np.float64)
    assert info["steps"] == oinfo["steps"]
    if precision == "f64":
        assert_f64_close(V, ref)
    else:
        check_f32_solve(V, ref, grid, "eno2")


def test_paper_context_run_grid():
    """The paper's experiment grid and model: 60x60x20x36, steering car,
    first-order upwind + Euler, 67 steps of the printed dt = 0.007497 s
    (Table II): FP32 against the oracle."""
    from paper_2012_04011_amd import hj

    grid = W.car_grid(60, 60, 20, 36)
    dyn = W.steer_dynamics()
    sch = W.scheme("upwind1", "euler")
    cyl = W.cylinders(70, 3)
    V0 = oracle.target_cylinders(grid, *cyl)
    ref = V0.copy()
    for _ in range(67):
        ref = oracle.step(grid, dyn, sch, V0, ref, 0.007497)
    with hj.Grid(grid, dyn, sch, "f32") as g:
        g.set_target_cylinders(*cyl)
        for _ in range(67):
            g.step(0.007497)
        V = g.value(np.float64)
    assert_f32_close(V, ref, grid)


# ----------------------------------------------------- convergence mode ---

GRID_C = W.car_grid(22, 20, 8, 12)
CYL_C = W.cylinders(14, 3)
UP_EU = W.scheme("upwind1", "euler")


def _oracle_eps(dyn, steps):
    V0 = oracle.target_cylinders(GRID_C, *CYL_C)
    dt = oracle.cfl_dt(GRID_C, dyn, 0.8, 1.0)
    U, eps = V0.copy(), []
    for _ in range(steps):
        P = U
        U = oracle.step(GRID_C, dyn, UP_EU, V0, U, dt)
        eps.append(np.abs(U - P).max())
    return np.array(eps)


@pytest.mark.parametrize("stop", [20, 35])  # inside the first and the second 32-step chunk
@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("dyn", [W.car_dynamics(), W.steer_dynamics()], ids=["car", "steer"])
def test_converge_stops_where_oracle_stops(stop, precision, dyn):
    """Threshold between the oracle's changes of steps stop-1 and stop (a
    margin of more than 5 % on each side, so the FP32 solve decides the same
    way): same step count, converged, V within the parity bars."""
    from paper_2012_04011_amd import hj

    e = _oracle_eps(dyn, stop + 2)
    thr = math.sqrt(e[stop - 1] * e[stop - 2])
    assert (e[: stop - 1] > 1.05 * thr).all() and e[stop - 1] < thr / 1.05
    V0 = oracle.target_cylinders(GRID_C, *CYL_C)
    ref, oinfo = oracle.solve_converge(GRID_C, dyn, UP_EU, V0, thr, 500)
    assert oinfo["steps"] == stop and oinfo["converged"]
    with hj.Grid(GRID_C, dyn, UP_EU, precision) as g:
        g.set_target_cylinders(*CYL_C)
        info = g.solve_converge(thr, 500)
        V = g.value(np.float64)
    assert info["steps"] == stop and info["converged"] and info["dt"] == oinfo["dt"]
    assert info["eps_last"] == pytest.approx(oinfo["eps_last"], rel=1e-3 if precision == "f32" else 1e-9)
    if precision == "f64":
        assert_f64_close(V, ref)
    else:
        assert_f32_close(V, ref, GRID_C)


def test_converge_cap_equals_plain_steps():
    """A threshold of zero is never met: exactly max_steps steps (across a
    chunk boundary), bitwise the same V as that many hj_step calls."""
    from paper_2012_04011_amd import hj

    sch = W.scheme("eno2", "rk2")
    with hj.Grid(GRID_C, W.car_dynamics(d_max=0.1), sch, "f32") as g:
        g.set_target_cylinders(*CYL_C)
        info = g.solve_converge(0.0, 45)
        V = g.value(np.float64)
        assert info["steps"] == 45 and not info["converged"]
        g.set_target_cylinders(*CYL_C)
        for _ in range(45):
            g.step()
        assert np.array_equal(g.value(np.float64), V)


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("deriv,integ", [("eno2", "rk2"), ("upwind1", "euler")])
def test_converge_fused_eps_equals_separate_pass(monkeypatch, precision, deriv, integ):
    """The plane kernel folds each step's largest change into its last stage
    (the whole plane, and a plane split into v segments); the streaming
    kernel leaves it to a separate pass over V_t and V_t+1.  Every step's
    eps, the stop and V are bitwise the same either way."""
    from paper_2012_04011_amd import hj

    sch = W.scheme(deriv, integ)
    dyn = W.car_dynamics(d_max=0.1)
    runs = {}
    monkeypatch.setenv("HJ_X_CHUNKS", "2")  # a fixed launch configuration: no autotuning in between
    for kernel, vseg in (("stream", None), ("plane", None), ("plane", "4")):
        if kernel == "stream":
            monkeypatch.setenv("HJ_STAGE_KERNEL", "stream")
        else:
            monkeypatch.delenv("HJ_STAGE_KERNEL", raising=False)
        if vseg:
            monkeypatch.setenv("HJ_PLANE_VSEG", vseg)
        else:
            monkeypatch.delenv("HJ_PLANE_VSEG", raising=False)
        with hj.Grid(GRID_C, dyn, sch, precision) as g:
            info_li = g.launch_info()
            assert info_li["kernel"] == kernel and (info_li["plane_segments"] > 1) == (vseg is not None)
            g.set_target_cylinders(*CYL_C)
            capped = g.solve_converge(0.0, 40)
            Vc = g.value(np.float64)
            thr = 0.5 * (capped["eps_last"] + g.solve_converge(0.0, 10)["eps_last"])
            stop = g.solve_converge(thr, 100)
            assert g.launch_info()["kernel"] == kernel
            runs[(kernel, vseg)] = (capped, Vc, stop, g.value(np.float64))
    ref = runs[("stream", None)]
    for key, r in runs.items():
        assert r[0] == ref[0] and r[2] == ref[2], key
        assert np.array_equal(r[1], ref[1]) and np.array_equal(r[3], ref[3]), key


def test_converge_zero_dynamics_one_step():
    from paper_2012_04011_amd import hj

    dyn = {"kind": "drift_input", "drift": (0.0, 0.0, 0.0, 0.0), "in_axes": (), "in_speed": 0.0}
    with hj.Grid(GRID_C, dyn, UP_EU, "f64") as g:
        g.set_target_cylinders(*CYL_C)
        info = g.solve_converge(1e-12, 100)
        assert info["steps"] == 1 and info["converged"] and info["eps_last"] == 0.0
        assert np.array_equal(g.value(), g.target())


# ---------------------------------------------------- optimal control ---


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("dyn", [W.car_dynamics(), W.steer_dynamics()], ids=["car", "steer"])
def test_optimal_control_matches_oracle(precision, dyn):
    """Controls, values and the device form of the query against the
    oracle's definition evaluated on the same V (the GPU's, widened to
    FP64): identical controls, values to rounding."""
    import torch

    from paper_2012_04011_amd import hj

    grid = W.car_grid(24, 22, 10, 18)
    rng = np.random.default_rng(9)
    lo, hi = np.array(grid["lo"]), np.array(grid["hi"])
    z = lo + (hi - lo) * rng.uniform(-0.05, 1.05, size=(500, 4))  # some states off the open axes
    z[:5, 3] += 2 * math.pi  # and one period away on theta
    with hj.Grid(grid, dyn, W.scheme("eno2", "rk2"), precision) as g:
        g.set_target_cylinders(*W.cylinders(3, 3))
        g.solve_brt(0.4)
        V = g.value(np.float64)
        u, val = g.optimal_control(z)
        ud, vald = g.optimal_control(torch.from_numpy(z).cuda())
        torch.cuda.synchronize()
    ur, valr, _ = oracle.optimal_control(grid, dyn, V, z)
    assert np.array_equal(u, ur)
    np.testing.assert_allclose(val, valr, rtol=0, atol=1e-12)
    assert np.array_equal(ud.cpu().numpy(), u) and np.array_equal(vald.cpu().numpy(), val)
    assert set(np.unique(u[:, 0])) <= {-1.5, 1.5}


def test_optimal_control_rejects_test_dynamics():
    from paper_2012_04011_amd import hj

    dyn = {"kind": "drift_input", "drift": (1.0, 0.0, 0.0, 0.0), "in_axes": (), "in_speed": 0.0}
    with hj.Grid(GRID_C, dyn, UP_EU, "f32") as g:
        g.set_target_cylinders(*CYL_C)
        with pytest.raises(hj.HJError) as e:
            g.optimal_control(np.zeros((3, 4)))
        assert e.value.status == hj.HJ_ERR_UNSUPPORTED
