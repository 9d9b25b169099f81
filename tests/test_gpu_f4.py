"""Algorithm 1's general Lax-Friedrichs scheme (alpha from each step's
derivative range, dt recomputed every step) through the C ABI, against the
oracle and closed forms."""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import assert_f32_close, assert_f64_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


def drift_dyn(drift, axes, speed, norm, role):
    return {"kind": "drift_input", "drift": tuple(float(x) for x in drift), "in_axes": tuple(axes),
            "in_speed": float(speed), "in_norm": norm, "in_role": role}


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_range_alpha_half_plane_closed_form(precision):
    """z' = 0.5 + u on x, |u| <= 1 minimising, V0 = x: alpha_x = 0.5 (not the
    state bound 1.5), so dt = 0.8 dx / 0.5 and 3 steps cover 2.1 s; V = x -
    0.5 T exactly (to rounding)."""
    from paper_2012_04011_amd import hj

    g = W.car_grid(21, 6, 5, 8)
    dyn = drift_dyn((0.5, 0, 0, 0), (0,), 1.0, "box", "min")
    x = oracle.nodes(g, 0)
    V0 = np.broadcast_to(x[:, None, None, None], g["n"]).copy()
    sch = W.scheme("upwind1", "euler", alpha="deriv_range")
    with hj.Grid(g, dyn, sch, precision) as h:
        h.set_target(V0)
        info = h.solve_brt(2.1)
        V = h.value(np.float64)
        assert h.cfl_dt() == pytest.approx(0.8 * 0.5 / 1.5, rel=1e-15)  # the state-bound step is unchanged
    assert info["steps"] == 3 and info["dt"] == pytest.approx(0.8, rel=1e-14)
    tol = 1e-12 if precision == "f64" else 5e-6
    np.testing.assert_allclose(V, V0 - 0.5 * 2.1, atol=tol)


CASES = [
    ("car-halfplane", W.car_dynamics(d_max=0.1), "plane"),
    ("steer-halfplane", W.steer_dynamics(d_max=0.1), "plane"),
    ("ball-disk", drift_dyn((0.3, -0.2, 0, 0), (0, 1), 1.0, "ball", "min"), "disk"),
    ("box-disk", drift_dyn((0.3, -0.2, 0, 0), (0, 1), 1.0, "box", "max"), "disk"),
]


@pytest.mark.parametrize("kernel", ["plane", "stream", "generic"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name,dyn,target", CASES, ids=[c[0] for c in CASES])
def test_range_alpha_solve_matches_oracle(monkeypatch, kernel, precision, name, dyn, target):
    """Whole solves in the derivative-range mode on every stage kernel: the
    same steps as the oracle, V within the parity bars.  Targets: a tilted
    half plane (one-signed x and y gradients: alpha shrinks) or a disk."""
    from paper_2012_04011_amd import hj

    if kernel != "plane":
        monkeypatch.setenv("HJ_STAGE_KERNEL", kernel)
    g = W.car_grid(26, 24, 8, 16)
    x, y = oracle.nodes(g, 0), oracle.nodes(g, 1)
    X, Y = x[:, None, None, None], y[None, :, None, None]
    if target == "plane":
        V0 = 0.8 * X + 0.6 * Y - 1.0 + np.zeros(g["n"])
    else:
        V0 = np.sqrt(X * X + Y * Y) - 1.0 + np.zeros(g["n"])
    sch = W.scheme("upwind1", "rk2", alpha="deriv_range")
    ref, oinfo = oracle.solve(g, dyn, sch, V0, 0.6)
    with hj.Grid(g, dyn, sch, precision) as h:
        h.set_target(V0)
        info = h.solve_brt(0.6)
        assert h.launch_info()["kernel"] == kernel
        V = h.value(np.float64)
    assert info["steps"] == oinfo["steps"]
    assert info["dt"] == pytest.approx(oinfo["dt"], rel=1e-12 if precision == "f64" else 1e-5)
    if precision == "f64":
        assert_f64_close(V, ref)
    else:
        assert_f32_close(V, ref, g, "upwind1")


def test_range_alpha_rejected_where_a_fixed_step_is_needed():
    from paper_2012_04011_amd import hj

    g = W.car_grid(10, 9, 5, 8)
    sch = W.scheme("upwind1", "euler", alpha="deriv_range")
    with hj.Grid(g, W.car_dynamics(), sch, "f32") as h:
        h.set_target_cylinders(*W.cylinders(1, 2))
        with pytest.raises(hj.HJError) as e:
            h.solve_converge(1e-3, 10)
        assert e.value.status == hj.HJ_ERR_UNSUPPORTED
        with pytest.raises(hj.HJError) as e:
            hj.Batch([h])
        assert e.value.status == hj.HJ_ERR_UNSUPPORTED
        dt = h.step()  # one step with its own range-based dt
        assert dt > 0
    with pytest.raises(hj.HJError) as e:
        hj.Server(sch, "f32")
    assert e.value.status == hj.HJ_ERR_UNSUPPORTED


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("deriv,integ", [("eno2", "rk2"), ("upwind1", "euler")])
def test_plane_range_pass_equals_column_pass(monkeypatch, precision, deriv, integ):
    """On plane-kernel grids the derivative range comes from the plane
    kernel's own traversal (the whole plane and a plane split into v
    segments); elsewhere from the one-thread-per-column pass.  The step
    sizes they give agree to rounding (the ends of the open axes take the
    closed-form one-sided differences in the one, extrapolated ghosts in the
    other), and so do the values."""
    from paper_2012_04011_amd import hj

    grid = W.car_grid(18, 16, 10, 24)
    dyn = W.car_dynamics(d_max=0.1)
    sch = W.scheme(deriv, integ, alpha="deriv_range")
    V0 = oracle.target_cylinders(grid, *W.cylinders(21, 3))
    monkeypatch.setenv("HJ_X_CHUNKS", "2")
    out = {}
    for kernel, vseg in (("stream", None), ("plane", None), ("plane", "4")):
        if kernel == "stream":
            monkeypatch.setenv("HJ_STAGE_KERNEL", "stream")
        else:
            monkeypatch.delenv("HJ_STAGE_KERNEL", raising=False)
        if vseg:
            monkeypatch.setenv("HJ_PLANE_VSEG", vseg)
        else:
            monkeypatch.delenv("HJ_PLANE_VSEG", raising=False)
        with hj.Grid(grid, dyn, sch, precision) as g:
            li = g.launch_info()
            assert li["kernel"] == kernel and (li["plane_segments"] > 1) == (vseg is not None)
            g.set_target(V0)
            info = g.solve_brt(0.3)
            out[(kernel, vseg)] = (info, g.value(np.float64))
    ref_info, ref_v = out[("stream", None)]
    rel = 1e-5 if precision == "f32" else 1e-12
    for key, (info, v) in out.items():
        assert info["steps"] == ref_info["steps"], key
        assert info["dt"] == pytest.approx(ref_info["dt"], rel=rel), key
        assert info["dt_last"] == pytest.approx(ref_info["dt_last"], rel=1e-3, abs=1e-9), key
        assert np.abs(v - ref_v).max() <= (1e-4 if precision == "f32" else 1e-10), key
