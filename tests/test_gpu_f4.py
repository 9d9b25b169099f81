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


@pytest.mark.parametrize("alpha", ["deriv_range", "deriv_range_onesided"], ids=["central", "onesided"])
@pytest.mark.parametrize("kernel", ["plane", "stream", "generic"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("name,dyn,target", CASES, ids=[c[0] for c in CASES])
def test_range_alpha_solve_matches_oracle(monkeypatch, kernel, precision, name, dyn, target, alpha):
    """Whole solves in both derivative-range modes (Algorithm 1's central
    derivative, and both one-sided ones) on every stage kernel: the same
    steps as the oracle, V within the parity bars.  Targets: a tilted half
    plane (one-signed x and y gradients: alpha shrinks) or a disk."""
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
    sch = W.scheme("upwind1", "rk2", alpha=alpha)
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
        assert_f32_close(V, ref, g)


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


@pytest.mark.parametrize("kernel", ["plane", "stream", "generic"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_range_modes_differ_on_sawtooth(monkeypatch, kernel, precision):
    """V_i = b (-1)^i on a periodic x axis: every central difference is 0,
    the one-sided ones are +-2b/h.  With z' = 0.5 + u on x, |u| <= 1
    minimising, Algorithm 1's central box gives alpha_x = 0.5 and the
    one-sided box 1.5 (hand-derived; the oracle pin checks the same), so
    dt = 0.8 h / 0.5 or 0.8 h / 1.5; V stays a sawtooth, so every step
    keeps that dt."""
    from paper_2012_04011_amd import hj

    if kernel != "plane":
        monkeypatch.setenv("HJ_STAGE_KERNEL", kernel)
    g = {"n": (8, 6, 4, 8), "lo": (0.0, -1.0, 0.0, -math.pi), "hi": (8.0, 1.0, 2.0, math.pi),
         "periodic_mask": 1 | 8}
    saw = 0.25 * (-1.0) ** np.arange(8)
    V0 = np.broadcast_to(saw[:, None, None, None], g["n"]).copy()
    dyn = drift_dyn((0.5, 0, 0, 0), (0,), 1.0, "box", "min")
    for alpha, ax in (("deriv_range", 0.5), ("deriv_range_onesided", 1.5)):
        sch = W.scheme("upwind1", "euler", clamp=False, alpha=alpha)
        ref, oinfo = oracle.solve(g, dyn, sch, V0, 4.0)
        with hj.Grid(g, dyn, sch, precision) as h:
            h.set_target(V0)
            info = h.solve_brt(4.0)
            assert h.launch_info()["kernel"] == kernel
            V = h.value(np.float64)
        assert info["dt"] == pytest.approx(0.8 / ax, rel=1e-12 if precision == "f64" else 1e-6), alpha
        assert info["steps"] == oinfo["steps"], alpha
        np.testing.assert_allclose(V, ref, rtol=0, atol=1e-12 if precision == "f64" else 1e-6)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_range_modes_differ_ball_open_axes(precision):
    """V = a x + b (-1)^i + c y on open x, y axes with a unit-ball input on
    (x, y): the central x box is [a - 2b/h, a], the one-sided one
    [a - 2b/h, a + 2b/h], so alpha_x = M / sqrt(M^2 + c^2) with M = a or
    a + 2b/h and alpha_y = c / sqrt(c^2 + (a - 2b/h)^2); the first step is
    0.8 / (alpha_x / h_x + alpha_y / h_y) (hand-derived, as in the oracle
    pin)."""
    from paper_2012_04011_amd import hj

    nx = 10
    g = {"n": (nx, 6, 4, 8), "lo": (-2.0, -1.0, 0.0, -math.pi), "hi": (2.5, 1.5, 2.0, math.pi),
         "periodic_mask": 8}
    hx, hy = 4.5 / (nx - 1), 2.5 / 5
    a, c = 1.0, 1.0
    b = 0.25 * hx
    x, y = oracle.nodes(g, 0), oracle.nodes(g, 1)
    V0 = (a * x + b * (-1.0) ** np.arange(nx))[:, None, None, None] + c * y[None, :, None, None] \
        + np.zeros(g["n"])
    dyn = drift_dyn((0, 0, 0, 0), (0, 1), 1.0, "ball", "max")
    for alpha, M in (("deriv_range", a), ("deriv_range_onesided", a + 0.5)):
        sch = W.scheme("upwind1", "euler", clamp=False, alpha=alpha)
        ax = M / math.sqrt(M * M + c * c)
        ay = c / math.sqrt(c * c + (a - 0.5) ** 2)
        with hj.Grid(g, dyn, sch, precision) as h:
            h.set_target(V0)
            info = h.solve_brt(5.0)
        dt = 0.8 / (ax / hx + ay / hy)
        assert info["dt"] == pytest.approx(dt, rel=1e-12 if precision == "f64" else 1e-5), alpha
