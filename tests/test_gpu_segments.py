"""The plane kernel on (v, theta) planes split along v.

A plane with more runs of theta nodes than a block has threads (the FP64
120x120x40x72 grid: 1440 runs) is split into v segments; each block holds
its segment plus two halo rows per side copied from global memory.  The
split must not change any result: every node sees the same neighbour values
as in the unsplit plane and the streaming kernel, so the outputs are bitwise
equal to the streaming kernel's, and they match the oracle to rounding.
HJ_PLANE_VSEG caps the rows per block to force a split on small grids.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import U64, assert_f32_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


# (shape, periodic mask, rows per block): segments of 4..7 rows, a last
# segment of 1..3 rows, runs of 4, 2 and 1 theta nodes, a periodic v axis
SPLITS = [((14, 12, 13, 16), W.THETA_PERIODIC, 4), ((11, 10, 11, 18), W.THETA_PERIODIC, 5),
          ((9, 8, 10, 21), W.THETA_PERIODIC, 4), ((10, 9, 17, 8), W.THETA_PERIODIC, 6),
          ((12, 10, 10, 16), W.THETA_PERIODIC | 4, 4), ((9, 9, 9, 19), W.THETA_PERIODIC | 4, 5)]


def _segments(nv: int, rows: int) -> int:
    """The library's split: the fewest segments of at most `rows` rows,
    balanced."""
    if nv <= rows:
        return 1
    n = -(-nv // rows)
    per = -(-nv // n)
    return -(-nv // per)


def _one_step(monkeypatch, shape, pmask, rows, precision, deriv, integ, kernel, dyn=None):
    from paper_2012_04011_amd import hj

    if kernel == "stream":
        monkeypatch.setenv("HJ_STAGE_KERNEL", "stream")
        monkeypatch.delenv("HJ_PLANE_VSEG", raising=False)
    else:
        monkeypatch.delenv("HJ_STAGE_KERNEL", raising=False)
        monkeypatch.setenv("HJ_PLANE_VSEG", str(rows))
    monkeypatch.setenv("HJ_X_CHUNKS", "3")
    grid = dict(W.car_grid(*shape), periodic_mask=pmask)
    dyn = dyn or W.car_dynamics(d_max=0.1)
    sch = W.scheme(deriv, integ)
    V0 = oracle.target_cylinders(grid, *W.cylinders(5, 4))
    rng = np.random.default_rng(sum(shape))
    Vk = np.minimum(V0, V0 + 0.02 * rng.standard_normal(V0.shape))
    if precision == "f32":
        Vk = Vk.astype(np.float32).astype(np.float64)
    dt = oracle.cfl_dt(grid, dyn, 0.8, 1.0)
    with hj.Grid(grid, dyn, sch, precision) as g:
        g.set_target(V0)
        g.set_value(Vk)
        g.step(dt)
        info = g.launch_info()
        V = g.value()
    return grid, dyn, sch, V0, Vk, dt, V, info


@pytest.mark.parametrize("shape,pmask,rows", SPLITS, ids=lambda x: str(x))
@pytest.mark.parametrize("deriv,integ", [("eno2", "rk2"), ("upwind1", "euler")])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_split_plane_one_step(monkeypatch, shape, pmask, rows, deriv, integ, precision):
    """One step from a rough input with a disturbance and the clamp on:
    the split plane kernel equals the streaming kernel bit for bit and the
    oracle to rounding."""
    grid, dyn, sch, V0, Vk, dt, V, info = _one_step(monkeypatch, shape, pmask, rows, precision, deriv, integ,
                                                     "plane")
    assert info["kernel"] == "plane" and info["plane_segments"] == _segments(shape[2], rows) > 1, info
    *_, Vs, sinfo = _one_step(monkeypatch, shape, pmask, rows, precision, deriv, integ, "stream")
    assert sinfo["kernel"] == "stream" and sinfo["plane_segments"] == 0
    assert np.array_equal(V, Vs)
    if precision == "f64":
        ref = oracle.step(grid, dyn, sch, V0, Vk, dt)
        bad = np.abs(V - ref) > 16 * U64 * np.maximum(np.abs(ref), 1.0)
        assert not bad.any(), (int(bad.sum()), float(np.abs(V - ref).max()))
    else:
        assert_f32_step(V, grid, dyn, sch, V0, Vk, dt)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_split_plane_ball_input(monkeypatch, precision):
    """The test dynamics with a Euclidean-ball input on x, y and theta (the
    ball term couples the axes) and drift on every axis, on a split plane
    with a periodic v axis: bitwise the streaming kernel, the oracle to
    rounding."""
    dyn = {"kind": "drift_input", "drift": (0.3, -0.2, 0.15, 0.4), "in_axes": (0, 1, 3), "in_speed": 0.6,
           "in_norm": "ball", "in_role": "min"}
    shape, pmask, rows = (11, 10, 13, 16), W.THETA_PERIODIC | 4, 5
    grid, dyn, sch, V0, Vk, dt, V, info = _one_step(monkeypatch, shape, pmask, rows, precision, "eno2", "rk2",
                                                     "plane", dyn)
    assert info["kernel"] == "plane" and info["plane_segments"] == _segments(shape[2], rows), info
    *_, Vs, _ = _one_step(monkeypatch, shape, pmask, rows, precision, "eno2", "rk2", "stream", dyn)
    assert np.array_equal(V, Vs)
    if precision == "f64":
        ref = oracle.step(grid, dyn, sch, V0, Vk, dt)
        bad = np.abs(V - ref) > 16 * U64 * np.maximum(np.abs(ref), 1.0)
        assert not bad.any(), (int(bad.sum()), float(np.abs(V - ref).max()))
    else:
        assert_f32_step(V, grid, dyn, sch, V0, Vk, dt)


def test_split_plane_solve_and_chunks(monkeypatch):
    """A short ENO2 + TVD-RK2 FP64 solve on a split plane: the same V for
    every x-chunking and rows-per-block choice, and the same as unsplit."""
    from paper_2012_04011_amd import hj

    grid = W.car_grid(16, 14, 12, 24)
    dyn = W.car_dynamics(d_max=0.1)
    sch = W.scheme("eno2", "rk2")
    cyl = W.cylinders(3, 3)
    outs = {}
    for rows, chunks in [(None, "1"), (4, "1"), (4, "4"), (5, "2"), (7, "3")]:
        if rows is None:
            monkeypatch.delenv("HJ_PLANE_VSEG", raising=False)
        else:
            monkeypatch.setenv("HJ_PLANE_VSEG", str(rows))
        monkeypatch.setenv("HJ_X_CHUNKS", chunks)
        with hj.Grid(grid, dyn, sch, "f64") as g:
            g.set_target_cylinders(*cyl)
            g.solve_brt(0.25)
            info = g.launch_info()
            assert info["kernel"] == "plane"
            assert info["plane_segments"] == (1 if rows is None else _segments(12, rows)), (rows, info)
            outs[(rows, chunks)] = g.value()
    ref = outs[(None, "1")]
    for k, v in outs.items():
        assert np.array_equal(v, ref), k


def test_large_f64_runs_split_plane():
    """The FP64 120x120x40x72 grid (1440 runs of two theta nodes per plane)
    runs the plane kernel in two v segments."""
    from paper_2012_04011_amd import hj

    wl = W.LARGE_120
    with hj.Grid(wl.grid, wl.dyn, wl.scheme, "f64") as g:
        info = g.launch_info()
    assert info["kernel"] == "plane" and info["plane_segments"] == 2, info
