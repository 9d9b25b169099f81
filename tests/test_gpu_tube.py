"""Closed-form properties of the BRT computed on the HIP path (through the C
ABI): the tube only grows (the clamp V = min(V0, V) of eq (4) and
Algorithm 2; first-order upwind is a monotone scheme) and the car's
mirror and quarter-turn symmetries carry over to the solution."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import U32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("deriv,integ", [("upwind1", "euler"), ("upwind1", "rk2"), ("eno2", "rk2")])
def test_tube_is_monotone(precision, deriv, integ):
    """Every step: V^n <= V0 bit for bit (the clamp).  First-order upwind with
    CFL <= 1 is monotone (each update a convex combination of neighbours;
    TVD-RK2 a convex combination of Euler steps), so no node leaves
    {V <= 0}.  ENO2 is not monotone: a node may leave, but only one lying
    within 0.1 h of the zero level set (the same bars as the oracle's own
    check).  The tube grows."""
    from paper_2012_04011_amd import hj

    g = W.car_grid(24, 24, 8, 12)
    dyn = W.car_dynamics()
    sch = W.scheme(deriv, integ)
    cyl = W.cylinders(5, 3)
    h = 10.0 / 23
    dt = oracle.cfl_dt(g, dyn, 0.8, 1.0)
    dtype = np.float32 if precision == "f32" else np.float64
    with hj.Grid(g, dyn, sch, precision) as grid:
        grid.set_target_cylinders(*cyl)
        V0 = grid.target(dtype)
        V = grid.value(dtype)
        sizes = [int((V0 <= 0).sum())]
        for _ in range(20):
            grid.step(dt)
            Vn = grid.value(dtype)
            assert np.all(Vn <= V0)
            lost = (V <= 0) & (Vn > 0)
            if deriv == "upwind1":
                assert not lost.any(), int(lost.sum())
            else:
                assert np.all(V[lost] > -0.1 * h) and np.all(Vn[lost] < 0.1 * h)
            sizes.append(int((Vn <= 0).sum()))
            V = Vn
    assert sizes[-1] > sizes[1] > sizes[0]


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_mirror_and_quarter_turn_symmetry(precision):
    """The car is invariant under the mirror (x, y, theta) -> (x, -y, -theta)
    and the quarter turn (x, y, theta) -> (y, -x, theta - pi/2) (N_x = N_y,
    equal ranges, N_theta % 4 == 0).  Solving for the mirrored / rotated
    obstacles gives the mirrored / rotated value function: with first-order
    upwind + Euler to rounding -- FP64 1e-11 as on the oracle; FP32: two
    solves whose every step is within 16 u max(|V|, 1) of exact arithmetic
    (the one-step bar) under a monotone, non-expanding scheme differ by at
    most 2 n 16 u max |V| after n steps."""
    g = W.car_grid(20, 20, 6, 12)
    dyn = W.car_dynamics()
    sch = W.scheme("upwind1", "euler")
    cx, cy, r = W.cylinders(7, 3)
    T = 0.5

    def solve(cxs, cys):
        from helpers import gpu_solve

        V, V0, info = gpu_solve(g, dyn, sch, precision, T, cylinders=(cxs, cys, r))
        return V, V0, info

    V, V0, info = solve(cx, cy)
    if precision == "f64":
        tol = 1e-11
    else:
        tol = 2 * info["steps"] * 16 * U32 * max(float(np.abs(V0).max()), 1.0)
    Vm, _, _ = solve(cx, -cy)
    lidx = (-np.arange(12)) % 12
    mapped = V[:, ::-1, :, :][:, :, :, lidx]
    assert np.abs(Vm - mapped).max() <= tol, (float(np.abs(Vm - mapped).max()), tol)
    # node (i, j, l) of the rotated problem holds the original value at
    # (N - 1 - j, i, l + N / 4)
    Vr, _, _ = solve(cy, -cx)
    rot = np.roll(np.transpose(V, (1, 0, 2, 3))[:, ::-1, :, :], -3, axis=3)
    assert np.abs(Vr - rot).max() <= tol, (float(np.abs(Vr - rot).max()), tol)
