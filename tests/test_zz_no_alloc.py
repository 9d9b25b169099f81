"""hj_optimal_control_noalloc -- the control query (eq (9)) for callers that
cannot allocate device memory -- against hj_optimal_control, the entry point
it varies (the same kernel on the same V, so the results are bitwise equal):
two calls in a row, the second with fewer states, host and device arrays,
both precisions, and the size limit."""

from __future__ import annotations

import numpy as np
import pytest

from paper_2012_04011_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


def _states(rng, m):
    # inside and beyond the grid on the open axes, several periods on theta
    return np.column_stack([rng.uniform(-5.5, 5.5, m), rng.uniform(-5.5, 5.5, m), rng.uniform(-0.2, 2.2, m),
                            rng.uniform(-7.0, 7.0, m)])


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("dyn", [W.car_dynamics(), W.steer_dynamics()], ids=["car", "steer"])
def test_noalloc_control_equals_allocating_query(precision, dyn):
    from paper_2012_04011_amd import hj

    grid = W.car_grid(30, 28, 12, 20)
    rng = np.random.default_rng(17)
    with hj.Grid(grid, dyn, W.scheme("eno2", "rk2"), precision) as g:
        g.set_target_cylinders(*W.cylinders(13, 4))
        g.solve_brt(0.4)
        for m in (5000, 37):  # the second call smaller than the first
            z = _states(rng, m)
            u, val = g.optimal_control_noalloc(z)
            u_ref, val_ref = g.optimal_control(z)
            assert u.shape == (m, 2) and val.shape == (m,)
            assert np.array_equal(u, u_ref) and np.array_equal(val, val_ref), m


def test_noalloc_control_device_arrays_and_limit():
    import torch
    from paper_2012_04011_amd import hj

    grid = W.car_grid(26, 24, 10, 16)
    rng = np.random.default_rng(23)
    with hj.Grid(grid, W.car_dynamics(), W.scheme("upwind1", "euler"), "f32") as g:
        g.set_target_cylinders(*W.cylinders(4, 3))
        g.solve_brt(0.3)
        z = _states(rng, hj.HJ_NOALLOC_MAX_STATES)
        u, val = g.optimal_control_noalloc(z)  # the largest size it takes
        u_ref, val_ref = g.optimal_control(z)
        assert np.array_equal(u, u_ref) and np.array_equal(val, val_ref)
        zd = torch.tensor(z[:1000], device="cuda")
        ud, vd = g.optimal_control_noalloc(zd)
        torch.cuda.synchronize()
        assert np.array_equal(ud.cpu().numpy(), u_ref[:1000]) and np.array_equal(vd.cpu().numpy(), val_ref[:1000])
        with pytest.raises(hj.HJError) as e:
            g.optimal_control_noalloc(_states(rng, hj.HJ_NOALLOC_MAX_STATES + 1))
        assert e.value.status == hj.HJ_ERR_INVALID_ARG
        # the rejected call left the staging untouched for the next one
        u2, val2 = g.optimal_control_noalloc(z[:64])
        assert np.array_equal(u2, u_ref[:64]) and np.array_equal(val2, val_ref[:64])
