"""hj_solve_brt's time loop replayed from a captured HIP graph.

On grids whose arrays are at most 64 MiB the solve loop is captured once per
(steps, step sizes, starting buffers, launch configuration) and replayed;
HJ_SOLVE_GRAPH=0/1 forces it off or on.  The graph runs the same kernels
with the same arguments, so every result must equal the plain loop's bit
for bit: repeated solves (graph reuse), new targets, odd and even step
counts (the buffer roles alternate), steps between solves, the autotuner
changing the launch configuration, profiling.
"""

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


def _session(monkeypatch, graph: str, precision: str, scheme: dict):
    """Solves, steps and re-solves on one handle; every value read back."""
    from paper_2012_04011_amd import hj

    monkeypatch.setenv("HJ_SOLVE_GRAPH", graph)
    grid = W.car_grid(24, 22, 10, 16)
    outs = []
    with hj.Grid(grid, W.car_dynamics(d_max=0.1), scheme, precision) as g:
        assert g.launch_info()["solve_graph"] == (graph == "1")
        g.set_profiling(True)
        dt = g.cfl_dt()
        for seed, steps in [(0, 7), (0, 7), (1, 7), (2, 8), (2, 8), (3, 7)]:
            g.set_target_cylinders(*W.cylinders(seed, 3))
            info = g.solve_brt((steps - 0.5) * dt)  # the last step shortened to dt / 2
            assert info["steps"] == steps
            outs.append(g.value(np.float64))
        g.step()  # one plain step between solves shifts the buffer roles
        outs.append(g.value(np.float64))
        info = g.solve_brt(5 * dt + 0.5 * dt)
        outs.append(g.value(np.float64))
        prof = g.profile()
        assert prof["solves"] == 7
    return outs


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("deriv,integ", [("eno2", "rk2"), ("upwind1", "euler")])
def test_solve_graph_equals_plain_loop(monkeypatch, precision, deriv, integ):
    sch = W.scheme(deriv, integ)
    plain = _session(monkeypatch, "0", precision, sch)
    graph = _session(monkeypatch, "1", precision, sch)
    for i, (a, b) in enumerate(zip(plain, graph)):
        assert np.array_equal(a, b), i
    # the same target solved twice gives the same V (graph replay)
    assert np.array_equal(graph[0], graph[1]) and np.array_equal(graph[3], graph[4])


def test_solve_graph_follows_launch_changes(monkeypatch):
    """A handle whose launch configuration changes between solves (autotune
    after solves with autotuning off) still gives the plain loop's V."""
    from paper_2012_04011_amd import hj

    grid = W.car_grid(30, 28, 12, 24)
    sch = W.scheme("eno2", "rk2")
    cyl = W.cylinders(4, 4)
    res = {}
    for graph in ("0", "1"):
        monkeypatch.setenv("HJ_SOLVE_GRAPH", graph)
        with hj.Grid(grid, W.car_dynamics(), sch, "f32") as g:
            g.set_autotune(False)
            g.set_target_cylinders(*cyl)
            g.solve_brt(0.2)
            a = g.value()
            before = g.launch_info()
            g.autotune()
            after = g.launch_info()
            g.solve_brt(0.2)
            b = g.value()
            g.set_target(g.target())  # the full-target form: another clamp path
            g.solve_brt(0.2)
            c = g.value()
        res[graph] = (a, b, c)
        print(graph, before["kernel"], before["x_chunks"], "->", after["kernel"], after["x_chunks"])
    for x, y in zip(res["0"], res["1"]):
        assert np.array_equal(x, y)
    assert np.array_equal(res["1"][0], res["1"][1]) and np.array_equal(res["1"][1], res["1"][2])


def test_solve_graph_default_by_size(monkeypatch):
    from paper_2012_04011_amd import hj

    monkeypatch.delenv("HJ_SOLVE_GRAPH", raising=False)
    with hj.Grid(W.car_grid(60, 60, 20, 36), W.car_dynamics(), W.scheme("eno2", "rk2"), "f32") as g:
        assert g.launch_info()["solve_graph"]
    wl = W.LARGE_120
    with hj.Grid(wl.grid, wl.dyn, wl.scheme, "f32") as g:
        assert not g.launch_info()["solve_graph"]
