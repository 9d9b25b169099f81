"""Batched solves through the C ABI (hj_batch_*): every instance of a batch
must equal the single-grid solve of the same handle bit for bit (the batch
kernels evaluate each node with the single-grid kernels' arithmetic), in all
four modes (one launch per step and stage; the same launches replayed from
a hipGraph; one persistent launch; each instance's own solve on concurrent
streams); and the batch must match the oracle."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import assert_f64_close, check_f32_solve, xfail_if_missed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()

MODES = ["launches", "graph", "persistent", "streams"]


def small_batch(precision: str):
    """Six uneven instances: theta runs of 4, 2 and 1, horizons giving 0, 1
    and many steps, with and without a disturbance in FP64 (a batch mixes
    dynamics freely)."""
    shapes = [(14, 12, 6, 16), (11, 13, 5, 18), (9, 10, 7, 19), (12, 9, 5, 21), (10, 11, 6, 8), (8, 8, 4, 3)]
    horizons = [0.6, 0.35, 0.0, 0.5, 0.01, 0.45]
    out = []
    for i, (n, T) in enumerate(zip(shapes, horizons)):
        dyn = W.car_dynamics(d_max=0.1 if (precision == "f64" and i % 2) else 0.0)
        out.append(W.Instance(W.car_grid(*n), dyn, W.scheme("eno2", "rk2"), W.cylinders(40 + i, 1 + i % 4), T))
    return out


def make_grids(hj, insts, precision):
    grids = []
    for ins in insts:
        g = hj.Grid(ins.grid, ins.dyn, ins.scheme, precision)
        g.set_target_cylinders(*ins.cylinders)
        grids.append(g)
    return grids


def single_solutions(hj, insts, precision):
    vals, infos = [], []
    for ins in insts:
        with hj.Grid(ins.grid, ins.dyn, ins.scheme, precision) as g:
            g.set_target_cylinders(*ins.cylinders)
            infos.append(g.solve_brt(ins.horizon))
            vals.append(g.value(np.float64))
    return vals, infos


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_equals_single_solves(mode, precision):
    from paper_2012_04011_amd import hj

    insts = small_batch(precision)
    ref, ref_infos = single_solutions(hj, insts, precision)
    grids = make_grids(hj, insts, precision)
    with hj.Batch(grids) as b:
        for tile in (16, 5):  # two tile shapes, the second re-plans (and re-captures the graph)
            for g, ins in zip(grids, insts):
                g.set_target_cylinders(*ins.cylinders)
            b.set_tile(tile)
            infos = b.solve([i.horizon for i in insts], mode)
            for j, g in enumerate(grids):
                assert infos[j]["steps"] == ref_infos[j]["steps"]
                assert infos[j]["dt"] == ref_infos[j]["dt"] and infos[j]["dt_last"] == ref_infos[j]["dt_last"]
                assert np.array_equal(g.value(np.float64), ref[j]), (mode, tile, j)
        info = b.info()
        assert info["m"] == len(insts) and info["x_planes"] == 5
        assert info["points"] == sum(i.points for i in insts)
        assert info["plane_kernel"] == (1 if mode in ("launches", "graph") else 0)
        if mode == "graph":
            # a node per (step, stage) of each launch class
            nmax = max(r["steps"] for r in ref_infos)
            assert 2 * nmax <= info["graph_nodes"] <= 2 * nmax * info["classes"]
        if mode == "persistent":
            assert info["persistent_blocks"] >= 1
    for g in grids:
        g.close()


def plane_batch(precision: str):
    """Instances that take every path of the batched launches: plane blocks
    with theta runs of 4, 3 and 2, planes split into v segments (runs of 2
    with more runs per plane than a block has work-items), one whose runs of
    3 would not fit a batched block, streaming tiles for runs of one (prime
    N_theta), and horizons of 0, 1 and many steps."""
    shapes = [(14, 12, 6, 16), (11, 13, 9, 21), (9, 10, 7, 18), (10, 9, 20, 43), (12, 8, 40, 60),
              (13, 11, 5, 19), (9, 9, 4, 3), (8, 8, 80, 30)]
    horizons = [0.6, 0.35, 0.0, 0.3, 0.2, 0.5, 0.01, 0.2]
    out = []
    for i, (n, T) in enumerate(zip(shapes, horizons)):
        dyn = W.car_dynamics(d_max=0.1 if (precision == "f64" and i % 2) else 0.0)
        out.append(W.Instance(W.car_grid(*n), dyn, W.scheme("eno2", "rk2"), W.cylinders(60 + i, 1 + i % 4), T))
    return out


@pytest.mark.parametrize("mode", ["launches", "graph"])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_plane_kernel_equals_single_solves(monkeypatch, mode, precision):
    """The batched plane kernel (an instance's blocks hold a y row's
    (v, theta) plane in LDS; launch classes by block size, each on its own
    lane, beside a class of streaming tiles) on instances covering its run
    lengths and split planes, at three block lengths (the second and third
    re-plan), bitwise equal to the single-grid solves; the streaming tiles
    alone (HJ_BATCH_KERNEL=stream) give the same."""
    from paper_2012_04011_amd import hj

    insts = plane_batch(precision)
    ref, ref_infos = single_solutions(hj, insts, precision)
    for kernel in ("plane", "stream"):
        if kernel == "stream":
            monkeypatch.setenv("HJ_BATCH_KERNEL", "stream")
        else:
            monkeypatch.delenv("HJ_BATCH_KERNEL", raising=False)
        grids = make_grids(hj, insts, precision)
        with hj.Batch(grids) as b:
            for tile in (0, 7, 100):
                for g, ins in zip(grids, insts):
                    g.set_target_cylinders(*ins.cylinders)
                b.set_tile(tile)
                infos = b.solve([i.horizon for i in insts], mode)
                info = b.info()
                assert info["plane_kernel"] == (1 if kernel == "plane" else 0), (kernel, tile)
                assert (info["classes"] >= 3) if kernel == "plane" else (info["classes"] == 1)
                assert info["x_planes"] == (tile if tile else (32 if kernel == "plane" else 16))
                for j, g in enumerate(grids):
                    assert infos[j]["steps"] == ref_infos[j]["steps"]
                    assert np.array_equal(g.value(np.float64), ref[j]), (kernel, tile, j)
        for g in grids:
            g.close()


def test_batch_plane_kernel_beside_streaming_tiles():
    """A plane with more theta nodes than a block holds work-items, on a
    prime N_theta (runs of one), beside a grid with runs of four: the one
    runs on the streaming tiles, the other on the plane kernel, in two
    classes, bitwise equal to the single solves; with runs of one alone the
    batch is one class of streaming tiles."""
    from paper_2012_04011_amd import hj

    insts = [W.Instance(W.car_grid(8, 7, 4, 769), W.car_dynamics(), W.scheme("eno2", "rk2"), W.cylinders(5, 2), 0.05),
             W.Instance(W.car_grid(12, 10, 6, 16), W.car_dynamics(), W.scheme("eno2", "rk2"), W.cylinders(6, 2), 0.3)]
    ref, _ = single_solutions(hj, insts, "f32")
    grids = make_grids(hj, insts, "f32")
    with hj.Batch(grids) as b:
        b.solve([i.horizon for i in insts], "launches")
        assert b.info()["plane_kernel"] == 1 and b.info()["classes"] == 2
        for j, g in enumerate(grids):
            assert np.array_equal(g.value(np.float64), ref[j]), j
    with hj.Batch(grids[:1]) as b:
        grids[0].set_target_cylinders(*insts[0].cylinders)
        b.solve([insts[0].horizon], "graph")
        assert b.info()["plane_kernel"] == 0 and b.info()["classes"] == 1
        assert np.array_equal(grids[0].value(np.float64), ref[0])
    for g in grids:
        g.close()


def test_batch_graph_replays_with_new_targets():
    """The captured graph is replayed (same step counts) with new obstacle
    sets and eager work in between; every replay equals the single solves."""
    from paper_2012_04011_amd import hj

    insts = small_batch("f32")
    grids = make_grids(hj, insts, "f32")
    with hj.Batch(grids) as b:
        for rep in range(3):
            moved = [W.Instance(i.grid, i.dyn, i.scheme, W.cylinders(100 * rep + j, 3), i.horizon)
                     for j, i in enumerate(insts)]
            for g, ins in zip(grids, moved):
                g.set_target_cylinders(*ins.cylinders)
            b.solve([i.horizon for i in moved], "graph")
            ref, _ = single_solutions(hj, moved, "f32")  # eager solves between replays
            for j, g in enumerate(grids):
                assert np.array_equal(g.value(np.float64), ref[j]), (rep, j)
    for g in grids:
        g.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_matches_oracle(precision):
    from paper_2012_04011_amd import hj

    insts = small_batch(precision)[:4]
    grids = make_grids(hj, insts, precision)
    with hj.Batch(grids) as b:
        infos = b.solve([i.horizon for i in insts], "persistent")
    ms = []
    for ins, g, info in zip(insts, grids, infos):
        V0 = oracle.target_cylinders(ins.grid, *ins.cylinders)
        ref, oinfo = oracle.solve(ins.grid, ins.dyn, ins.scheme, V0, ins.horizon)
        assert info["steps"] == oinfo["steps"]
        V = g.value(np.float64)
        if precision == "f64":
            assert_f64_close(V, ref)
        else:
            ms.append(check_f32_solve(V, ref, ins.grid, "eno2", defer=True))
        g.close()
    xfail_if_missed(ms)


def test_batch_persistent_spin_limit_error_path():
    """A spin limit of 0 makes a tile give up as soon as its dependency is
    not yet met: the kernel still ends, the call reports a device error (or,
    if no tile ever had to wait, the results are right), and the next solve
    with the default limit is correct."""
    from paper_2012_04011_amd import hj

    insts = small_batch("f32")
    ref, _ = single_solutions(hj, insts, "f32")
    grids = make_grids(hj, insts, "f32")
    with hj.Batch(grids) as b:
        b.set_spin_limit(0)
        try:
            b.solve([i.horizon for i in insts], "persistent")
            for j, g in enumerate(grids):
                assert np.array_equal(g.value(np.float64), ref[j])
        except hj.HJError as e:
            assert e.status == hj.HJ_ERR_DEVICE
        b.set_spin_limit(1 << 21)
        for g, ins in zip(grids, insts):
            g.set_target_cylinders(*ins.cylinders)
        b.solve([i.horizon for i in insts], "persistent")
        for j, g in enumerate(grids):
            assert np.array_equal(g.value(np.float64), ref[j])
    for g in grids:
        g.close()


def test_batch_autotune_picks_a_candidate():
    from paper_2012_04011_amd import hj

    insts = small_batch("f32")
    ref, _ = single_solutions(hj, insts, "f32")
    grids = make_grids(hj, insts, "f32")
    with hj.Batch(grids) as b:
        t = b.autotune([i.horizon for i in insts], "launches")
        assert t in (4, 8, 12, 16, 24, 32, 48, 80) and b.info()["x_planes"] == t
        for j, g in enumerate(grids):
            assert np.array_equal(g.value(np.float64), ref[j])
    for g in grids:
        g.close()


@pytest.mark.parametrize("mode", ["graph", "persistent", "streams"])
def test_batch_64_uneven_sampled(mode):
    """The 64-instance uneven batch (30x30x12x18 .. 80x80x24x48, 1-8
    cylinders, horizons 0.5-2 s) through the batched plane kernel's graph,
    in one persistent launch and on concurrent streams: five instances (the
    largest, the smallest, the longest and the shortest horizon, and one
    with a prime N_theta, which runs on the streaming tiles) equal their
    single-grid solves bit for bit."""
    from paper_2012_04011_amd import hj

    insts = W.batch_instances(**W.BATCH_64)
    grids = make_grids(hj, insts, "f32")
    with hj.Batch(grids) as b:
        infos = b.solve([i.horizon for i in insts], mode)
        assert b.info()["points"] == sum(i.points for i in insts)
        assert b.info()["plane_kernel"] == (1 if mode == "graph" else 0)
    pick = {int(np.argmax([i.points for i in insts])), int(np.argmin([i.points for i in insts])),
            int(np.argmax([i.horizon for i in insts])), int(np.argmin([i.horizon for i in insts])),
            next(j for j, i in enumerate(insts) if i.grid["n"][2] * i.grid["n"][3] > 768 and i.grid["n"][3] == 43)}
    sub = [insts[j] for j in sorted(pick)]
    ref, ref_infos = single_solutions(hj, sub, "f32")
    for r, ri, j in zip(ref, ref_infos, sorted(pick)):
        assert infos[j]["steps"] == ri["steps"]
        assert np.array_equal(grids[j].value(np.float64), r), j
    for g in grids:
        g.close()


def test_batch_streams_mode_ordering_and_errors():
    """The streams mode is ordered on the batch stream (eager work enqueued
    before and after it sees the right values), repeats bitwise, and has no
    tile length to tune."""
    from paper_2012_04011_amd import hj

    insts = small_batch("f32")
    ref, _ = single_solutions(hj, insts, "f32")
    grids = make_grids(hj, insts, "f32")
    H = [i.horizon for i in insts]
    with hj.Batch(grids) as b:
        for rep in range(3):
            for g, ins in zip(grids, insts):
                g.set_target_cylinders(*W.cylinders(90 + rep, 2))  # replaced below, same stream
                g.set_target_cylinders(*ins.cylinders)
            b.solve(H, "streams")
            for j, g in enumerate(grids):
                assert np.array_equal(g.value(np.float64), ref[j]), (rep, j)
        with pytest.raises(hj.HJError) as e:
            b.autotune(H, "streams")
        assert e.value.status == hj.HJ_ERR_INVALID_ARG
    for g in grids:
        g.close()
