"""The continuous-batching server (hj_server_*): requests that arrive while
others are stepping are admitted as slots and memory free up, step together
in shared launches, and each result equals the same re-solve alone (a fresh
handle's hj_solve_brt) bit for bit; the memory budget bounds the slots."""

from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
from paper_2012_04011_amd import workloads as W

from helpers import assert_f64_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_04011_amd import hj

    hj.load_library()


SMALL_GRIDS = (W.car_grid(20, 18, 8, 12), W.car_grid(16, 17, 6, 9))


def small_requests(n=10):
    return W.serving_requests(n, rate=1000.0, seed=3, mix=0.6, horizon=0.4, grids=SMALL_GRIDS)


def alone(hj, req, precision="f32", scheme=None):
    with hj.Grid(req.grid, req.dyn, scheme or W.scheme("eno2", "rk2"), precision) as g:
        g.set_target_cylinders(*req.cylinders)
        info = g.solve_brt(req.horizon)
        return g.value(np.float64), info


def drain(srv, ids, results, shapes, max_ticks=100000):
    ticks = 0
    while len(results) < len(ids):
        srv.tick()
        ticks += 1
        assert ticks < max_ticks
        for rid in srv.poll():
            out = np.empty(shapes[rid], np.float64)
            srv.take(rid, out)
            results[rid] = out
    return ticks


@pytest.mark.parametrize("policy", ["small_first", "share"])
@pytest.mark.parametrize("max_inflight,steps_per_tick", [(3, 1), (5, 3), (64, 0)])
def test_served_equals_alone(max_inflight, steps_per_tick, policy):
    """Requests submitted between ticks (others already stepping), a queue
    when max_inflight is small, slots reused across requests of one shape,
    requests finishing inside a multi-step tick."""
    from paper_2012_04011_amd import hj

    reqs = small_requests(10)
    ref = [alone(hj, r)[0] for r in reqs]
    with hj.Server(W.scheme("eno2", "rk2"), "f32", max_inflight=max_inflight,
                   steps_per_tick=steps_per_tick, policy=policy) as srv:
        ids, shapes, results = [], {}, {}
        for i, r in enumerate(reqs):
            rid = srv.submit(r.grid, r.dyn, r.cylinders, r.horizon)
            ids.append(rid)
            shapes[rid] = tuple(r.grid["n"])
            if i % 3 == 2:  # let the running ones step before the next arrivals
                for _ in range(4):
                    srv.tick()
                for rid2 in srv.poll():
                    out = np.empty(shapes[rid2], np.float64)
                    srv.take(rid2, out)
                    results[rid2] = out
        drain(srv, ids, results, shapes)
        st = srv.stats()
        assert st["submitted"] == st["admitted"] == st["completed"] == len(reqs)
        assert st["running"] == 0 and st["queued"] == 0
        # finished requests hold their slot until taken, so slots can exceed
        # max_inflight without a budget; one slot per request at most
        assert 1 <= st["slots"] <= len(reqs)
    for rid, r in zip(ids, ref):
        assert np.array_equal(results[rid], r), rid


def test_server_budget_bounds_slots():
    """A budget of two slots of the larger shape: at most that many bytes are
    held, idle slots of the other shape are freed to fit, all results right."""
    from paper_2012_04011_amd import hj

    reqs = small_requests(8)
    ref = [alone(hj, r)[0] for r in reqs]
    n_big = max(int(np.prod(g["n"])) for g in SMALL_GRIDS)
    budget = 2 * (4 * n_big * 4 + 4 * 8 * 20 * 12 + 4 * 20 * 18 + 16 * 8 * 12) + 1
    with hj.Server(W.scheme("eno2", "rk2"), "f32", hbm_budget=budget, max_inflight=8) as srv:
        ids, shapes, results = [], {}, {}
        for r in reqs:
            rid = srv.submit(r.grid, r.dyn, r.cylinders, r.horizon)
            ids.append(rid)
            shapes[rid] = tuple(r.grid["n"])
        peak = 0
        while len(results) < len(ids):
            srv.tick()
            peak = max(peak, srv.stats()["slot_bytes"])
            for rid in srv.poll():
                out = np.empty(shapes[rid], np.float64)
                srv.take(rid, out)
                results[rid] = out
        assert peak <= budget
    for rid, r in zip(ids, ref):
        assert np.array_equal(results[rid], r), rid


def test_server_zero_horizon_and_errors():
    from paper_2012_04011_amd import hj

    req = small_requests(1)[0]
    with hj.Server(W.scheme("eno2", "rk2"), "f32", max_inflight=2) as srv:
        rid = srv.submit(req.grid, req.dyn, req.cylinders, 0.0)
        with pytest.raises(hj.HJError):
            srv.take(rid)  # not complete yet
        results = {}
        drain(srv, [rid], results, {rid: tuple(req.grid["n"])})
        ref, info = alone(hj, dataclasses.replace(req, horizon=0.0))
        assert info["steps"] == 0 and np.array_equal(results[rid], ref)
        with pytest.raises(hj.HJError):
            srv.take(rid)  # already taken
        with pytest.raises(hj.HJError):
            srv.submit(req.grid, req.dyn, req.cylinders, -1.0)
    with hj.Server(W.scheme("eno2", "rk2"), "f32", hbm_budget=1000) as srv:
        with pytest.raises(hj.HJError) as e:
            srv.submit(req.grid, req.dyn, req.cylinders, 0.3)
        assert e.value.status == hj.HJ_ERR_OUT_OF_MEMORY


def test_served_fp64_matches_oracle():
    from paper_2012_04011_amd import hj

    reqs = small_requests(3)
    with hj.Server(W.scheme("eno2", "rk2"), "f64", max_inflight=4) as srv:
        ids, shapes, results = [], {}, {}
        for r in reqs:
            rid = srv.submit(r.grid, r.dyn, r.cylinders, r.horizon)
            ids.append(rid)
            shapes[rid] = tuple(r.grid["n"])
        drain(srv, ids, results, shapes)
    for rid, r in zip(ids, reqs):
        V0 = oracle.target_cylinders(r.grid, *r.cylinders)
        ref, _ = oracle.solve(r.grid, r.dyn, W.scheme("eno2", "rk2"), V0, r.horizon)
        assert_f64_close(results[rid], ref)


def test_served_mix_of_large_and_small_equals_alone():
    """A grid above the size that steps alone (64x64x24x48, 4.7M nodes)
    served together with small batched ones, requests ending inside ticks:
    every result equals its solve alone."""
    from paper_2012_04011_amd import hj

    big = W.car_grid(64, 64, 24, 48)
    reqs = small_requests(5)
    reqs.insert(1, W.Request(0.0, 2, big, W.car_dynamics(), W.cylinders(77, 4), 0.25))
    reqs.append(W.Request(0.0, 2, big, W.car_dynamics(), W.cylinders(78, 2), 0.15))
    ref = [alone(hj, r)[0] for r in reqs]
    with hj.Server(W.scheme("eno2", "rk2"), "f32", max_inflight=8, steps_per_tick=3) as srv:
        ids, shapes, results = [], {}, {}
        for r in reqs:
            rid = srv.submit(r.grid, r.dyn, r.cylinders, r.horizon)
            ids.append(rid)
            shapes[rid] = tuple(r.grid["n"])
            srv.tick()
        drain(srv, ids, results, shapes)
    for rid, r in zip(ids, ref):
        assert np.array_equal(results[rid], r), rid


@pytest.mark.parametrize("policy,age_ms", [("small_first", 1e9), ("small_first", 1e-6), ("share", 0.0)],
                         ids=["small_first", "small_first_aged", "share"])
def test_policy_order_of_completion(policy, age_ms):
    """Two 60x60x20x36 requests with a long horizon (less work each than the
    100x100x24x48 request beside them, but more steps) and the large one,
    submitted together.  Small-first (no request reaching the age limit)
    steps the two small ones (together they fill the device) and holds the
    large one, so both small ones finish first; past the age limit (here at
    once) the order is first come, first served and the large one, submitted
    first, finishes first; sharing steps all three and the large one, with
    fewer steps, finishes first.  Every result equals its solve alone."""
    from paper_2012_04011_amd import hj

    small, large = W.SERVE_GRIDS
    reqs = [W.Request(0.0, 1, large, W.car_dynamics(), W.cylinders(80, 3), 1.5),
            W.Request(0.0, 0, small, W.car_dynamics(), W.cylinders(81, 2), 5.0),
            W.Request(0.0, 0, small, W.car_dynamics(), W.cylinders(82, 2), 5.0)]
    ref = [alone(hj, r) for r in reqs]
    work = [int(np.prod(r.grid["n"])) * info["steps"] for r, (_, info) in zip(reqs, ref)]
    assert work[1] < work[0] and work[2] < work[0] and ref[1][1]["steps"] > ref[0][1]["steps"]
    with hj.Server(W.scheme("eno2", "rk2"), "f32", max_inflight=8, steps_per_tick=4, policy=policy,
                   age_ms=age_ms) as srv:
        ids = [srv.submit(r.grid, r.dyn, r.cylinders, r.horizon) for r in reqs]
        shapes = {rid: tuple(r.grid["n"]) for rid, r in zip(ids, reqs)}
        order, results = [], {}
        for _ in range(100000):
            if len(results) == len(ids):
                break
            srv.tick()
            for rid in srv.poll():
                out = np.empty(shapes[rid], np.float64)
                srv.take(rid, out)
                results[rid] = out
                order.append(rid)
    if policy == "small_first" and age_ms > 1e3:
        assert order[-1] == ids[0], order
    else:
        assert order[0] == ids[0], order
    for rid, (V, _) in zip(ids, ref):
        assert np.array_equal(results[rid], V), rid
