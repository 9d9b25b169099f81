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
    """Accuracy of an FP32 result against an FP64 reference.

    tol = 1e-4 * h_pos.  Reported: max |dV| over the band |V_ref| <= 1 and
    over all nodes, the RMS over all nodes, band percentiles, the fraction of
    band nodes beyond tol, and BRT-membership ({V <= 0}) disagreements in
    total and farther than tol from the zero level set."""
    tol = 1e-4 * h_pos(grid)
    err = np.abs(V.astype(np.float64) - ref)
    band = np.abs(ref) <= 1.0
    eb = err[band] if band.any() else np.zeros(1)
    flips = (V <= 0) != (ref <= 0)
    return {
        "tol": tol,
        "max_band": float(eb.max()),
        "max_all": float(err.max()),
        "rms": float(math.sqrt(np.mean(err ** 2))),
        "p50_band": float(np.percentile(eb, 50)),
        "p99_band": float(np.percentile(eb, 99)),
        "frac_band_gt_tol": float((eb > tol).mean()),
        "flips": int(flips.sum()),
        "flips_outside": int((flips & (np.abs(ref) > tol)).sum()),
    }


def assert_f32_close(V, ref, grid, deriv="upwind1"):
    """FP32 solve vs FP64 reference.

    Both schemes: no BRT-membership disagreement farther than tol from the
    zero level set, and the median band error at rounding level (1e-6).
    First-order upwind (no discrete choice in the update): max band error
    and RMS <= tol.  ENO2: the stencil choice compares two second
    differences, and FP32 takes it differently from FP64 near ties; a
    divergent choice moves V by up to CFL * |Q| at that node (an O(h^2 V'')
    change, the size of the scheme's own truncation error), which then
    propagates.  The bar is the bulk: >= 97% of band nodes within tol."""
    m = f32_metrics(V, ref, grid)
    assert m["flips_outside"] == 0, m
    assert m["p50_band"] <= 1e-6, m
    if deriv == "upwind1":
        assert m["max_band"] <= m["tol"], m
        assert m["rms"] <= m["tol"], m
    else:
        assert m["frac_band_gt_tol"] <= 0.03, m
    return m


def assert_f64_close(V, ref, sensitivity: float = 0.0):
    """FP64 solve vs the FP64 oracle.  The two compute the same scheme with
    different rounding order, so they differ by rounding noise as amplified
    by the scheme over the solve.  Bar: max |dV| <= max(1e-10, 10 S), where S
    is the oracle's own sensitivity to that noise (see
    oracle_rounding_sensitivity; 0 for short solves)."""
    err = float(np.abs(V - ref).max())
    tol = max(1e-10, 10.0 * sensitivity)
    assert err <= tol, (err, tol)
    return err


@functools.lru_cache(maxsize=None)
def oracle_rounding_sensitivity(name: str, seed: int) -> float:
    """How far the oracle's own solve moves when every step's result is
    perturbed by one unit roundoff (relative, random sign per node): the
    amplification of rounding noise by the scheme itself over the whole
    horizon (ENO2 choices and the extrapolated boundaries amplify it)."""
    import oracle

    wl = W.WORKLOADS[name]
    V0, ref, info = oracle_solution(name, seed)
    rng = np.random.default_rng(12345 + seed)
    V = V0.copy()
    n, dt, last = info["steps"], info["dt"], info["dt_last"]
    for k in range(n):
        V = oracle.step(wl.grid, wl.dyn, wl.scheme, V0, V, dt if k + 1 < n else last)
        V *= 1.0 + U64 * rng.choice((-1.0, 1.0), size=V.shape)
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
