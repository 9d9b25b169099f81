"""Accuracy figures of a computed value function against a reference one.

V is a distance-like function in metres (the target of eq (7)), and the BRT
is {V <= 0} (section "Hamilton-Jacobi Reachability Analysis"), so an FP32
result is judged by:
  - the largest |dV| over the band |V_ref| <= 1 around the zero level set and
    over all nodes, and the RMS over all nodes, against tol = 1e-4 of the
    in-plane grid spacing min(dx, dy);
  - BRT-membership disagreements (V <= 0 on one side only), in total and
    farther than tol from the reference's zero level set.
Two solutions of different resolution are compared at the coarse nodes by
multilinear interpolation of the fine one (the coarse grid's nodes need not
be fine nodes on the open axes).  The paper measures its fixed-point FPGA the
same way, as the largest difference from a reference solver (section
"Hardware Correctness", Table I).

Plain NumPy; nothing here takes part in computing V.
"""

from __future__ import annotations

import math

import numpy as np


def h_pos(grid) -> float:
    """min(dx, dy) of a grid description (open x and y axes, ends included)."""
    return min((grid["hi"][d] - grid["lo"][d]) / (grid["n"][d] - 1) for d in (0, 1))


def precision_metrics(V, ref, grid, band: float = 1.0) -> dict:
    """Errors of V against ref (any float arrays of one shape), with
    tol = 1e-4 h_pos(grid): band / all-node max, RMS, band percentiles, the
    share of band nodes beyond tol, and membership flips (total, where
    |ref| > tol, and the largest |ref| of a flipped node: its distance from
    the reference's zero level set)."""
    tol = 1e-4 * h_pos(grid)
    V = np.asarray(V, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(V - ref)
    inb = np.abs(ref) <= band
    eb = err[inb] if inb.any() else np.zeros(1)
    flips = (V <= 0) != (ref <= 0)
    return {
        "tol": tol,
        "max_band": float(eb.max()),
        "max_all": float(err.max()),
        "rms": float(math.sqrt(float(np.mean(err * err)))),
        "p50_band": float(np.percentile(eb, 50)),
        "p99_band": float(np.percentile(eb, 99)),
        "frac_band_gt_tol": float((eb > tol).mean()),
        "flips": int(flips.sum()),
        "flips_outside": int((flips & (np.abs(ref) > tol)).sum()),
        "flip_max_abs_ref": float(np.abs(ref[flips]).max()) if flips.any() else 0.0,
    }


def _nodes(grid, d: int) -> np.ndarray:
    n, lo, hi = int(grid["n"][d]), float(grid["lo"][d]), float(grid["hi"][d])
    if (int(grid["periodic_mask"]) >> d) & 1:
        return lo + np.arange(n) * ((hi - lo) / n)
    return lo + np.arange(n) * ((hi - lo) / (n - 1))


def sample_multilinear(V, grid, at_grid) -> np.ndarray:
    """V on `grid`, interpolated multilinearly at the nodes of `at_grid`
    (same axis ranges), one axis at a time: on an open axis between the two
    nodes around the point (the last cell for the upper end), on a periodic
    axis between node floor(t) and the next one modulo n."""
    A = np.asarray(V, dtype=np.float64)
    for d in range(4):
        n = int(grid["n"][d])
        lo, hi = float(grid["lo"][d]), float(grid["hi"][d])
        per = (int(grid["periodic_mask"]) >> d) & 1
        h = (hi - lo) / (n if per else n - 1)
        t = (_nodes(at_grid, d) - lo) / h
        if per:
            t = np.mod(t, n)
            i0 = np.minimum(np.floor(t).astype(np.int64), n - 1)
            i1 = (i0 + 1) % n
        else:
            i0 = np.clip(np.floor(t).astype(np.int64), 0, n - 2)
            i1 = i0 + 1
        w = t - i0
        shape = [1, 1, 1, 1]
        shape[d] = len(w)
        w = w.reshape(shape)
        A = np.take(A, i0, axis=d) * (1.0 - w) + np.take(A, i1, axis=d) * w
    return A


def consistency_metrics(V_fine, fine_grid, V_coarse, coarse_grid, band: float = 1.0) -> dict:
    """A fine solution sampled at the coarse nodes against a coarse one:
    max |dV| over the coarse band and all nodes, RMS, and membership flips
    in total and where |V_coarse| > 2 dx_coarse (the coarse solution's own
    resolution)."""
    S = sample_multilinear(V_fine, fine_grid, coarse_grid)
    Vc = np.asarray(V_coarse, dtype=np.float64)
    err = np.abs(S - Vc)
    dxc = h_pos(coarse_grid)
    inb = np.abs(Vc) <= band
    flips = (S <= 0) != (Vc <= 0)
    return {
        "dx_coarse": dxc,
        "max_band": float(err[inb].max()) if inb.any() else 0.0,
        "max_all": float(err.max()),
        "rms": float(math.sqrt(float(np.mean(err * err)))),
        "flips": int(flips.sum()),
        "flips_beyond_2dx": int((flips & (np.abs(Vc) > 2 * dxc)).sum()),
    }
