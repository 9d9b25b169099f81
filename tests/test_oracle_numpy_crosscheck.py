"""Brute-force cross-check of the C oracle on tiny grids.

An independent vectorised NumPy implementation -- ghost layers padded
explicitly, ENO choices by np.where, the Hamiltonian in its separable
closed form (sum of p_d times drift plus |p_d| times the input bound) rather
than the oracle's explicit optimal controls -- must agree with the C oracle to
1e-13 on 6x5x4x8-sized grids for every scheme, dynamics and boundary kind.
This pins indexing, ghost handling and transcription, not the method itself
(the closed-form pins do that).
"""

import math

import numpy as np
import pytest

from paper_2012_04011_amd import workloads as W


def _axis_info(grid, d):
    n, lo, hi = grid["n"][d], grid["lo"][d], grid["hi"][d]
    per = bool((grid["periodic_mask"] >> d) & 1)
    h = (hi - lo) / (n if per else n - 1)
    return n, lo, h, per


def _pad(V, d, per):
    """Two ghost layers on each side of axis d."""
    if per:
        return np.concatenate([np.take(V, [-2, -1], axis=d), V, np.take(V, [0, 1], axis=d)], axis=d)
    e0, e1 = np.take(V, [0], axis=d), np.take(V, [1], axis=d)
    f0, f1 = np.take(V, [-1], axis=d), np.take(V, [-2], axis=d)
    left = [e0 + 2 * (e0 - e1), e0 + (e0 - e1)]
    right = [f0 + (f0 - f1), f0 + 2 * (f0 - f1)]
    return np.concatenate(left + [V] + right, axis=d)


def _sl(d, a, b, n):
    s = [slice(None)] * 4
    s[d] = slice(a, a + n if b is None else b)
    return tuple(s)


def np_derivs(grid, deriv, V):
    pms, pps = [], []
    for d in range(4):
        n, _, h, per = _axis_info(grid, d)
        P = _pad(V, d, per)
        w = [P[_sl(d, k, None, n)] for k in range(5)]  # V_{i-2} .. V_{i+2}
        if deriv == "upwind1":
            pm, pp = (w[2] - w[1]) / h, (w[3] - w[2]) / h
        else:
            ql = w[0] - 2 * w[1] + w[2]
            qm = w[1] - 2 * w[2] + w[3]
            qr = w[2] - 2 * w[3] + w[4]
            cm = np.where(np.abs(ql) <= np.abs(qm), ql, qm)
            cp = np.where(np.abs(qm) <= np.abs(qr), qm, qr)
            pm = (w[2] - w[1]) / h + cm / (2 * h)
            pp = (w[3] - w[2]) / h - cp / (2 * h)
        pms.append(pm)
        pps.append(pp)
    return pms, pps


def np_coords(grid):
    out = []
    for d in range(4):
        n, lo, h, _ = _axis_info(grid, d)
        shape = [1, 1, 1, 1]
        shape[d] = n
        out.append((lo + np.arange(n) * h).reshape(shape))
    return out


def np_rhs(grid, dyn, deriv, V):
    pm, pp = np_derivs(grid, deriv, V)
    pbar = [(a + b) / 2 for a, b in zip(pp, pm)]
    half = [(a - b) / 2 for a, b in zip(pp, pm)]
    x, y, v, th = np_coords(grid)
    if dyn["kind"] == "car4d":
        dx, dy = dyn["d_max"]
        cx, cy = v * np.cos(th), v * np.sin(th)
        H = (pbar[0] * cx + pbar[1] * cy + dyn["a_max"] * np.abs(pbar[2]) + dyn["w_max"] * np.abs(pbar[3])
             - dx * np.abs(pbar[0]) - dy * np.abs(pbar[1]))
        alpha = [np.abs(cx) + dx, np.abs(cy) + dy, dyn["a_max"], dyn["w_max"]]
    else:
        sgn = 1.0 if dyn["in_role"] == "max" else -1.0
        s = dyn["in_speed"]
        axes = dyn["in_axes"]
        H = sum(dyn["drift"][d] * pbar[d] for d in range(4))
        if dyn["in_norm"] == "box":
            H = H + sgn * s * sum(np.abs(pbar[d]) for d in axes)
        else:
            H = H + sgn * s * np.sqrt(sum(pbar[d] ** 2 for d in axes))
        alpha = [abs(dyn["drift"][d]) + (s if d in axes else 0.0) for d in range(4)]
    return H + sum(alpha[d] * half[d] for d in range(4))


def np_step(grid, dyn, scheme, V0, V, dt):
    L = np_rhs(grid, dyn, scheme["deriv"], V)
    if scheme["integrator"] == "euler":
        out = V + dt * L
    else:
        V1 = V + dt * L
        V2 = V1 + dt * np_rhs(grid, dyn, scheme["deriv"], V1)
        out = (V + V2) / 2
    return np.minimum(V0, out) if scheme["clamp"] else out


DYNS = [
    W.car_dynamics(),
    W.car_dynamics(a_max=1.2, w_max=0.7, d_max=0.1),
    {"kind": "drift_input", "drift": (0.3, -0.5, 0.2, 0.9), "in_axes": (0, 1), "in_speed": 0.8,
     "in_norm": "box", "in_role": "max"},
    {"kind": "drift_input", "drift": (-0.3, 0.1, 0.0, 0.4), "in_axes": (0, 1, 3), "in_speed": 0.6,
     "in_norm": "ball", "in_role": "min"},
]


@pytest.mark.parametrize("dyn", DYNS, ids=["car", "car_dist", "box_max", "ball_min"])
@pytest.mark.parametrize("deriv", ["upwind1", "eno2"])
@pytest.mark.parametrize("periodic_mask", [0b1000, 0b1010, 0b0000])
def test_rhs_agrees(oracle_lib, dyn, deriv, periodic_mask):
    g = W.car_grid(6, 5, 4, 8)
    g["periodic_mask"] = periodic_mask
    rng = np.random.default_rng(16 * ("upwind1", "eno2").index(deriv) + periodic_mask)
    V = rng.normal(size=g["n"])
    L = oracle_lib.rhs(g, dyn, W.scheme(deriv, "euler"), V)
    np.testing.assert_allclose(L, np_rhs(g, dyn, deriv, V), rtol=0, atol=1e-12)


@pytest.mark.parametrize("integrator", ["euler", "rk2"])
@pytest.mark.parametrize("deriv", ["upwind1", "eno2"])
@pytest.mark.parametrize("clamp", [True, False])
def test_steps_agree(oracle_lib, integrator, deriv, clamp):
    g = W.car_grid(7, 6, 5, 8)
    dyn = W.car_dynamics(d_max=0.1)
    sch = W.scheme(deriv, integrator, clamp=clamp)
    cx, cy, r = W.cylinders(4, 2)
    V0 = oracle_lib.target_cylinders(g, cx, cy, r)
    dt = oracle_lib.cfl_dt(g, dyn, 0.8, 1.0)
    Vo, Vn = V0.copy(), V0.copy()
    for _ in range(5):
        Vo = oracle_lib.step(g, dyn, sch, V0, Vo, dt)
        Vn = np_step(g, dyn, sch, V0, Vn, dt)
    np.testing.assert_allclose(Vo, Vn, rtol=0, atol=1e-13)
