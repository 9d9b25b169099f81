"""Seeded synthetic workloads for the BRT solver.

This module holds problem descriptions (grids, dynamics, schemes) and the
seeded obstacle draws.  It contains none of the method's arithmetic, so both
the HIP library's callers and the FP64 oracle can take their inputs from it.

Obstacles are cylinders in (x, y) extruded over (v, theta), standing in for
the paper's motion-captured cone layouts (section "Experiment setup", eq (7):
cone radius 0.08 m inflated to 0.75 m), which were never published.  Centres
are uniform in [-3, 3]^2 and radii uniform in [0.4, 1.0]; the draw order is
cx[0..m), cy[0..m), r[0..m) from ``numpy.random.default_rng(seed)``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

THETA_PERIODIC = 1 << 3  # bit d set = axis d periodic; theta is axis 3


def car_grid(nx: int, ny: int, nv: int, nth: int, xy=(-5.0, 5.0), v=(0.0, 2.0)) -> dict:
    """4D car grid: x, y in [-5, 5], v in [0, 2] (ends included), theta in
    [-pi, pi) periodic."""
    return {
        "n": (int(nx), int(ny), int(nv), int(nth)),
        "lo": (xy[0], xy[0], v[0], -math.pi),
        "hi": (xy[1], xy[1], v[1], math.pi),
        "periodic_mask": THETA_PERIODIC,
    }


def car_dynamics(a_max: float = 1.5, w_max: float = 1.0, d_max: float = 0.0) -> dict:
    """x' = v cos(theta) + d_x, y' = v sin(theta) + d_y, v' = a, theta' = w;
    |a| <= a_max, |w| <= w_max (control, maximises); |d_x|, |d_y| <= d_max
    (disturbance, minimises)."""
    return {"kind": "car4d", "a_max": a_max, "w_max": w_max, "d_max": (d_max, d_max)}


def steer_dynamics(a_max: float = 1.5, steer_max: float = math.pi / 18, wheelbase: float = 0.3,
                   d_max: float = 0.0) -> dict:
    """The experiment's car (section "Experiment setup", eq (6)):
    x' = v cos(theta) + d_x, y' = v sin(theta) + d_y, v' = a,
    theta' = v tan(delta) / L; |a| <= a_max, |delta| <= steer_max (control,
    maximises); the paper's values a in [-1.5, 1.5], delta in
    [-pi/18, pi/18], L = 0.3 m."""
    return {"kind": "car4d_steer", "a_max": a_max, "steer_max": steer_max, "wheelbase": wheelbase,
            "d_max": (d_max, d_max)}


def scheme(deriv: str, integrator: str, cfl: float = 0.8, clamp: bool = True, alpha: str = "state") -> dict:
    """alpha: "state" (the bound on |f_d| over all inputs), "deriv_range"
    (Algorithm 1's global Lax-Friedrichs over the range of the central
    derivative of eq (5) on the grid) or "deriv_range_onesided" (over the
    range of both one-sided derivatives)."""
    return {"deriv": deriv, "integrator": integrator, "clamp": clamp, "cfl": cfl, "alpha": alpha}


def cylinders(seed: int, m: int):
    """Seeded obstacle set: (cx, cy, r) float64 arrays of length m."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(-3.0, 3.0, size=m)
    cy = rng.uniform(-3.0, 3.0, size=m)
    r = rng.uniform(0.4, 1.0, size=m)
    return cx, cy, r


@dataclass
class Workload:
    name: str
    grid: dict
    dyn: dict
    scheme: dict
    horizon: float
    obstacles: int
    seeds: tuple
    precision: str = "f32"
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def points(self) -> int:
        n = self.grid["n"]
        return int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])


# Plain method, FP64, first order upwind + Euler, 3 cylinders, T = 1 s.
PLAIN_40 = Workload(
    name="car4d 40x40x20x24 upwind1+euler f64 T=1",
    grid=car_grid(40, 40, 20, 24),
    dyn=car_dynamics(),
    scheme=scheme("upwind1", "euler"),
    horizon=1.0,
    obstacles=3,
    seeds=(0, 1, 2),
    precision="f64",
)

# The paper's grid size, ENO2 + TVD-RK2, disturbance |d| <= 0.1, 5 cylinders, T = 2 s.
ENO_60_DIST = Workload(
    name="car4d 60x60x20x36 eno2+rk2 d=0.1 f32 T=2",
    grid=car_grid(60, 60, 20, 36),
    dyn=car_dynamics(d_max=0.1),
    scheme=scheme("eno2", "rk2"),
    horizon=2.0,
    obstacles=5,
    seeds=(0, 1, 2),
    precision="f32",
)

# Large single grid, 41.5M points, ENO2 + TVD-RK2, 8 cylinders, T = 2 s.
LARGE_120 = Workload(
    name="car4d 120x120x40x72 eno2+rk2 f32 T=2",
    grid=car_grid(120, 120, 40, 72),
    dyn=car_dynamics(),
    scheme=scheme("eno2", "rk2"),
    horizon=2.0,
    obstacles=8,
    seeds=(0,),
    precision="f32",
)

# The large grid coarsened 2x (the oracle's companion of LARGE_120).
LARGE_120_COARSE = Workload(
    name="car4d 60x60x20x36 eno2+rk2 f64 T=2 (2x-coarsened large grid)",
    grid=car_grid(60, 60, 20, 36),
    dyn=car_dynamics(),
    scheme=scheme("eno2", "rk2"),
    horizon=2.0,
    obstacles=8,
    seeds=(0,),
    precision="f64",
)

WORKLOADS = {w.name: w for w in (PLAIN_40, ENO_60_DIST, LARGE_120, LARGE_120_COARSE)}


@dataclass
class Instance:
    """One problem of a batch: grid, dynamics, scheme, obstacle set, horizon."""
    grid: dict
    dyn: dict
    scheme: dict
    cylinders: tuple
    horizon: float

    @property
    def points(self) -> int:
        n = self.grid["n"]
        return int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])


def batch_instances(count: int = 64, seed0: int = 1000, sizes=((30, 80), (30, 80), (12, 24), (18, 48)),
                    obstacles=(1, 8), horizon=(0.5, 2.0)) -> list:
    """Uneven batch: instance i draws, from default_rng(seed0 + i) in this
    order, its axis sizes (independent uniform integers in `sizes`, ends
    included), its obstacle count (uniform in `obstacles`) and its horizon
    (uniform in `horizon`); its cylinders are cylinders(seed0 + i, m) for that count m.
    4D car without disturbance, ENO2 + TVD-RK2."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = [int(rng.integers(lo, hi + 1)) for lo, hi in sizes]
        m = int(rng.integers(obstacles[0], obstacles[1] + 1))
        T = float(rng.uniform(*horizon))
        out.append(Instance(car_grid(*n), car_dynamics(), scheme("eno2", "rk2"), cylinders(seed0 + i, m), T))
    return out


# 64 uneven instances, 30x30x12x18 .. 80x80x24x48, 1-8 cylinders,
# horizons in [0.5, 2] s, FP32 ENO2 + TVD-RK2 (the batched workload).
BATCH_64 = dict(count=64, seed0=1000)


@dataclass
class Request:
    """A re-solve request of a served stream."""
    arrival: float   # seconds after the stream starts
    cls: int         # grid class
    grid: dict
    dyn: dict
    cylinders: tuple
    horizon: float


# Served mix: the paper's grid 60x60x20x36 and a finer 100x100x24x48.
SERVE_GRIDS = (car_grid(60, 60, 20, 36), car_grid(100, 100, 24, 48))


def serving_requests(count: int, rate: float = 20.0, seed: int = 7, mix: float = 0.7, horizon: float = 1.5,
                     grids=SERVE_GRIDS, cap: int = 8) -> list:
    """Poisson arrivals (exponential gaps at `rate` per second from
    default_rng(seed)); each request picks grid class 0 with probability
    `mix` (same stream), then, from default_rng(7000 + i), changes that
    class's obstacle map (which starts as cylinders(70 + class, 3)) 1-3
    times: add a cylinder (centre U[-3, 3]^2, radius U[0.4, 1.0]) when fewer
    than `cap` and a fair coin says so, else move a random one by
    U[-0.5, 0.5]^2 (clipped to [-3, 3]).  The request carries a copy of the
    map."""
    rng = np.random.default_rng(seed)
    scenes = {}
    for c in range(len(grids)):
        cx, cy, r = cylinders(70 + c, 3)
        scenes[c] = [(float(a), float(b), float(d)) for a, b, d in zip(cx, cy, r)]
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        c = 0 if rng.uniform() < mix else 1
        r2 = np.random.default_rng(7000 + i)
        scene = scenes[c]
        for _ in range(int(r2.integers(1, 4))):
            if len(scene) < cap and r2.uniform() < 0.5:
                scene.append((float(r2.uniform(-3, 3)), float(r2.uniform(-3, 3)), float(r2.uniform(0.4, 1.0))))
            else:
                j = int(r2.integers(0, len(scene)))
                x, y, rad = scene[j]
                scene[j] = (float(np.clip(x + r2.uniform(-0.5, 0.5), -3, 3)),
                            float(np.clip(y + r2.uniform(-0.5, 0.5), -3, 3)), rad)
        cyl = tuple(np.array(v, dtype=np.float64) for v in zip(*scene))
        out.append(Request(t, c, grids[c], car_dynamics(), cyl, horizon))
    return out
