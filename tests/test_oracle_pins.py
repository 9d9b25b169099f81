"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a number the paper prints, a
closed-form solution of the PDE, a polynomial-exactness property of the
difference formulas, a brute-force max/min over the input sets, or a symmetry
of the car dynamics.  All run on the CPU.
"""

import math
import os

import numpy as np
import pytest

from paper_2012_04011_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

UP_EU = W.scheme("upwind1", "euler")
ENO_RK = W.scheme("eno2", "rk2")
ALL_SCHEMES = [W.scheme(d, i) for d in ("upwind1", "eno2") for i in ("euler", "rk2")]


def small_grid(nx=12, ny=11, nv=6, nth=8, periodic_mask=W.THETA_PERIODIC):
    g = W.car_grid(nx, ny, nv, nth)
    g["periodic_mask"] = periodic_mask
    return g


def drift_dyn(drift=(0, 0, 0, 0), axes=(), speed=0.0, norm="box", role="max"):
    return {"kind": "drift_input", "drift": tuple(float(x) for x in drift), "in_axes": tuple(axes),
            "in_speed": float(speed), "in_norm": norm, "in_role": role}


# --------------------------------------------------------------- schedule ---


def test_schedule_matches_paper_table2(oracle_lib):
    """Table II: horizon 0.5 s at dt = 0.007497 s takes 67 iterations."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_schedule.txt")) if l.strip() and l[0] != "#"]
    for dt, T, iters in rows:
        n, last = oracle_lib.schedule(float(dt), float(T))
        assert n == int(iters)
        assert 0.0 < last <= float(dt)
        # n - 1 full steps fall short of the horizon, n full steps do not
        assert (n - 1) * float(dt) < float(T) <= n * float(dt)


def test_schedule_edge_cases(oracle_lib):
    assert oracle_lib.schedule(0.1, 0.0) == (0, 0.0)
    n, last = oracle_lib.schedule(0.25, 1.0)  # exact multiple: 4 full steps
    assert n == 4 and last == 0.25
    n, last = oracle_lib.schedule(2.0, 1.0)  # horizon shorter than one step
    assert n == 1 and last == 1.0


@pytest.mark.parametrize("wl", [W.PLAIN_40, W.ENO_60_DIST, W.LARGE_120])
def test_cfl_step_closed_form(oracle_lib, wl):
    """alpha^max over the nodes of the car grids in closed form: theta = -pi
    and theta = -pi/2 are nodes (N_theta divisible by 4), and the top speed
    node is v = 2, so alpha_x^max = alpha_y^max = 2 + d_max, alpha_v = 1.5,
    alpha_theta = 1; spacings are 10/(N-1), 2/(N-1), 2 pi / N."""
    n = wl.grid["n"]
    d = wl.dyn["d_max"][0]
    s = (2 + d) / (10 / (n[0] - 1)) + (2 + d) / (10 / (n[1] - 1)) + 1.5 / (2 / (n[2] - 1)) + 1.0 / (2 * math.pi / n[3])
    dt = oracle_lib.cfl_dt(wl.grid, wl.dyn, 0.8, wl.horizon)
    assert dt == pytest.approx(0.8 / s, rel=1e-14)
    steps, _ = oracle_lib.schedule(dt, wl.horizon)
    assert steps == math.ceil(wl.horizon * s / 0.8)


def test_cfl_uses_nodes_not_supremum(oracle_lib):
    """With 18 theta nodes (20 degree spacing) no node sits at +-90 degrees:
    alpha_y^max = 2 sin(80 deg), not 2."""
    g = W.car_grid(30, 30, 12, 18)
    amax = oracle_lib.alpha_max(g, W.car_dynamics())
    assert amax[1] == pytest.approx(2 * math.sin(math.radians(80)), rel=1e-14)
    assert amax[0] == pytest.approx(2.0, rel=1e-15)


def test_zero_motion_takes_one_step(oracle_lib):
    g = small_grid()
    assert oracle_lib.cfl_dt(g, drift_dyn(), 0.8, 1.7) == 1.7


# ------------------------------------------------------------ derivatives ---


def _line(grid, axis):
    """Node coordinates broadcast along `axis` (independent of the oracle's
    own node helper: lo + i * spacing from the grid description)."""
    n, lo, hi = grid["n"][axis], grid["lo"][axis], grid["hi"][axis]
    per = (grid["periodic_mask"] >> axis) & 1
    h = (hi - lo) / (n if per else n - 1)
    x = lo + np.arange(n) * h
    shape = [1, 1, 1, 1]
    shape[axis] = n
    return x.reshape(shape), h


@pytest.mark.parametrize("deriv", ["upwind1", "eno2"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_derivative_exact_on_linear(oracle_lib, deriv, axis):
    """A linear function has exact one-sided differences, and linear
    extrapolation reproduces it beyond the ends: p- = p+ = slope everywhere."""
    g = small_grid()
    x, _ = _line(g, axis)
    V = np.broadcast_to(0.7 - 1.3 * x, g["n"]).copy()
    pm, pp = oracle_lib.derivs(g, W.scheme(deriv, "euler"), V, axis)
    np.testing.assert_allclose(pm, -1.3, rtol=0, atol=1e-12)
    np.testing.assert_allclose(pp, -1.3, rtol=0, atol=1e-12)


def test_eno2_exact_on_quadratic_interior(oracle_lib):
    """Second-order one-sided differences are exact for quadratics; first
    order ones are off by exactly -h and +h."""
    g = small_grid(nx=14)
    x, h = _line(g, 0)
    V = np.broadcast_to((x - 0.3) ** 2, g["n"]).copy()
    exact = np.broadcast_to(2 * (x - 0.3), g["n"])
    pm, pp = oracle_lib.derivs(g, W.scheme("eno2", "euler"), V, 0)
    inner = slice(2, -2)
    np.testing.assert_allclose(pm[inner], exact[inner], atol=1e-12)
    np.testing.assert_allclose(pp[inner], exact[inner], atol=1e-12)
    pm1, pp1 = oracle_lib.derivs(g, W.scheme("upwind1", "euler"), V, 0)
    np.testing.assert_allclose(pm1[inner], exact[inner] - h, atol=1e-12)
    np.testing.assert_allclose(pp1[inner], exact[inner] + h, atol=1e-12)


def test_eno2_avoids_kink(oracle_lib):
    """V = |x - k| with the kink between two nodes: every one-sided
    derivative whose own two-point difference stays on one side of the kink
    is the exact slope (+-1): the ENO choice takes the second difference that
    does not straddle the kink."""
    g = small_grid(nx=20)
    x, h = _line(g, 0)
    k = x.ravel()[9] + 0.37 * h
    V = np.broadcast_to(np.abs(x - k), g["n"]).copy()
    pm, pp = oracle_lib.derivs(g, W.scheme("eno2", "euler"), V, 0)
    xs = x.ravel()
    for i in range(2, 18):
        if xs[i - 1] > k or xs[i] < k:  # left difference does not straddle
            assert pm[i, 0, 0, 0] == pytest.approx(np.sign(xs[i] - k), abs=1e-12)
        if xs[i] > k or xs[i + 1] < k:
            assert pp[i, 0, 0, 0] == pytest.approx(np.sign(xs[i] - k), abs=1e-12)


@pytest.mark.parametrize("sizes", [(9, 7, 6), (3, 3, 3)], ids=["mid", "three_nodes"])
@pytest.mark.parametrize("deriv", ["upwind1", "eno2"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_edge_nodes_take_plain_first_differences(oracle_lib, deriv, axis, sizes):
    """Next to the ends of an open axis the linearly extrapolated ghosts make
    every outer first difference equal to the last inner one and the outer
    second differences vanish, so the ENO correction on the ghost side is
    zero: at i = 0 both one-sided differences are V_1 - V_0, at i = 1 the
    left one is, at n - 2 the right one is V_{n-1} - V_{n-2}, at n - 1 both
    are.  Checked on random data (up to rounding of the ghost values)."""
    g = small_grid(nx=sizes[0], ny=sizes[1], nv=sizes[2])
    rng = np.random.default_rng(11 + axis)
    V = rng.standard_normal(g["n"])
    _, h = _line(g, axis)
    pm, pp = oracle_lib.derivs(g, W.scheme(deriv, "euler"), V, axis)
    n = g["n"][axis]
    take = lambda A, i: np.take(A, i, axis=axis)  # noqa: E731
    lo = (take(V, 1) - take(V, 0)) / h
    hi = (take(V, n - 1) - take(V, n - 2)) / h
    tol = dict(rtol=0, atol=1e-12)
    np.testing.assert_allclose(take(pm, 0), lo, **tol)
    np.testing.assert_allclose(take(pp, 0), lo, **tol)
    np.testing.assert_allclose(take(pm, 1), lo, **tol)
    np.testing.assert_allclose(take(pp, n - 2), hi, **tol)
    np.testing.assert_allclose(take(pm, n - 1), hi, **tol)
    np.testing.assert_allclose(take(pp, n - 1), hi, **tol)
    if deriv == "eno2" and n > 3:
        # the other side of nodes 1 and n - 2 still takes its ENO correction
        assert np.abs(take(pp, 1) - (take(V, 2) - take(V, 1)) / h).max() > 1e-3
        assert np.abs(take(pm, n - 2) - (take(V, n - 2) - take(V, n - 3)) / h).max() > 1e-3


@pytest.mark.parametrize("deriv,order", [("upwind1", 1), ("eno2", 2)])
def test_periodic_axis_convergence(oracle_lib, deriv, order):
    """On the periodic theta axis, d/dtheta sin(theta) = cos(theta): the
    error over all nodes (including the wrapped ends) falls as h^order."""
    errs = []
    for nth in (32, 64):
        g = small_grid(nx=4, ny=4, nv=4, nth=nth)
        th, _ = _line(g, 3)
        V = np.broadcast_to(np.sin(th), g["n"]).copy()
        pm, pp = oracle_lib.derivs(g, W.scheme(deriv, "euler"), V, 3)
        ex = np.broadcast_to(np.cos(th), g["n"])
        errs.append(max(np.abs(pm - ex).max(), np.abs(pp - ex).max()))
    ratio = errs[0] / errs[1]
    assert ratio > 2 ** order * 0.8, (errs, ratio)


# ----------------------------------------------------- Hamiltonian / alpha ---


def _car_f(z, a, w, dx, dy):
    return np.stack(np.broadcast_arrays(z[2] * np.cos(z[3]) + dx, z[2] * np.sin(z[3]) + dy, a, w), axis=-1)


def test_car_hamiltonian_brute_force(oracle_lib):
    """H = max over controls of min over disturbances of p.f, by exhaustive
    search over a grid of each input box (box vertices included, so the
    search is exact for this input-affine f)."""
    rng = np.random.default_rng(11)
    dyn = W.car_dynamics(a_max=1.5, w_max=1.0, d_max=0.1)
    s = np.linspace(-1, 1, 9)
    A, Wc, DX, DY = np.meshgrid(1.5 * s, 1.0 * s, 0.1 * s, 0.1 * s, indexing="ij")
    for _ in range(40):
        z = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(0, 2), rng.uniform(-math.pi, math.pi)])
        p = rng.normal(size=4)
        if rng.random() < 0.2:
            p[rng.integers(4)] = 0.0
        val = (_car_f(z, A, Wc, DX, DY) @ p)  # shape (a, w, dx, dy)
        bf = val.min(axis=(2, 3)).max()
        assert oracle_lib.hamiltonian(dyn, z, p) == pytest.approx(bf, abs=1e-12)


def test_car_alpha_brute_force(oracle_lib):
    """alpha_d(z) = max over all inputs of |f_d(z, u, d)|."""
    rng = np.random.default_rng(12)
    dyn = W.car_dynamics(a_max=1.5, w_max=1.0, d_max=0.1)
    s = np.linspace(-1, 1, 9)
    A, Wc, DX, DY = np.meshgrid(1.5 * s, 1.0 * s, 0.1 * s, 0.1 * s, indexing="ij")
    for _ in range(20):
        z = np.array([0.0, 0.0, rng.uniform(0, 2), rng.uniform(-math.pi, math.pi)])
        f = _car_f(z, A, Wc, DX, DY)
        bf = np.abs(f).reshape(-1, 4).max(axis=0)
        np.testing.assert_allclose(oracle_lib.alpha(dyn, z), bf, atol=1e-13)


@pytest.mark.parametrize("role", ["max", "min"])
@pytest.mark.parametrize("norm", ["box", "ball"])
def test_drift_input_hamiltonian_brute_force(oracle_lib, role, norm):
    """z' = drift + u on axes (0, 2), |u| <= 0.7 in the box or ball norm; the
    input maximises (role max) or minimises (role min) p.f."""
    rng = np.random.default_rng(13)
    dyn = drift_dyn(drift=(0.3, -0.2, 0.1, 0.5), axes=(0, 2), speed=0.7, norm=norm, role=role)
    if norm == "box":
        s = np.linspace(-0.7, 0.7, 15)
        U0, U2 = np.meshgrid(s, s, indexing="ij")
    else:
        ang = np.linspace(0, 2 * math.pi, 20001)
        U0, U2 = 0.7 * np.cos(ang), 0.7 * np.sin(ang)
    for _ in range(30):
        p = rng.normal(size=4)
        vals = p[0] * (0.3 + U0) + p[1] * -0.2 + p[2] * (0.1 + U2) + p[3] * 0.5
        bf = vals.max() if role == "max" else vals.min()
        got = oracle_lib.hamiltonian(dyn, np.zeros(4), p)
        assert got == pytest.approx(bf, abs=1e-7 if norm == "ball" else 1e-12)
    a = oracle_lib.alpha(dyn, np.zeros(4))
    np.testing.assert_allclose(a, [1.0, 0.2, 0.8, 0.5], atol=1e-15)


def test_rhs_on_linear_is_hamiltonian(oracle_lib):
    """For linear V, p+ = p- = grad V at every node, the dissipation vanishes
    and L(V) = H(z, grad V): the car's H written out at the theta nodes with
    exactly known cos/sin (theta = -pi, -pi/2, 0, pi/2)."""
    g = small_grid(nx=7, ny=7, nv=5, nth=4)
    dyn = W.car_dynamics(a_max=1.5, w_max=1.0, d_max=0.1)
    x, _ = _line(g, 0)
    y, _ = _line(g, 1)
    v, _ = _line(g, 2)
    px, py, pv = 0.4, -0.9, 0.25
    V = np.broadcast_to(px * x + py * y + pv * v, g["n"]).copy()
    for deriv in ("upwind1", "eno2"):
        L = oracle_lib.rhs(g, dyn, W.scheme(deriv, "euler"), V)
        vs = v.ravel()
        cos_t = np.array([-1.0, 0.0, 1.0, 0.0])
        sin_t = np.array([0.0, -1.0, 0.0, 1.0])
        # control maximises: a = +1.5 since pv > 0, w term zero (p_theta = 0);
        # disturbance minimises: d_x = -0.1 (px > 0), d_y = +0.1 (py < 0)
        exp = (px * (vs[:, None] * cos_t[None, :] - 0.1) + py * (vs[:, None] * sin_t[None, :] + 0.1) + pv * 1.5)
        np.testing.assert_allclose(L, np.broadcast_to(exp, g["n"]), atol=1e-12)


# ------------------------------------------------------------ closed forms ---


@pytest.mark.parametrize("sch", ALL_SCHEMES)
@pytest.mark.parametrize("clamp", [True, False])
def test_p1_zero_dynamics_is_identity(oracle_lib, sch, clamp):
    """No motion: one step of the whole horizon with H = 0 and zero
    dissipation leaves V0 unchanged bit for bit."""
    g = small_grid()
    rng = np.random.default_rng(1)
    V0 = rng.normal(size=g["n"])
    sch = dict(sch, clamp=clamp)
    V, info = oracle_lib.solve(g, drift_dyn(), sch, V0, 0.9)
    assert info["steps"] == 1 and info["dt"] == 0.9
    assert np.array_equal(V, V0)


@pytest.mark.parametrize("sch", ALL_SCHEMES)
def test_p2_affine_translation(oracle_lib, sch):
    """Car with a = w = d = 0 and V0 = ax + by + c (clamp off): the level sets
    translate rigidly, V_T = V0 + T v (a cos(theta) + b sin(theta)) at every
    node including the ends (linear ghosts are exact, RK2 is exact because
    L(V) stays constant in time)."""
    g = small_grid(nx=10, ny=9, nv=5, nth=12)
    dyn = W.car_dynamics(a_max=0.0, w_max=0.0, d_max=0.0)
    x, _ = _line(g, 0)
    y, _ = _line(g, 1)
    v, _ = _line(g, 2)
    th, _ = _line(g, 3)
    a, b, c = 0.35, -0.6, 1.2
    V0 = np.broadcast_to(a * x + b * y + c, g["n"]).copy()
    T = 0.77
    V, info = oracle_lib.solve(g, dyn, dict(sch, clamp=False), V0, T)
    exact = V0 + T * v * (a * np.cos(th) + b * np.sin(th))
    assert info["steps"] > 3
    ulp = np.spacing(np.abs(exact).max())
    assert np.abs(V - exact).max() <= 8 * info["steps"] * ulp


@pytest.mark.parametrize("c", [0.8, -1.3])
def test_p3_courant_one_shift_periodic(oracle_lib, c):
    """Pure drift c along periodic theta, first order upwind, Euler, CFL 1:
    each step copies the upwind neighbour, V^n = roll(V0, -n sign(c)).  The
    paper's printed dissipation sign would instead give 2 V_i - V_(i-1) and
    blow up."""
    g = small_grid(nx=3, ny=3, nv=3, nth=16)
    dyn = drift_dyn(drift=(0, 0, 0, c))
    sch = W.scheme("upwind1", "euler", cfl=1.0, clamp=False)
    rng = np.random.default_rng(2)
    V0 = rng.uniform(-1, 1, size=g["n"])
    dt = oracle_lib.cfl_dt(g, dyn, 1.0, 10.0)
    assert dt == pytest.approx(abs((2 * math.pi / 16) / c), rel=1e-15)
    V = V0.copy()
    n = 21
    for _ in range(n):
        V = oracle_lib.step(g, dyn, sch, V0, V, dt)
    exp = np.roll(V0, -n if c > 0 else n, axis=3)
    assert np.abs(V - exp).max() <= 2 * n * np.spacing(1.0)


def test_p3_courant_one_shift_open_axis(oracle_lib):
    """The same shift along the open x axis: information enters from the
    right end only, so nodes more than n from it are exact shifts."""
    g = small_grid(nx=30, ny=3, nv=3, nth=4)
    c = 1.7
    dyn = drift_dyn(drift=(c, 0, 0, 0))
    sch = W.scheme("upwind1", "euler", cfl=1.0, clamp=False)
    V0 = np.random.default_rng(3).uniform(-1, 1, size=g["n"])
    dt = oracle_lib.cfl_dt(g, dyn, 1.0, 10.0)
    V = V0.copy()
    n = 9
    for _ in range(n):
        V = oracle_lib.step(g, dyn, sch, V0, V, dt)
    m = 30 - 1 - n
    assert np.abs(V[:m] - V0[n:n + m]).max() <= 2 * n * np.spacing(1.0)


def _disk_problem(N, role, r=1.0):
    g = W.car_grid(N, N, 3, 4, xy=(-4.0, 4.0))
    dyn = drift_dyn(axes=(0, 1), speed=1.0, norm="ball", role=role)
    return g, dyn


@pytest.mark.parametrize("sch", [UP_EU, ENO_RK])
def test_p4_disk_grows_at_unit_speed(oracle_lib, sch):
    """z' = u on (x, y), |u| <= 1, the input minimising (adversarial): the
    exact value is max(|z| - t, 0) - r, a disk whose radius grows to r + t.
    First-order scheme: the error in a band around the zero level set halves
    with h; ENO2 + RK2 is at least as accurate."""
    errs = []
    for N in (41, 81):
        g, dyn = _disk_problem(N, "min")
        V0 = oracle_lib.target_cylinders(g, [0.0], [0.0], [1.0])
        V, _ = oracle_lib.solve(g, dyn, sch, V0, 1.0)
        x, _ = _line(g, 0)
        y, _ = _line(g, 1)
        rad = np.broadcast_to(np.sqrt(x ** 2 + y ** 2), g["n"])
        exact = np.maximum(rad - 1.0, 0.0) - 1.0
        band = (rad > 1.5) & (rad < 3.0)
        errs.append(np.abs(V - exact)[band].max())
    h = 8.0 / 40
    assert errs[0] < 1.5 * h
    assert errs[0] / errs[1] > 1.6, errs
    if sch is ENO_RK:
        assert errs[1] < 0.05


def test_p4_disk_eno_beats_upwind(oracle_lib):
    g, dyn = _disk_problem(61, "min")
    V0 = oracle_lib.target_cylinders(g, [0.0], [0.0], [1.0])
    x, _ = _line(g, 0)
    y, _ = _line(g, 1)
    rad = np.broadcast_to(np.sqrt(x ** 2 + y ** 2), g["n"])
    exact = np.maximum(rad - 1.0, 0.0) - 1.0
    band = (rad > 1.5) & (rad < 3.0)
    e1 = np.abs(oracle_lib.solve(g, dyn, UP_EU, V0, 1.0)[0] - exact)[band].max()
    e2 = np.abs(oracle_lib.solve(g, dyn, ENO_RK, V0, 1.0)[0] - exact)[band].max()
    assert e2 < e1


@pytest.mark.parametrize("sch", ALL_SCHEMES)
def test_p4_disk_stays_when_input_maximises(oracle_lib, sch):
    """With the input maximising (escaping), the tube is the disk itself:
    V0 is convex, L(V) >= 0 everywhere and the clamp keeps V = V0."""
    g, dyn = _disk_problem(31, "max")
    V0 = oracle_lib.target_cylinders(g, [0.13], [-0.21], [1.0])
    V, _ = oracle_lib.solve(g, dyn, sch, V0, 1.0)
    assert np.array_equal(V, V0)


def _car_small(nth=12):
    g = W.car_grid(24, 24, 8, nth)
    return g


@pytest.mark.parametrize("sch", [UP_EU, W.scheme("upwind1", "rk2"), ENO_RK])
def test_p5_tube_is_monotone(oracle_lib, sch):
    """The BRT only grows.  V^n <= V0 bit for bit at every step (the clamp).
    First-order upwind with CFL <= 1 is a monotone scheme (every update is a
    convex combination of neighbours, and TVD-RK2 is a convex combination of
    Euler steps), so {V^n <= 0} stays inside {V^(n+1) <= 0}.  ENO2 is not
    monotone: it may drop a node, but only one lying within a small band
    (0.1 h) of the zero level set."""
    g = _car_small()
    dyn = W.car_dynamics()
    cx, cy, r = W.cylinders(5, 3)
    V0 = oracle_lib.target_cylinders(g, cx, cy, r)
    dt = oracle_lib.cfl_dt(g, dyn, 0.8, 1.0)
    h = min(oracle_lib.spacing(g, 0), oracle_lib.spacing(g, 1))
    V = V0.copy()
    sizes = []
    for _ in range(20):
        Vn = oracle_lib.step(g, dyn, sch, V0, V, dt)
        assert np.all(Vn <= V0)
        lost = (V <= 0) & (Vn > 0)
        if sch["deriv"] == "upwind1":
            assert not lost.any()
        else:
            assert np.all(V[lost] > -0.1 * h)
            assert np.all(Vn[lost] < 0.1 * h)
        sizes.append(int((Vn <= 0).sum()))
        V = Vn
    assert sizes[-1] > sizes[0] > int((V0 <= 0).sum())


def test_p6_mirror_and_rotation_symmetry(oracle_lib):
    """The car is invariant under the mirror (x, y, theta) -> (x, -y, -theta)
    and the quarter turn (x, y, theta) -> (y, -x, theta - pi/2).  Solving
    for the mirrored/rotated obstacles gives the mirrored/rotated value
    function (first order scheme: to rounding)."""
    g = W.car_grid(20, 20, 6, 12)
    dyn = W.car_dynamics()
    cx, cy, r = W.cylinders(7, 3)
    T = 0.5
    V0 = oracle_lib.target_cylinders(g, cx, cy, r)
    V, _ = oracle_lib.solve(g, dyn, UP_EU, V0, T)
    # mirror: y -> -y, theta node l -> (N - l) mod N
    Vm0 = oracle_lib.target_cylinders(g, cx, -cy, r)
    Vm, _ = oracle_lib.solve(g, dyn, UP_EU, Vm0, T)
    lidx = (-np.arange(12)) % 12
    mapped = V[:, ::-1, :, :][:, :, :, lidx]
    assert np.abs(Vm - mapped).max() < 1e-11
    # rotation: obstacle (cx, cy) -> (cy, -cx); node (i, j, l) of the rotated
    # problem holds the original value at (N-1-j, i, l + N/4)
    Vr0 = oracle_lib.target_cylinders(g, cy, -cx, r)
    Vr, _ = oracle_lib.solve(g, dyn, UP_EU, Vr0, T)
    rot = np.transpose(V, (1, 0, 2, 3))[:, ::-1, :, :]
    rot = np.roll(rot, -3, axis=3)
    assert np.abs(Vr - rot).max() < 1e-11


def test_thread_count_invariance(oracle_lib):
    g = _car_small(nth=8)
    cx, cy, r = W.cylinders(3, 2)
    V0 = oracle_lib.target_cylinders(g, cx, cy, r)
    before = oracle_lib.threads()
    try:
        oracle_lib.set_threads(1)
        V1, _ = oracle_lib.solve(g, W.car_dynamics(d_max=0.1), ENO_RK, V0, 0.3)
        oracle_lib.set_threads(4)
        V4, _ = oracle_lib.solve(g, W.car_dynamics(d_max=0.1), ENO_RK, V0, 0.3)
    finally:
        oracle_lib.set_threads(before)
    assert np.array_equal(V1, V4)


def test_target_is_signed_distance(oracle_lib):
    """Eq (7): distance to the cone centre minus its radius; for a union the
    minimum over cones; the same value for every (v, theta)."""
    g = small_grid(nx=9, ny=7, nv=3, nth=4)
    V0 = oracle_lib.target_cylinders(g, [0.5, -2.0], [1.0, 0.0], [0.75, 0.4])
    x, _ = _line(g, 0)
    y, _ = _line(g, 1)
    d1 = np.hypot(x - 0.5, y - 1.0) - 0.75
    d2 = np.hypot(x + 2.0, y - 0.0) - 0.4
    np.testing.assert_allclose(V0, np.broadcast_to(np.minimum(d1, d2), g["n"]), atol=1e-14)


# ------------------------------------------------- steering car, eq (6) ---


def _steer_f(z, A, D, DX, DY, L):
    v, th = z[2], z[3]
    return np.stack([v * np.cos(th) + DX, v * np.sin(th) + DY, A, v * np.tan(D) / L], axis=-1)


def test_steer_hamiltonian_and_alpha_brute_force(oracle_lib):
    """The steering car's H (max over (a, delta), min over the disturbance)
    and alpha (max |f_d| over all inputs) by exhaustive search over grids of
    the input boxes that include their vertices; v of both signs."""
    rng = np.random.default_rng(21)
    dyn = W.steer_dynamics(d_max=0.1)
    dm, L = dyn["steer_max"], dyn["wheelbase"]
    s = np.linspace(-1, 1, 11)
    A, D, DX, DY = np.meshgrid(1.5 * s, dm * s, 0.1 * s, 0.1 * s, indexing="ij")
    for _ in range(40):
        z = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-2, 2), rng.uniform(-math.pi, math.pi)])
        p = rng.normal(size=4)
        if rng.random() < 0.2:
            p[rng.integers(4)] = 0.0
        f = _steer_f(z, A, D, DX, DY, L)
        bf = (f @ p).min(axis=(2, 3)).max()
        assert oracle_lib.hamiltonian(dyn, z, p) == pytest.approx(bf, abs=1e-12)
        np.testing.assert_allclose(oracle_lib.alpha(dyn, z), np.abs(f).reshape(-1, 4).max(axis=0), atol=1e-13)


def test_steer_is_car_with_speed_scaled_turn_rate(oracle_lib):
    """At speed v the steering car turns at most |v| tan(delta_max) / L, so
    its H and alpha equal the unicycle car's with that turn-rate bound."""
    rng = np.random.default_rng(22)
    st = W.steer_dynamics(d_max=0.05)
    for _ in range(30):
        z = np.array([0.3, -1.0, rng.uniform(0, 2), rng.uniform(-math.pi, math.pi)])
        p = rng.normal(size=4)
        car = W.car_dynamics(a_max=1.5, w_max=abs(z[2]) * math.tan(math.pi / 18) / 0.3, d_max=0.05)
        assert oracle_lib.hamiltonian(st, z, p) == pytest.approx(oracle_lib.hamiltonian(car, z, p), rel=1e-14,
                                                                  abs=1e-15)
        np.testing.assert_allclose(oracle_lib.alpha(st, z), oracle_lib.alpha(car, z), rtol=1e-14)


def test_steer_paper_turn_rate_bound(oracle_lib):
    """The paper's steering limits (delta in [-pi/18, pi/18], L = 0.3 m) at
    the grid's top speed of 2 m/s: the largest turn rate is
    2 tan(10 deg) / 0.3 = 1.17551 rad/s, which bounds alpha_theta."""
    a = oracle_lib.alpha(W.steer_dynamics(), np.array([0.0, 0.0, 2.0, 0.0]))
    assert a[3] == pytest.approx(1.1755132047, abs=1e-9)


def test_steer_mirror_symmetry(oracle_lib):
    """The steering car is invariant under the mirror (x, y, theta) ->
    (x, -y, -theta) too (delta -> -delta is admissible)."""
    g = W.car_grid(18, 18, 6, 12)
    dyn = W.steer_dynamics()
    cx, cy, r = W.cylinders(9, 3)
    V, _ = oracle_lib.solve(g, dyn, UP_EU, oracle_lib.target_cylinders(g, cx, cy, r), 0.5)
    Vm, _ = oracle_lib.solve(g, dyn, UP_EU, oracle_lib.target_cylinders(g, cx, -cy, r), 0.5)
    lidx = (-np.arange(12)) % 12
    assert np.abs(Vm - V[:, ::-1, :, :][:, :, :, lidx]).max() < 1e-11


# ------------------------------------------------------ convergence mode ---


@pytest.mark.parametrize("dyn", [W.car_dynamics(), W.steer_dynamics()], ids=["car", "steer"])
def test_converge_stops_at_first_small_change(oracle_lib, dyn):
    """The loop stops after the first step whose largest change is below the
    threshold: the result is that many plain steps, the change of the last
    step (recomputed here) is below it and the one before is not."""
    g = W.car_grid(16, 15, 6, 12)
    V0 = oracle_lib.target_cylinders(g, *W.cylinders(4, 3))
    thr = 2e-3
    V, info = oracle_lib.solve_converge(g, dyn, UP_EU, V0, thr, 500)
    assert info["converged"] and 2 <= info["steps"] < 500
    dt = oracle_lib.cfl_dt(g, dyn, 0.8, 1.0)
    assert info["dt"] == dt
    U, prev, eps = V0.copy(), None, []
    for _ in range(info["steps"]):
        prev = U
        U = oracle_lib.step(g, dyn, UP_EU, V0, U, dt)
        eps.append(np.abs(U - prev).max())
    assert np.array_equal(U, V)
    assert eps[-1] < thr <= eps[-2] and info["eps_last"] == eps[-1]


def test_converge_zero_dynamics_and_cap(oracle_lib):
    """Nothing moves: the first step changes nothing and stops the loop.  A
    zero threshold is never met: the loop runs exactly max_steps."""
    g = W.car_grid(10, 9, 5, 8)
    V0 = oracle_lib.target_cylinders(g, *W.cylinders(2, 2))
    V, info = oracle_lib.solve_converge(g, drift_dyn(), UP_EU, V0, 1e-12, 50)
    assert info["steps"] == 1 and info["converged"] and info["eps_last"] == 0.0 and np.array_equal(V, V0)
    V, info = oracle_lib.solve_converge(g, W.car_dynamics(), ENO_RK, V0, 0.0, 7)
    assert info["steps"] == 7 and not info["converged"]
    dt = oracle_lib.cfl_dt(g, W.car_dynamics(), 0.8, 1.0)
    U = V0.copy()
    for _ in range(7):
        U = oracle_lib.step(g, W.car_dynamics(), ENO_RK, V0, U, dt)
    assert np.array_equal(U, V)


# -------------------------------------------- optimal control, eq (9) ---


def _states(rng, m, g):
    lo, hi = np.array(g["lo"]), np.array(g["hi"])
    return lo + (hi - lo) * rng.uniform(size=(m, 4))


def test_control_on_linear_value(oracle_lib):
    """V = 0.7 x - 0.3 y - 1.2 v (constant in theta): every difference
    formula and the multilinear interpolation are exact, so the gradient is
    (0.7, -0.3, -1.2, 0) and V is reproduced at any state; the acceleration
    takes -a_max and the turn rate the tie value +w_max."""
    g = W.car_grid(9, 8, 6, 10)
    x, y, v = (oracle_lib.nodes(g, d) for d in range(3))
    V = 0.7 * x[:, None, None, None] - 0.3 * y[None, :, None, None] - 1.2 * v[None, None, :, None] \
        + np.zeros(g["n"])
    z = _states(np.random.default_rng(5), 200, g)
    u, val, gr = oracle_lib.optimal_control(g, W.car_dynamics(), V, z)
    np.testing.assert_allclose(gr, np.tile([0.7, -0.3, -1.2, 0.0], (200, 1)), atol=1e-13)
    np.testing.assert_allclose(val, 0.7 * z[:, 0] - 0.3 * z[:, 1] - 1.2 * z[:, 2], atol=1e-12)
    assert (u[:, 0] == -1.5).all() and (u[:, 1] == 1.0).all()


def test_control_turns_with_cos_theta(oracle_lib):
    """V = sin(theta) on the periodic axis: the nodal central difference is
    cos(theta) sin(h)/h, so the turn control follows the sign of cos(theta)
    away from its zeros, and the interpolated V is within h^2/8 of sin; a
    state one period away gives the same answer."""
    g = W.car_grid(5, 5, 4, 36)
    th = oracle_lib.nodes(g, 3)
    V = np.broadcast_to(np.sin(th), g["n"]).copy()
    rng = np.random.default_rng(6)
    z = _states(rng, 300, g)
    u, val, gr = oracle_lib.optimal_control(g, W.car_dynamics(), V, z)
    h = 2 * math.pi / 36
    clear = np.abs(np.cos(z[:, 3])) > 0.2
    assert (u[clear, 1] == np.where(np.cos(z[clear, 3]) > 0, 1.0, -1.0)).all()
    assert np.abs(val - np.sin(z[:, 3])).max() <= h * h / 8 + 1e-12
    z2 = z.copy()
    z2[:, 3] += 2 * math.pi
    u2, val2, _ = oracle_lib.optimal_control(g, W.car_dynamics(), V, z2)
    assert np.array_equal(u, u2) and np.allclose(val, val2, atol=1e-12)


@pytest.mark.parametrize("dyn", [W.car_dynamics(), W.steer_dynamics()], ids=["car", "steer"])
def test_control_is_argmax_over_inputs(oracle_lib, dyn):
    """With the interpolated gradient p the query returns, its control
    maximises p . f(z, u) over a grid of the control box (vertices
    included); for the steering car the turn follows the sign of p_theta v
    (v of both signs on this grid)."""
    g = W.car_grid(8, 7, 6, 9, v=(-1.0, 2.0))
    V = np.random.default_rng(7).normal(size=g["n"])
    z = _states(np.random.default_rng(8), 200, g)
    u, _, p = oracle_lib.optimal_control(g, dyn, V, z)
    s = np.linspace(-1, 1, 21)
    for q in range(len(z)):
        v, th = z[q, 2], z[q, 3]
        if dyn["kind"] == "car4d":
            A, Wr = np.meshgrid(1.5 * s, 1.0 * s, indexing="ij")
            turn = Wr
            chosen_turn = u[q, 1]
        else:
            A, Dl = np.meshgrid(1.5 * s, dyn["steer_max"] * s, indexing="ij")
            turn = v * np.tan(Dl) / dyn["wheelbase"]
            chosen_turn = v * math.tan(u[q, 1]) / dyn["wheelbase"]
        best = (p[q, 2] * A + p[q, 3] * turn).max()
        got = p[q, 2] * u[q, 0] + p[q, 3] * chosen_turn
        assert got == pytest.approx(best, abs=1e-12)


def test_control_undefined_for_test_dynamics(oracle_lib):
    g = W.car_grid(5, 5, 4, 8)
    with pytest.raises(ValueError):
        oracle_lib.optimal_control(g, drift_dyn(), np.zeros(g["n"]), np.zeros((1, 4)))


# ------------------------------ Algorithm 1: derivative-range alpha (f4) ---


def _dH_dp(dyn, z, p):
    """dH/dp at p (envelope: f at the optimal inputs), by the definitions."""
    k = dyn["kind"]
    if k in ("car4d", "car4d_steer"):
        dm = dyn.get("d_max", (0.0, 0.0))
        dx = -dm[0] if p[0] >= 0 else dm[0]
        dy = -dm[1] if p[1] >= 0 else dm[1]
        a = dyn["a_max"] if p[2] >= 0 else -dyn["a_max"]
        if k == "car4d":
            w = dyn["w_max"] if p[3] >= 0 else -dyn["w_max"]
        else:
            delta = dyn["steer_max"] if p[3] * z[2] >= 0 else -dyn["steer_max"]
            w = z[2] * math.tan(delta) / dyn["wheelbase"]
        return np.array([z[2] * math.cos(z[3]) + dx, z[2] * math.sin(z[3]) + dy, a, w])
    sgn = 1.0 if dyn["in_role"] == "max" else -1.0
    out = np.array(dyn["drift"], dtype=float)
    axes = dyn["in_axes"]
    if dyn["in_norm"] == "box":
        for d in axes:
            out[d] += sgn * (dyn["in_speed"] if p[d] >= 0 else -dyn["in_speed"])
    else:
        nrm = math.sqrt(sum(p[d] ** 2 for d in axes))
        if nrm > 0:
            for d in axes:
                out[d] += sgn * dyn["in_speed"] * p[d] / nrm
    return out


def _box_samples(lo, hi, k=7):
    s = set(np.linspace(lo, hi, k).tolist())
    if lo <= 0.0 <= hi:
        s.add(0.0)
    return sorted(s)


@pytest.mark.parametrize("dyn", [
    W.car_dynamics(d_max=0.1), W.steer_dynamics(d_max=0.05),
    drift_dyn((0.4, -0.3, 0.2, 0.0), (0, 1), 0.7, "box", "max"),
    drift_dyn((0.4, -0.3, 0.2, 0.0), (0, 1), 0.7, "box", "min"),
    drift_dyn((0.4, -0.3, 0.0, 0.1), (0, 1, 3), 0.7, "ball", "max"),
    drift_dyn((0.4, -0.3, 0.0, 0.1), (0, 1, 3), 0.7, "ball", "min"),
], ids=["car", "steer", "box-max", "box-min", "ball-max", "ball-min"])
def test_alpha_box_brute_force(oracle_lib, dyn):
    """Algorithm 1's alpha_d = max over the gradient box of |dH/dp_d|, by
    exhaustive search over a grid of the box that contains its corners and
    (where inside) zero: boxes of both signs, one-signed and degenerate."""
    rng = np.random.default_rng(31)
    for trial in range(25):
        lo, hi = np.empty(4), np.empty(4)
        for d in range(4):
            kind = rng.integers(4)
            a, b = sorted(rng.normal(size=2))
            if kind == 1:
                a, b = abs(a), abs(a) + abs(b)  # positive
            elif kind == 2:
                a, b = -abs(a) - abs(b), -abs(a)  # negative
            elif kind == 3:
                a = b = 0.0 if rng.random() < 0.5 else abs(a)
            lo[d], hi[d] = a, b
        z = np.array([0.1, -0.2, rng.uniform(-2, 2), rng.uniform(-math.pi, math.pi)])
        best = np.zeros(4)
        for p0 in _box_samples(lo[0], hi[0]):
            for p1 in _box_samples(lo[1], hi[1]):
                for p2 in _box_samples(lo[2], hi[2], 3):
                    for p3 in _box_samples(lo[3], hi[3]):
                        best = np.maximum(best, np.abs(_dH_dp(dyn, z, (p0, p1, p2, p3))))
        np.testing.assert_allclose(oracle_lib.alpha_box(dyn, z, lo, hi), best, rtol=0, atol=1e-12,
                                   err_msg=f"trial {trial}: box {lo} {hi}")


def test_deriv_range_exact_on_linear(oracle_lib):
    """V = 0.7 x - 0.3 y + 1.2 v: every one-sided difference (ends included,
    both schemes) is exact, so the ranges are the coefficients, and 0 on
    theta."""
    g = W.car_grid(9, 8, 6, 10)
    x, y, v = (oracle_lib.nodes(g, d) for d in range(3))
    V = 0.7 * x[:, None, None, None] - 0.3 * y[None, :, None, None] + 1.2 * v[None, None, :, None] \
        + np.zeros(g["n"])
    for sch in (UP_EU, ENO_RK):
        lo, hi = oracle_lib.deriv_range(g, sch, V)
        np.testing.assert_allclose(lo, [0.7, -0.3, 1.2, 0.0], atol=1e-12)
        np.testing.assert_allclose(hi, [0.7, -0.3, 1.2, 0.0], atol=1e-12)


def test_deriv_range_alpha_half_plane_closed_form(oracle_lib):
    """z' = 0.5 + u on x, |u| <= 1, u minimising, target V0 = x: the
    gradient is (1, 0, 0, 0) everywhere, the input is -1, so Algorithm 1's
    alpha_x = |0.5 - 1| = 0.5 (the state bound is 1.5): dt = 0.8 dx / 0.5,
    n = ceil(T / dt), and V_T = x - 0.5 T exactly (linear data, exact
    differences, no dissipation)."""
    g = W.car_grid(21, 6, 5, 8)
    dyn = drift_dyn((0.5, 0, 0, 0), (0,), 1.0, "box", "min")
    x = oracle_lib.nodes(g, 0)
    V0 = np.broadcast_to(x[:, None, None, None], g["n"]).copy()
    T = 2.1
    sch = W.scheme("upwind1", "euler", alpha="deriv_range")
    V, info = oracle_lib.solve(g, dyn, sch, V0, T)
    dx = 10.0 / 20
    dt = 0.8 * dx / 0.5
    assert info["dt"] == pytest.approx(dt, rel=1e-15)
    assert info["steps"] == math.ceil(T / dt)
    np.testing.assert_allclose(V, V0 - 0.5 * T, atol=1e-13)
    _, info_state = oracle_lib.solve(g, dyn, W.scheme("upwind1", "euler"), V0, T)
    assert info_state["dt"] == pytest.approx(0.8 * dx / 1.5, rel=1e-15)


@pytest.mark.parametrize("sch", [UP_EU, ENO_RK], ids=["upwind", "eno2"])
def test_deriv_range_equals_state_bound_when_gradients_span_zero(oracle_lib, sch):
    """Cylinder targets have gradients of every sign on x and y, so
    Algorithm 1's alpha reaches the state bound: the same steps and the same
    V (to the last bits of the accumulated time)."""
    g = W.car_grid(16, 15, 6, 12)
    dyn = W.car_dynamics(d_max=0.1)
    V0 = oracle_lib.target_cylinders(g, *W.cylinders(6, 3))
    a = dict(sch, alpha="deriv_range")
    V1, i1 = oracle_lib.solve(g, dyn, a, V0, 0.6)
    V2, i2 = oracle_lib.solve(g, dyn, sch, V0, 0.6)
    assert i1["steps"] == i2["steps"] and i1["dt"] == i2["dt"]
    assert np.abs(V1 - V2).max() < 1e-12


def test_deriv_range_central_vs_onesided_sawtooth_periodic(oracle_lib):
    """Algorithm 1 takes minDeriv / maxDeriv over the central derivative
    D_d V = (D+ + D-) / 2 of eq (5); the one-sided option over D- and D+
    together.  On a periodic axis with V_i = b (-1)^i (N even) every central
    difference is 0 while the one-sided ones are +-2b/h.  With z' = 0.5 + u
    on x, |u| <= 1 minimising (u = -1 where p >= 0, +1 where p < 0), the
    central box [0, 0] gives alpha_x = |0.5 - 1| = 0.5; the one-sided box
    [-2b/h, 2b/h] also admits u = +1, alpha_x = 1.5.  Nothing else moves,
    so dt = 0.8 h / alpha_x."""
    g = {"n": (8, 4, 3, 6), "lo": (0.0, -1.0, 0.0, -math.pi), "hi": (8.0, 1.0, 2.0, math.pi),
         "periodic_mask": 1 | 8}
    h, b = 1.0, 0.25
    saw = b * (-1.0) ** np.arange(8)
    V0 = np.broadcast_to(saw[:, None, None, None], g["n"]).copy()
    dyn = drift_dyn((0.5, 0, 0, 0), (0,), 1.0, "box", "min")
    central = W.scheme("upwind1", "euler", clamp=False, alpha="deriv_range")
    onesided = dict(central, alpha="deriv_range_onesided")
    lo, hi = oracle_lib.deriv_range(g, central, V0)
    assert lo[0] == 0.0 and hi[0] == 0.0
    lo, hi = oracle_lib.deriv_range(g, onesided, V0)
    assert lo[0] == -2 * b / h and hi[0] == 2 * b / h
    _, ic = oracle_lib.solve(g, dyn, central, V0, 10.0)
    _, io = oracle_lib.solve(g, dyn, onesided, V0, 10.0)
    assert ic["dt"] == pytest.approx(0.8 * h / 0.5, rel=1e-15)
    assert io["dt"] == pytest.approx(0.8 * h / 1.5, rel=1e-15)


def test_deriv_range_central_vs_onesided_ball_open_axes(oracle_lib):
    """V = a x + b (-1)^i + c y on open x, y axes (N_x even; linear
    extrapolation ghosts): interior central x-differences are a, the end
    nodes' (both one-sided differences equal there) a - 2b/h; interior
    one-sided ones a +- 2b/h.  So the central x box is [a - 2b/h, a], the
    one-sided one [a - 2b/h, a + 2b/h]; y is c everywhere.  With a
    maximising unit-ball input on (x, y) and no drift, dH/dp_x = p_x / |p|,
    largest at the box's largest p_x and smallest |p_y|: alpha_x = M /
    sqrt(M^2 + c^2), M = a (central) or a + 2b/h (one-sided); alpha_y =
    c / sqrt(c^2 + (a - 2b/h)^2) either way.  dt = 0.8 / (alpha_x / h_x +
    alpha_y / h_y)."""
    nx = 10
    g = {"n": (nx, 5, 3, 4), "lo": (-2.0, -1.0, 0.0, -math.pi), "hi": (2.5, 1.0, 2.0, math.pi),
         "periodic_mask": 8}
    hx, hy = 4.5 / (nx - 1), 2.0 / 4
    a, c = 1.0, 1.0
    b = 0.25 * hx  # 2b/h = 0.5
    x, y = oracle_lib.nodes(g, 0), oracle_lib.nodes(g, 1)
    V0 = (a * x + b * (-1.0) ** np.arange(nx))[:, None, None, None] + c * y[None, :, None, None] \
        + np.zeros(g["n"])
    dyn = drift_dyn((0, 0, 0, 0), (0, 1), 1.0, "ball", "max")
    central = W.scheme("upwind1", "euler", clamp=False, alpha="deriv_range")
    onesided = dict(central, alpha="deriv_range_onesided")
    for sch, M in ((central, a), (onesided, a + 0.5)):
        lo, hi = oracle_lib.deriv_range(g, sch, V0)
        np.testing.assert_allclose([lo[0], hi[0], lo[1], hi[1]], [a - 0.5, M, c, c], rtol=0, atol=1e-12)
        ax = M / math.sqrt(M * M + c * c)
        ay = c / math.sqrt(c * c + (a - 0.5) ** 2)
        _, info = oracle_lib.solve(g, dyn, sch, V0, 5.0)
        assert info["dt"] == pytest.approx(0.8 / (ax / hx + ay / hy), rel=1e-12), sch["alpha"]


# ------------------------- ENO choices taken in binary32 (FP32 parity checks) ---


def _line_grid(nx=8, ny=3):
    return {"n": (nx, ny, 3, 4), "lo": (0.0, 0.0, 0.0, -math.pi), "hi": (nx - 1.0, ny - 1.0, 2.0, math.pi),
            "periodic_mask": 8}


def _along_x(grid, prof):
    return np.broadcast_to(np.asarray(prof, dtype=float)[:, None, None, None], grid["n"]).copy()


@pytest.mark.parametrize("integ", ["euler", "rk2"])
def test_f32_decisions_upwind_has_no_choice(oracle_lib, integ):
    """First-order upwind takes no discrete choice: the binary32-decision step
    is the plain step, bit for bit, and its interval is a point."""
    g = W.car_grid(9, 8, 5, 8)
    dyn = W.car_dynamics(d_max=0.1)
    sch = W.scheme("upwind1", integ)
    V0 = oracle_lib.target_cylinders(g, *W.cylinders(3, 2))
    V = (V0 + 0.05 * np.random.default_rng(5).standard_normal(V0.shape)).astype(np.float32).astype(float)
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V0, V, 0.05, 0.0, 1e-5)
    ref = oracle_lib.step(g, dyn, sch, V0, V, 0.05)
    assert np.array_equal(lo, ref) and np.array_equal(hi, ref)


def test_f32_decisions_equal_f64_where_binary32_is_exact(oracle_lib):
    """Multiples of 1/64 below 2^10: every first and second difference is
    exact in binary32, so binary32 takes the binary64 choices and the step
    equals the plain ENO2 step bit for bit."""
    g = W.car_grid(9, 8, 5, 8)
    dyn = W.car_dynamics(d_max=0.1)
    sch = W.scheme("eno2", "euler")
    V = np.random.default_rng(8).integers(-256, 256, size=g["n"]) / 64.0
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V, V, 0.03)
    ref = oracle_lib.step(g, dyn, sch, V, V, 0.03)
    assert np.array_equal(lo, ref) and np.array_equal(hi, ref)


def test_f32_decisions_binary32_tie(oracle_lib):
    """An exact binary32 tie that binary64 does not see.  Along x (h = 1) the
    values ... 0, -2^-30, 1, 1.5, 2.5 ... around node 3: binary64 has
    Q_3 = 0.5 - (1 + 2^-30) = -0.5 - 2^-30 and Q_4 = 0.5, so |Q_3| > |Q_4|
    and p+ takes Q_4; in binary32 1 + 2^-30 rounds to 1, Q_3 = -0.5 ties with
    Q_4 and the tie takes the left one, Q_3.  With z' = 0.5 on x only, L =
    0.5 p+ (upwind), p+ = (V_4 - V_3) - c+/2: binary64 p+ = 0.25, binary32
    p+ = 0.75 + 2^-31; one Euler step of 0.5 from V_3 = 1 gives 1.0625 and
    1.1875 + 2^-33."""
    assert np.float32(1.0) - np.float32(-(2.0 ** -30)) == np.float32(1.0)  # the rounding that makes the tie
    g = _line_grid()
    V = _along_x(g, [0.0, 0.0, -(2.0 ** -30), 1.0, 1.5, 2.5, 3.5, 4.5])
    dyn = {"kind": "drift_input", "drift": (0.5, 0.0, 0.0, 0.0), "in_axes": (), "in_speed": 0.0,
           "in_norm": "box", "in_role": "max"}
    sch = W.scheme("eno2", "euler", clamp=False)
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V, V, 0.5)
    ref = oracle_lib.step(g, dyn, sch, V, V, 0.5)
    assert np.all(lo[3] == 1.1875 + 2.0 ** -33) and np.all(hi[3] == lo[3])
    assert np.all(ref[3] == 1.0625)


def test_f32_decisions_open_choice_interval(oracle_lib):
    """A binary32 margin of 2^-20 (Q_3 = -0.5 - 2^-30 against Q_4 = 0.5 +
    2^-20): closed (tau = 0) binary32 takes Q_3, the value 1.1875 + 2^-33; left
    open (tau = 1e-6 > 2^-20 / 2.5) the interval spans both candidates, p+ in
    {0.75 + 2^-31, 0.25 - 2^-21}: [1.0625 - 2^-23, 1.1875 + 2^-33]."""
    g = _line_grid()
    V = _along_x(g, [0.0, 0.0, -(2.0 ** -30), 1.0, 1.5, 2.5 + 2.0 ** -20, 3.5, 4.5])
    dyn = {"kind": "drift_input", "drift": (0.5, 0.0, 0.0, 0.0), "in_axes": (), "in_speed": 0.0,
           "in_norm": "box", "in_role": "max"}
    sch = W.scheme("eno2", "euler", clamp=False)
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V, V, 0.5)
    assert np.all(lo[3] == 1.1875 + 2.0 ** -33) and np.all(hi[3] == lo[3])
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V, V, 0.5, tau1=1e-6)
    assert np.all(lo[3] == 1.0625 - 2.0 ** -23) and np.all(hi[3] == 1.1875 + 2.0 ** -33)
    with pytest.raises(ValueError):
        oracle_lib.step_f32_decisions(g, dyn, W.scheme("eno2", "rk2"), V, V, 0.5, tau1=1e-6)


def test_f32_decisions_interval_corners_ball(oracle_lib):
    """The interval's ends are the corners of the open choices (L rises with
    every p+ and falls with every p-), also for the non-separable ball
    Hamiltonian: with open p+ choices on both x and y at node (3, 3), the
    ends equal the smallest and largest of the four combinations evaluated
    from the definition H = drift . pbar - s |pbar_xy| (a minimising unit
    ball), alpha_d = |drift_d| + s."""
    prof = np.array([0.0, 0.0, -(2.0 ** -30), 1.0, 1.5, 2.5 + 2.0 ** -20, 3.5, 4.5])
    g = _line_grid(8, 8)
    V = np.broadcast_to(prof[:, None, None, None] + 0.5 * prof[None, :, None, None], g["n"]).copy()
    drift = (0.3, -0.2, 0.0, 0.0)
    dyn = {"kind": "drift_input", "drift": drift, "in_axes": (0, 1), "in_speed": 1.0, "in_norm": "ball",
           "in_role": "min"}
    sch = W.scheme("eno2", "euler", clamp=False)
    dt = 0.1
    lo, hi = oracle_lib.step_f32_decisions(g, dyn, sch, V, V, dt, tau1=1e-6)
    # one-sided differences at node 3 of the profile (h = 1): p- takes Q_3 (|Q_2| > |Q_3|);
    # p+ candidates Q_3 = -0.5 - 2^-30 and Q_4 = 0.5 + 2^-20
    d1, d2 = 1.0 + 2.0 ** -30, 0.5
    q3, q4 = d2 - d1, (1.0 + 2.0 ** -20) - d2
    pm = d1 + q3 / 2
    cands = [d2 - q3 / 2, d2 - q4 / 2]
    vals = []
    for ppx in cands:
        for ppy in cands:
            p_plus, p_minus = np.array([ppx, 0.5 * ppy]), np.array([pm, 0.5 * pm])
            pbar = (p_plus + p_minus) / 2
            H = drift[0] * pbar[0] + drift[1] * pbar[1] - math.hypot(pbar[0], pbar[1])
            al = np.array([abs(drift[0]) + 1.0, abs(drift[1]) + 1.0])
            vals.append(V[3, 3, 0, 0] + dt * (H + float(np.sum(al * (p_plus - p_minus) / 2))))
    np.testing.assert_allclose(lo[3, 3], min(vals), rtol=0, atol=1e-14)
    np.testing.assert_allclose(hi[3, 3], max(vals), rtol=0, atol=1e-14)
