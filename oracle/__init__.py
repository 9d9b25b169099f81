"""FP64 CPU oracle for the HJ reachability time step (arXiv 2012.04011).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the HIP library never does.  It
shares no code with the HIP path: the C source ``hj_oracle.c`` recomputes every
quantity from the paper's definitions (section "Basic Numerical Solution",
eq (5), Algorithm 2, eq (6)-(7)) and the textbook ENO2 / TVD-RK2 methods.

Problem descriptions are plain dicts (see ``paper_2012_04011_amd.workloads``):

    grid   = {"n": (Nx, Ny, Nv, Nth), "lo": (...), "hi": (...), "periodic_mask": 8}
    dyn    = {"kind": "car4d", "a_max": 1.5, "w_max": 1.0, "d_max": (0.0, 0.0)}
             {"kind": "drift_input", "drift": (..4..), "in_speed": s,
              "in_axes": (0, 1), "in_norm": "box"|"ball", "in_role": "max"|"min"}
             {"kind": "car4d_steer", "a_max": 1.5, "steer_max": pi/18, "wheelbase": 0.3,
              "d_max": (0.0, 0.0)}
    scheme = {"deriv": "upwind1"|"eno2", "integrator": "euler"|"rk2",
              "clamp": True, "cfl": 0.8, "alpha": "state"|"deriv_range"|"deriv_range_onesided"}

Arrays are float64 numpy arrays of shape ``n`` in C order [x][y][v][theta].
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hj_oracle.c")
_LIB = os.path.join(_HERE, "libhjoracle.so")

# Plain optimisation, no fused multiply-add, portable x86-64 code (the library
# built here also runs on other hosts), OpenMP over the outermost grid axis.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


# HJ_SANITIZE=1: the same source built with AddressSanitizer and
# UndefinedBehaviorSanitizer by clang (the runtime the sanitized HIP library
# uses, so that one runtime serves both in an interpreter that preloads it),
# into libhjoracle_san.so, which is then the one loaded.
_LIB_SAN = os.path.join(_HERE, "libhjoracle_san.so")
SAN_CC = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan",
             "-fno-omit-frame-pointer", "-g"]


def _sanitize() -> bool:
    return os.environ.get("HJ_SANITIZE") == "1"


def build(force: bool = True, sanitize: bool | None = None) -> str:
    """Compile ``hj_oracle.c`` into ``libhjoracle.so`` with gcc (or, sanitized,
    into ``libhjoracle_san.so`` with clang)."""
    sanitize = _sanitize() if sanitize is None else sanitize
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp"
        if sanitize:
            flags = [f for f in CFLAGS if f != "-fopenmp"] + SAN_FLAGS
            subprocess.check_call([SAN_CC, *flags, "-o", tmp, _SRC, "-lm"])
        else:
            subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


class _Grid(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 4),
        ("lo", ctypes.c_double * 4),
        ("hi", ctypes.c_double * 4),
        ("periodic_mask", ctypes.c_uint32),
    ]


class _Dyn(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("a_max", ctypes.c_double),
        ("w_max", ctypes.c_double),
        ("d_max", ctypes.c_double * 2),
        ("drift", ctypes.c_double * 4),
        ("in_speed", ctypes.c_double),
        ("in_axes_mask", ctypes.c_uint32),
        ("in_norm", ctypes.c_int32),
        ("in_role", ctypes.c_int32),
        ("steer_max", ctypes.c_double),
        ("wheelbase", ctypes.c_double),
    ]


class _Scheme(ctypes.Structure):
    _fields_ = [
        ("deriv", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("clamp", ctypes.c_int32),
        ("alpha_mode", ctypes.c_int32),
        ("cfl", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _LIB_SAN if _sanitize() else _LIB
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        g, dy, sc = P(_Grid), P(_Dyn), P(_Scheme)
        lib.hjo_spacing.argtypes = [g, ctypes.c_int]
        lib.hjo_spacing.restype = ctypes.c_double
        lib.hjo_node.argtypes = [g, ctypes.c_int, ctypes.c_int]
        lib.hjo_node.restype = ctypes.c_double
        lib.hjo_target_cylinders.argtypes = [g, dp, dp, dp, ctypes.c_int32, dp]
        lib.hjo_hamiltonian.argtypes = [dy, dp, dp]
        lib.hjo_hamiltonian.restype = ctypes.c_double
        lib.hjo_alpha.argtypes = [dy, dp, dp]
        lib.hjo_alpha_max.argtypes = [g, dy, dp]
        lib.hjo_cfl_dt.argtypes = [g, dy, ctypes.c_double, ctypes.c_double]
        lib.hjo_cfl_dt.restype = ctypes.c_double
        lib.hjo_schedule.argtypes = [ctypes.c_double, ctypes.c_double, P(ctypes.c_int64), dp]
        lib.hjo_derivs.argtypes = [g, sc, dp, ctypes.c_int32, dp, dp]
        lib.hjo_rhs.argtypes = [g, dy, sc, dp, dp]
        lib.hjo_step.argtypes = [g, dy, sc, dp, dp, ctypes.c_double, dp]
        lib.hjo_step_f32dec.argtypes = [g, dy, sc, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        dp, dp]
        lib.hjo_step_f32dec.restype = ctypes.c_int
        lib.hjo_solve.argtypes = [g, dy, sc, dp, ctypes.c_double, dp, P(ctypes.c_int64), dp, dp]
        lib.hjo_solve.restype = ctypes.c_int
        lib.hjo_solve_converge.argtypes = [g, dy, sc, dp, ctypes.c_double, ctypes.c_int64, dp, P(ctypes.c_int64),
                                           P(ctypes.c_int32), dp, dp]
        lib.hjo_solve_converge.restype = ctypes.c_int
        lib.hjo_optimal_control.argtypes = [g, dy, dp, dp, ctypes.c_int64, dp, dp, dp]
        lib.hjo_deriv_range.argtypes = [g, sc, dp, dp, dp]
        lib.hjo_alpha_box.argtypes = [dy, dp, dp, dp, dp]
        lib.hjo_optimal_control.restype = ctypes.c_int
        lib.hjo_threads.restype = ctypes.c_int32
        lib.hjo_set_threads.argtypes = [ctypes.c_int32]
        _lib = lib
    return _lib


# ----------------------------------------------------------- marshalling ---

_KIND = {"car4d": 0, "drift_input": 1, "car4d_steer": 2}
_DERIV = {"upwind1": 0, "eno2": 1}
_INTEG = {"euler": 0, "rk2": 1}
_NORM = {"box": 0, "ball": 1}
_ROLE = {"max": 0, "min": 1}
_ALPHA = {"state": 0, "deriv_range": 1, "deriv_range_onesided": 2}


def _grid(grid) -> _Grid:
    s = _Grid()
    for d in range(4):
        s.n[d] = int(grid["n"][d])
        s.lo[d] = float(grid["lo"][d])
        s.hi[d] = float(grid["hi"][d])
    s.periodic_mask = int(grid.get("periodic_mask", 0))
    return s


def _dyn(dyn) -> _Dyn:
    s = _Dyn()
    s.kind = _KIND[dyn["kind"]]
    s.a_max = float(dyn.get("a_max", 0.0))
    s.w_max = float(dyn.get("w_max", 0.0))
    dm = dyn.get("d_max", (0.0, 0.0))
    s.d_max[0], s.d_max[1] = float(dm[0]), float(dm[1])
    dr = dyn.get("drift", (0.0, 0.0, 0.0, 0.0))
    for d in range(4):
        s.drift[d] = float(dr[d])
    s.in_speed = float(dyn.get("in_speed", 0.0))
    mask = 0
    for a in dyn.get("in_axes", ()):
        mask |= 1 << int(a)
    s.in_axes_mask = mask
    s.in_norm = _NORM[dyn.get("in_norm", "box")]
    s.in_role = _ROLE[dyn.get("in_role", "max")]
    s.steer_max = float(dyn.get("steer_max", 0.0))
    s.wheelbase = float(dyn.get("wheelbase", 1.0))
    return s


def _scheme(scheme) -> _Scheme:
    s = _Scheme()
    s.deriv = _DERIV[scheme["deriv"]]
    s.integrator = _INTEG[scheme["integrator"]]
    s.clamp = 1 if scheme.get("clamp", True) else 0
    s.alpha_mode = _ALPHA[scheme.get("alpha", "state")]
    s.cfl = float(scheme.get("cfl", 0.8))
    return s


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _shape(grid):
    return tuple(int(x) for x in grid["n"])


# ------------------------------------------------------------- public API ---


def spacing(grid, d: int) -> float:
    return _load().hjo_spacing(ctypes.byref(_grid(grid)), d)


def nodes(grid, d: int) -> np.ndarray:
    lib, g = _load(), _grid(grid)
    return np.array([lib.hjo_node(ctypes.byref(g), d, i) for i in range(int(grid["n"][d]))])


def target_cylinders(grid, cx, cy, r) -> np.ndarray:
    cx, cy, r = _f64(cx), _f64(cy), _f64(r)
    out = np.empty(_shape(grid), dtype=np.float64)
    _load().hjo_target_cylinders(ctypes.byref(_grid(grid)), _dptr(cx), _dptr(cy), _dptr(r), len(cx), _dptr(out))
    return out


def hamiltonian(dyn, z, p) -> float:
    z, p = _f64(z), _f64(p)
    return _load().hjo_hamiltonian(ctypes.byref(_dyn(dyn)), _dptr(z), _dptr(p))


def alpha(dyn, z) -> np.ndarray:
    z = _f64(z)
    out = np.empty(4)
    _load().hjo_alpha(ctypes.byref(_dyn(dyn)), _dptr(z), _dptr(out))
    return out


def alpha_max(grid, dyn) -> np.ndarray:
    out = np.empty(4)
    _load().hjo_alpha_max(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), _dptr(out))
    return out


def cfl_dt(grid, dyn, cfl: float, horizon: float) -> float:
    return _load().hjo_cfl_dt(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), cfl, horizon)


def schedule(dt: float, horizon: float):
    n = ctypes.c_int64()
    last = ctypes.c_double()
    _load().hjo_schedule(dt, horizon, ctypes.byref(n), ctypes.byref(last))
    return n.value, last.value


def derivs(grid, scheme, V, axis: int):
    V = _f64(V, _shape(grid))
    pm = np.empty_like(V)
    pp = np.empty_like(V)
    _load().hjo_derivs(ctypes.byref(_grid(grid)), ctypes.byref(_scheme(scheme)), _dptr(V), axis, _dptr(pm), _dptr(pp))
    return pm, pp


def rhs(grid, dyn, scheme, V) -> np.ndarray:
    V = _f64(V, _shape(grid))
    L = np.empty_like(V)
    _load().hjo_rhs(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), ctypes.byref(_scheme(scheme)), _dptr(V), _dptr(L))
    return L


def step(grid, dyn, scheme, V0, V, dt: float) -> np.ndarray:
    """One full step of length dt from V (returns a new array)."""
    V0 = _f64(V0, _shape(grid))
    out = _f64(V, _shape(grid)).copy()
    work = np.empty(2 * out.size)
    _load().hjo_step(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), ctypes.byref(_scheme(scheme)),
                     _dptr(V0), _dptr(out), float(dt), _dptr(work))
    return out


def step_f32_decisions(grid, dyn, scheme, V0, V, dt: float, tau1: float = 0.0, tau2: float = 0.0):
    """One full step from V whose ENO choices are those a binary32 evaluation
    takes (decided on binary32 second differences; all other arithmetic
    binary64).  Returns (lo, hi): per node the smallest and largest result
    over the choices left open -- those within tau * max(1, |window|) of a
    tie, tau1 in the first stage, tau2 in the second TVD-RK2 stage (tau1 must
    be 0 with TVD-RK2)."""
    V0 = _f64(V0, _shape(grid))
    V = _f64(V, _shape(grid))
    lo = np.empty_like(V)
    hi = np.empty_like(V)
    rc = _load().hjo_step_f32dec(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), ctypes.byref(_scheme(scheme)),
                                 _dptr(V0), _dptr(V), float(dt), float(tau1), float(tau2), _dptr(lo), _dptr(hi))
    if rc == -2:
        raise ValueError("tau1 > 0 needs a one-stage (Euler) step")
    if rc != 0:
        raise MemoryError("oracle step: out of memory")
    return lo, hi


def solve(grid, dyn, scheme, V0, horizon: float):
    """Fixed-horizon solve; returns (V, info) with info = {steps, dt, dt_last}."""
    V0 = _f64(V0, _shape(grid))
    V = np.empty_like(V0)
    n = ctypes.c_int64()
    dt = ctypes.c_double()
    last = ctypes.c_double()
    rc = _load().hjo_solve(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), ctypes.byref(_scheme(scheme)),
                           _dptr(V0), float(horizon), _dptr(V), ctypes.byref(n), ctypes.byref(dt), ctypes.byref(last))
    if rc != 0:
        raise MemoryError("oracle solve: out of memory")
    return V, {"steps": n.value, "dt": dt.value, "dt_last": last.value}


def solve_converge(grid, dyn, scheme, V0, threshold: float, max_steps: int):
    """Convergence-mode solve (steps of the CFL dt until the largest change of
    a step falls below `threshold`, at most max_steps); returns (V, info)
    with info = {steps, converged, eps_last, dt}."""
    V0 = _f64(V0, _shape(grid))
    V = np.empty_like(V0)
    n = ctypes.c_int64()
    conv = ctypes.c_int32()
    eps = ctypes.c_double()
    dt = ctypes.c_double()
    rc = _load().hjo_solve_converge(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), ctypes.byref(_scheme(scheme)),
                                    _dptr(V0), float(threshold), int(max_steps), _dptr(V), ctypes.byref(n),
                                    ctypes.byref(conv), ctypes.byref(eps), ctypes.byref(dt))
    if rc == -2:
        raise ValueError("convergence mode needs the state-bound alpha")
    if rc != 0:
        raise MemoryError("oracle converge: out of memory")
    return V, {"steps": n.value, "converged": bool(conv.value), "eps_last": eps.value, "dt": dt.value}


def optimal_control(grid, dyn, V, states):
    """Eq (9) at each state (rows of `states`, shape (m, 4)): returns
    (controls (m, 2), values (m,), gradients (m, 4))."""
    V = _f64(V, _shape(grid))
    z = np.ascontiguousarray(np.asarray(states, dtype=np.float64).reshape(-1, 4))
    m = z.shape[0]
    u = np.empty((m, 2))
    val = np.empty(m)
    gr = np.empty((m, 4))
    rc = _load().hjo_optimal_control(ctypes.byref(_grid(grid)), ctypes.byref(_dyn(dyn)), _dptr(V), _dptr(z), m,
                                     _dptr(u), _dptr(val), _dptr(gr))
    if rc != 0:
        raise ValueError("optimal control is defined for the car dynamics only")
    return u, val, gr


def deriv_range(grid, scheme, V):
    """(pmin, pmax) per axis: Algorithm 1's minDeriv / maxDeriv, over the
    central derivative (alpha "deriv_range") or over both one-sided
    derivatives (alpha "deriv_range_onesided")."""
    V = _f64(V, _shape(grid))
    lo, hi = np.empty(4), np.empty(4)
    _load().hjo_deriv_range(ctypes.byref(_grid(grid)), ctypes.byref(_scheme(scheme)), _dptr(V), _dptr(lo), _dptr(hi))
    return lo, hi


def alpha_box(dyn, z, pmin, pmax) -> np.ndarray:
    """Algorithm 1's alpha at state z for the gradient box [pmin, pmax]."""
    z, lo, hi = _f64(z), _f64(pmin), _f64(pmax)
    out = np.empty(4)
    _load().hjo_alpha_box(ctypes.byref(_dyn(dyn)), _dptr(z), _dptr(lo), _dptr(hi), _dptr(out))
    return out


def threads() -> int:
    return int(_load().hjo_threads())


def set_threads(n: int) -> None:
    _load().hjo_set_threads(int(n))
