"""Python binding of the C ABI in ``include/hj.h`` (ctypes; argument
marshalling only -- every step of the solve runs in the gfx950 kernels of
``libhj.so``).

The functions keep the C names (``hj_grid_create`` ...).  Problem
descriptions are the dicts of ``paper_2012_04011_amd.workloads``.  Arrays are
numpy arrays (host) or torch tensors on the GPU (device; passed by
``data_ptr()``); streams are torch streams or raw ``hipStream_t`` integers.

There is no fallback: if ``libhj.so`` is missing, loading fails with an
error that says how to build it.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhj.so")

HJ_OK, HJ_ERR_INVALID_ARG, HJ_ERR_OUT_OF_MEMORY, HJ_ERR_DEVICE, HJ_ERR_NOT_READY, HJ_ERR_NONFINITE, \
    HJ_ERR_UNSUPPORTED = range(7)
HJ_F32, HJ_F64 = 0, 1
HJ_HOST, HJ_DEVICE = 0, 1
HJ_DYN_CAR4D, HJ_DYN_DRIFT_INPUT, HJ_DYN_CAR4D_STEER = 0, 1, 2
HJ_UPWIND1, HJ_ENO2 = 0, 1
HJ_EULER, HJ_TVD_RK2 = 0, 1
HJ_CLAMP_NONE, HJ_CLAMP_MIN_V0 = 0, 1
HJ_NORM_BOX, HJ_NORM_BALL = 0, 1
HJ_INPUT_MAXIMIZES, HJ_INPUT_MINIMIZES = 0, 1
HJ_BATCH_LAUNCHES, HJ_BATCH_GRAPH, HJ_BATCH_PERSISTENT, HJ_BATCH_STREAMS = 0, 1, 2, 3
HJ_ALPHA_STATE, HJ_ALPHA_DERIV_RANGE, HJ_ALPHA_DERIV_RANGE_ONESIDED = 0, 1, 2
HJ_NOALLOC_MAX_STATES = 65536
HJ_SERVE_SMALL_FIRST, HJ_SERVE_SHARE = 0, 1
SERVE_POLICIES = {"small_first": HJ_SERVE_SMALL_FIRST, "share": HJ_SERVE_SHARE}
BATCH_MODES = {"launches": HJ_BATCH_LAUNCHES, "graph": HJ_BATCH_GRAPH, "persistent": HJ_BATCH_PERSISTENT,
               "streams": HJ_BATCH_STREAMS}

STATUS_NAMES = {0: "HJ_OK", 1: "HJ_ERR_INVALID_ARG", 2: "HJ_ERR_OUT_OF_MEMORY", 3: "HJ_ERR_DEVICE",
                4: "HJ_ERR_NOT_READY", 5: "HJ_ERR_NONFINITE", 6: "HJ_ERR_UNSUPPORTED"}

EXPORTED = [
    "hj_grid_create", "hj_grid_destroy", "hj_set_target", "hj_set_target_cylinders", "hj_solve_brt",
    "hj_step", "hj_get_cfl_dt", "hj_get_alpha_max", "hj_get_value", "hj_get_target", "hj_set_value",
    "hj_get_num_points", "hj_set_profiling", "hj_get_profile", "hj_get_launch_info", "hj_autotune",
    "hj_set_autotune", "hj_solve_converge", "hj_optimal_control", "hj_optimal_control_noalloc", "hj_batch_create", "hj_batch_destroy", "hj_batch_solve", "hj_batch_set_tile",
    "hj_batch_set_spin_limit", "hj_batch_autotune", "hj_batch_get_info", "hj_server_create", "hj_server_destroy",
    "hj_server_submit", "hj_server_tick", "hj_server_poll", "hj_server_take", "hj_server_get_stats",
    "hj_last_error", "hj_version",
]


class HJError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class hj_grid_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 4), ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4),
                ("periodic_mask", ctypes.c_uint32)]


class hj_dynamics_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a_max", ctypes.c_double), ("w_max", ctypes.c_double),
                ("d_max", ctypes.c_double * 2), ("drift", ctypes.c_double * 4), ("in_speed", ctypes.c_double),
                ("in_axes_mask", ctypes.c_uint32), ("in_norm", ctypes.c_int32), ("in_role", ctypes.c_int32),
                ("steer_max", ctypes.c_double), ("wheelbase", ctypes.c_double)]


class hj_scheme_desc(ctypes.Structure):
    _fields_ = [("deriv", ctypes.c_int32), ("integrator", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("clamp", ctypes.c_int32), ("alpha_mode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("cfl", ctypes.c_double)]


class hj_solve_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("dt", ctypes.c_double), ("dt_last", ctypes.c_double),
                ("t_final", ctypes.c_double)]


class hj_launch_info(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("x_chunks", ctypes.c_int32), ("target_xy", ctypes.c_int32),
                ("autotuned", ctypes.c_int32), ("plane_segments", ctypes.c_int32), ("solve_graph", ctypes.c_int32),
                ("theta_run", ctypes.c_int32), ("span_blocks", ctypes.c_int32),
                ("plane_rows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bytes_per_point_step", ctypes.c_double)]


KERNEL_NAMES = {0: "generic", 1: "stream", 2: "plane"}


class hj_converge_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("converged", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dt", ctypes.c_double), ("eps_last", ctypes.c_double)]


class hj_batch_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("x_planes", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("graph_nodes", ctypes.c_int32), ("tiles_per_sweep", ctypes.c_int64),
                ("work_items", ctypes.c_int64), ("points", ctypes.c_int64), ("plane_kernel", ctypes.c_int32),
                ("classes", ctypes.c_int32)]


class hj_server_desc(ctypes.Structure):
    _fields_ = [("scheme", hj_scheme_desc), ("hbm_budget", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("x_planes", ctypes.c_int32), ("steps_per_tick", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("age_ms", ctypes.c_double)]


class hj_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("running", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("pad", ctypes.c_int32), ("slot_bytes", ctypes.c_int64)]


class hj_profile(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int64), ("step_launches", ctypes.c_int64), ("loop_ms", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libhj.so`` (raises if it has not been built).  With
    HJ_SANITIZE=1 the sanitizer build ``libhj_san.so`` is loaded instead
    (its runtime must be preloaded; see build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if os.environ.get("HJ_SANITIZE") == "1" and path == LIB_PATH:
        path = os.path.join(os.path.dirname(LIB_PATH), "libhj_san.so")
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run `python -m paper_2012_04011_amd.build` "
                          "(or __graft_entry__.build())")
    # PyTorch ships its own HIP runtime; loading it first makes libhj.so bind
    # to that one, so that torch tensors, streams and this library share one
    # runtime in the process whatever is imported first.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "hj_grid_create": [P(hj_grid_desc), P(hj_dynamics_desc), P(hj_scheme_desc), vp, P(vp)],
        "hj_grid_destroy": [vp],
        "hj_set_target": [vp, vp, i32, i32],
        "hj_set_target_cylinders": [vp, P(dbl), P(dbl), P(dbl), i32],
        "hj_solve_brt": [vp, dbl, P(hj_solve_info)],
        "hj_step": [vp, dbl, P(dbl)],
        "hj_get_cfl_dt": [vp, P(dbl)],
        "hj_get_alpha_max": [vp, P(dbl)],
        "hj_get_value": [vp, vp, i32, i32],
        "hj_get_target": [vp, vp, i32, i32],
        "hj_set_value": [vp, vp, i32, i32],
        "hj_get_num_points": [vp, P(i64)],
        "hj_set_profiling": [vp, i32],
        "hj_get_profile": [vp, P(hj_profile)],
        "hj_get_launch_info": [vp, P(hj_launch_info)],
        "hj_autotune": [vp],
        "hj_set_autotune": [vp, i32],
        "hj_solve_converge": [vp, dbl, i64, P(hj_converge_info)],
        "hj_optimal_control": [vp, vp, i64, i32, vp, vp],
        "hj_optimal_control_noalloc": [vp, vp, i64, i32, vp, vp],
        "hj_batch_create": [P(vp), i32, P(vp)],
        "hj_batch_destroy": [vp],
        "hj_batch_solve": [vp, P(dbl), i32, P(hj_solve_info)],
        "hj_batch_set_tile": [vp, i32],
        "hj_batch_set_spin_limit": [vp, i64],
        "hj_batch_autotune": [vp, P(dbl), i32, P(i32)],
        "hj_batch_get_info": [vp, P(hj_batch_info)],
        "hj_server_create": [P(hj_server_desc), vp, P(vp)],
        "hj_server_destroy": [vp],
        "hj_server_submit": [vp, P(hj_grid_desc), P(hj_dynamics_desc), P(dbl), P(dbl), P(dbl), i32, dbl, P(i64)],
        "hj_server_tick": [vp, P(i32)],
        "hj_server_poll": [vp, P(i64), i32, P(i32)],
        "hj_server_take": [vp, i64, vp, i32, i32],
        "hj_server_get_stats": [vp, P(hj_server_stats)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.hj_last_error.restype = ctypes.c_char_p
    lib.hj_last_error.argtypes = []
    lib.hj_version.restype = ctypes.c_char_p
    lib.hj_version.argtypes = []
    _lib = lib
    return lib


def _check(status: int, func: str):
    if status != HJ_OK:
        raise HJError(status, func, _lib.hj_last_error().decode())


# ----------------------------------------------------------- marshalling ---

_KIND = {"car4d": HJ_DYN_CAR4D, "drift_input": HJ_DYN_DRIFT_INPUT, "car4d_steer": HJ_DYN_CAR4D_STEER}
_DERIV = {"upwind1": HJ_UPWIND1, "eno2": HJ_ENO2}
_INTEG = {"euler": HJ_EULER, "rk2": HJ_TVD_RK2}
_NORM = {"box": HJ_NORM_BOX, "ball": HJ_NORM_BALL}
_ROLE = {"max": HJ_INPUT_MAXIMIZES, "min": HJ_INPUT_MINIMIZES}
_PREC = {"f32": HJ_F32, "f64": HJ_F64}


def grid_desc(grid: dict) -> hj_grid_desc:
    s = hj_grid_desc()
    for d in range(4):
        s.n[d], s.lo[d], s.hi[d] = int(grid["n"][d]), float(grid["lo"][d]), float(grid["hi"][d])
    s.periodic_mask = int(grid.get("periodic_mask", 0))
    return s


def dynamics_desc(dyn: dict) -> hj_dynamics_desc:
    s = hj_dynamics_desc()
    s.kind = _KIND[dyn["kind"]]
    s.a_max, s.w_max = float(dyn.get("a_max", 0.0)), float(dyn.get("w_max", 0.0))
    dm = dyn.get("d_max", (0.0, 0.0))
    s.d_max[0], s.d_max[1] = float(dm[0]), float(dm[1])
    for d, x in enumerate(dyn.get("drift", (0.0,) * 4)):
        s.drift[d] = float(x)
    s.in_speed = float(dyn.get("in_speed", 0.0))
    s.in_axes_mask = sum(1 << int(a) for a in dyn.get("in_axes", ()))
    s.in_norm = _NORM[dyn.get("in_norm", "box")]
    s.in_role = _ROLE[dyn.get("in_role", "max")]
    s.steer_max = float(dyn.get("steer_max", 0.0))
    s.wheelbase = float(dyn.get("wheelbase", 0.0))
    return s


def scheme_desc(scheme: dict, precision: str) -> hj_scheme_desc:
    s = hj_scheme_desc()
    s.deriv = _DERIV[scheme["deriv"]]
    s.integrator = _INTEG[scheme["integrator"]]
    s.precision = _PREC[precision]
    s.clamp = HJ_CLAMP_MIN_V0 if scheme.get("clamp", True) else HJ_CLAMP_NONE
    s.alpha_mode = {"state": HJ_ALPHA_STATE, "deriv_range": HJ_ALPHA_DERIV_RANGE,
                    "deriv_range_onesided": HJ_ALPHA_DERIV_RANGE_ONESIDED}[scheme.get("alpha", "state")]
    s.cfl = float(scheme.get("cfl", 0.8))
    return s


def _stream_handle(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _array_arg(a):
    """(pointer, dtype code, where code) of a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        dt = {np.dtype(np.float32): HJ_F32, np.dtype(np.float64): HJ_F64}.get(a.dtype)
        if dt is None:
            raise TypeError(f"unsupported dtype {a.dtype}")
        return a.ctypes.data, dt, HJ_HOST
    import torch

    if not isinstance(a, torch.Tensor):
        raise TypeError("expected a numpy array or a torch tensor")
    if not a.is_contiguous():
        raise ValueError("tensor must be contiguous")
    dt = {torch.float32: HJ_F32, torch.float64: HJ_F64}.get(a.dtype)
    if dt is None:
        raise TypeError(f"unsupported dtype {a.dtype}")
    if a.device.type == "cuda":
        return a.data_ptr(), dt, HJ_DEVICE
    return a.data_ptr(), dt, HJ_HOST


# --------------------------------------------------------- C-named calls ---


def hj_grid_create(grid: dict, dyn: dict, scheme: dict, precision: str = "f32", stream=None) -> int:
    lib = load_library()
    g, d, s = grid_desc(grid), dynamics_desc(dyn), scheme_desc(scheme, precision)
    out = ctypes.c_void_p()
    _check(lib.hj_grid_create(ctypes.byref(g), ctypes.byref(d), ctypes.byref(s), _stream_handle(stream),
                              ctypes.byref(out)), "hj_grid_create")
    return out.value


def hj_grid_destroy(h: int) -> None:
    _check(load_library().hj_grid_destroy(h), "hj_grid_destroy")


def hj_set_target(h: int, v0) -> None:
    ptr, dt, where = _array_arg(v0)
    _check(load_library().hj_set_target(h, ptr, dt, where), "hj_set_target")


def hj_set_target_cylinders(h: int, cx, cy, r) -> None:
    cx, cy, r = (np.ascontiguousarray(a, dtype=np.float64) for a in (cx, cy, r))
    if not (len(cx) == len(cy) == len(r)):
        raise ValueError("cx, cy, r must have the same length")
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load_library().hj_set_target_cylinders(h, cx.ctypes.data_as(dp), cy.ctypes.data_as(dp),
                                                  r.ctypes.data_as(dp), len(cx)), "hj_set_target_cylinders")


def hj_solve_brt(h: int, horizon: float) -> dict:
    info = hj_solve_info()
    _check(load_library().hj_solve_brt(h, float(horizon), ctypes.byref(info)), "hj_solve_brt")
    return {"steps": info.steps, "dt": info.dt, "dt_last": info.dt_last, "t_final": info.t_final}


def hj_step(h: int, dt: float = 0.0) -> float:
    taken = ctypes.c_double()
    _check(load_library().hj_step(h, float(dt), ctypes.byref(taken)), "hj_step")
    return taken.value


def hj_get_cfl_dt(h: int) -> float:
    dt = ctypes.c_double()
    _check(load_library().hj_get_cfl_dt(h, ctypes.byref(dt)), "hj_get_cfl_dt")
    return dt.value


def hj_get_alpha_max(h: int) -> np.ndarray:
    out = (ctypes.c_double * 4)()
    _check(load_library().hj_get_alpha_max(h, out), "hj_get_alpha_max")
    return np.array(out[:])


def hj_get_value(h: int, out) -> None:
    ptr, dt, where = _array_arg(out)
    _check(load_library().hj_get_value(h, ptr, dt, where), "hj_get_value")


def hj_get_target(h: int, out) -> None:
    ptr, dt, where = _array_arg(out)
    _check(load_library().hj_get_target(h, ptr, dt, where), "hj_get_target")


def hj_set_value(h: int, v) -> None:
    ptr, dt, where = _array_arg(v)
    _check(load_library().hj_set_value(h, ptr, dt, where), "hj_set_value")


def hj_get_num_points(h: int) -> int:
    n = ctypes.c_int64()
    _check(load_library().hj_get_num_points(h, ctypes.byref(n)), "hj_get_num_points")
    return n.value


def hj_set_profiling(h: int, enable: bool) -> None:
    _check(load_library().hj_set_profiling(h, 1 if enable else 0), "hj_set_profiling")


def hj_get_profile(h: int) -> dict:
    p = hj_profile()
    _check(load_library().hj_get_profile(h, ctypes.byref(p)), "hj_get_profile")
    return {"solves": p.solves, "step_launches": p.step_launches, "loop_ms": p.loop_ms}


def hj_get_launch_info(h: int) -> dict:
    li = hj_launch_info()
    _check(load_library().hj_get_launch_info(h, ctypes.byref(li)), "hj_get_launch_info")
    return {"kernel": KERNEL_NAMES.get(li.kernel, li.kernel), "x_chunks": li.x_chunks, "target_xy": bool(li.target_xy),
            "autotuned": bool(li.autotuned), "plane_segments": li.plane_segments,
            "solve_graph": bool(li.solve_graph), "theta_run": li.theta_run, "span_blocks": li.span_blocks,
            "plane_rows": li.plane_rows, "bytes_per_point_step": li.bytes_per_point_step}


def hj_autotune(h: int) -> None:
    _check(load_library().hj_autotune(h), "hj_autotune")


def hj_set_autotune(h: int, enable: bool) -> None:
    _check(load_library().hj_set_autotune(h, 1 if enable else 0), "hj_set_autotune")


def hj_solve_converge(h: int, threshold: float, max_steps: int) -> dict:
    i = hj_converge_info()
    _check(_lib.hj_solve_converge(h, float(threshold), int(max_steps), ctypes.byref(i)), "hj_solve_converge")
    return {"steps": i.steps, "converged": bool(i.converged), "dt": i.dt, "eps_last": i.eps_last}


def hj_optimal_control(h: int, states, controls=None, values=None, name: str = "hj_optimal_control"):
    """states: (m, 4) float64 numpy array (host) or torch tensor (device).
    Returns (controls (m, 2), values (m,)) of the same kind.  name selects
    the entry point: hj_optimal_control or hj_optimal_control_noalloc."""
    fn = getattr(_lib, name)
    if isinstance(states, np.ndarray) or not hasattr(states, "data_ptr"):
        z = np.ascontiguousarray(np.asarray(states, dtype=np.float64).reshape(-1, 4))
        m = z.shape[0]
        u = np.empty((m, 2)) if controls is None else controls
        val = np.empty(m) if values is None else values
        _check(fn(h, z.ctypes.data, m, HJ_HOST, u.ctypes.data, val.ctypes.data), name)
        return u, val
    import torch

    z = states.contiguous()
    if z.dtype != torch.float64:
        raise TypeError("states must be float64")
    m = z.shape[0]
    u = torch.empty((m, 2), dtype=torch.float64, device=z.device) if controls is None else controls
    val = torch.empty(m, dtype=torch.float64, device=z.device) if values is None else values
    _check(fn(h, z.data_ptr(), m, HJ_DEVICE, u.data_ptr(), val.data_ptr()), name)
    return u, val


def hj_optimal_control_noalloc(h: int, states, controls=None, values=None):
    """hj_optimal_control through the entry point that allocates no device
    memory (at most HJ_NOALLOC_MAX_STATES states)."""
    return hj_optimal_control(h, states, controls, values, "hj_optimal_control_noalloc")


def hj_batch_create(handles) -> int:
    arr = (ctypes.c_void_p * len(handles))(*handles)
    out = ctypes.c_void_p()
    _check(_lib.hj_batch_create(arr, len(handles), ctypes.byref(out)), "hj_batch_create")
    return out.value


def hj_batch_destroy(b: int) -> None:
    _check(_lib.hj_batch_destroy(b), "hj_batch_destroy")


def _horizons(h, m: int):
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (m,)))
    return h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def hj_batch_solve(b: int, m: int, horizons, mode: str = "launches") -> list:
    h, hp = _horizons(horizons, m)
    infos = (hj_solve_info * m)()
    _check(_lib.hj_batch_solve(b, hp, BATCH_MODES[mode], infos), "hj_batch_solve")
    return [{"steps": i.steps, "dt": i.dt, "dt_last": i.dt_last, "t_final": i.t_final} for i in infos]


def hj_batch_set_tile(b: int, x_planes: int) -> None:
    _check(_lib.hj_batch_set_tile(b, int(x_planes)), "hj_batch_set_tile")


def hj_batch_set_spin_limit(b: int, polls: int) -> None:
    _check(_lib.hj_batch_set_spin_limit(b, int(polls)), "hj_batch_set_spin_limit")


def hj_batch_autotune(b: int, m: int, horizons, mode: str = "launches") -> int:
    h, hp = _horizons(horizons, m)
    out = ctypes.c_int32()
    _check(_lib.hj_batch_autotune(b, hp, BATCH_MODES[mode], ctypes.byref(out)), "hj_batch_autotune")
    return out.value


def hj_batch_get_info(b: int) -> dict:
    i = hj_batch_info()
    _check(_lib.hj_batch_get_info(b, ctypes.byref(i)), "hj_batch_get_info")
    return {f: getattr(i, f) for f, _ in hj_batch_info._fields_}


def hj_server_create(scheme: dict, precision: str = "f32", hbm_budget: int = 0, max_inflight: int = 64,
                     x_planes: int = 0, stream=None, steps_per_tick: int = 0, policy: str = "small_first",
                     age_ms: float = 0.0) -> int:
    d = hj_server_desc()
    d.scheme = scheme_desc(scheme, precision)
    d.hbm_budget, d.max_inflight, d.x_planes = int(hbm_budget), int(max_inflight), int(x_planes)
    d.steps_per_tick = int(steps_per_tick)
    d.policy = SERVE_POLICIES[policy] if isinstance(policy, str) else int(policy)
    d.age_ms = float(age_ms)
    out = ctypes.c_void_p()
    _check(_lib.hj_server_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(out)), "hj_server_create")
    return out.value


def hj_server_destroy(s: int) -> None:
    _check(_lib.hj_server_destroy(s), "hj_server_destroy")


def hj_server_submit(s: int, grid: dict, dyn: dict, cx, cy, r, horizon: float) -> int:
    g, d = grid_desc(grid), dynamics_desc(dyn)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (cx, cy, r)]
    P = ctypes.POINTER(ctypes.c_double)
    out = ctypes.c_int64()
    _check(_lib.hj_server_submit(s, ctypes.byref(g), ctypes.byref(d), *[a.ctypes.data_as(P) for a in arrs],
                                 len(arrs[0]), float(horizon), ctypes.byref(out)), "hj_server_submit")
    return out.value


def hj_server_tick(s: int) -> int:
    n = ctypes.c_int32()
    _check(_lib.hj_server_tick(s, ctypes.byref(n)), "hj_server_tick")
    return n.value


def hj_server_poll(s: int, cap: int = 256) -> list:
    ids = (ctypes.c_int64 * cap)()
    n = ctypes.c_int32()
    _check(_lib.hj_server_poll(s, ids, cap, ctypes.byref(n)), "hj_server_poll")
    return list(ids[:n.value])


def hj_server_take(s: int, rid: int, out=None) -> None:
    if out is None:
        _check(_lib.hj_server_take(s, int(rid), None, HJ_F64, HJ_HOST), "hj_server_take")
        return
    p, dt, where = _array_arg(out)
    _check(_lib.hj_server_take(s, int(rid), p, dt, where), "hj_server_take")


def hj_server_get_stats(s: int) -> dict:
    st = hj_server_stats()
    _check(_lib.hj_server_get_stats(s, ctypes.byref(st)), "hj_server_get_stats")
    return {f: getattr(st, f) for f, _ in hj_server_stats._fields_ if f != "pad"}


def hj_last_error() -> str:
    return load_library().hj_last_error().decode()


def hj_version() -> str:
    return load_library().hj_version().decode()


# ------------------------------------------------------------ convenience ---


class Grid:
    """Owning wrapper of an ``hj_grid`` handle (same operations as the C
    calls)."""

    def __init__(self, grid: dict, dyn: dict, scheme: dict, precision: str = "f32", stream=None):
        self.grid, self.dyn, self.scheme, self.precision = grid, dyn, scheme, precision
        self.shape = tuple(int(x) for x in grid["n"])
        self.handle = hj_grid_create(grid, dyn, scheme, precision, stream)

    def close(self):
        if self.handle:
            hj_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_target(self, v0):
        hj_set_target(self.handle, v0)

    def set_target_cylinders(self, cx, cy, r):
        hj_set_target_cylinders(self.handle, cx, cy, r)

    def solve_brt(self, horizon: float) -> dict:
        return hj_solve_brt(self.handle, horizon)

    def step(self, dt: float = 0.0) -> float:
        return hj_step(self.handle, dt)

    def cfl_dt(self) -> float:
        return hj_get_cfl_dt(self.handle)

    def alpha_max(self) -> np.ndarray:
        return hj_get_alpha_max(self.handle)

    def value(self, dtype=np.float64) -> np.ndarray:
        out = np.empty(self.shape, dtype=dtype)
        hj_get_value(self.handle, out)
        return out

    def target(self, dtype=np.float64) -> np.ndarray:
        out = np.empty(self.shape, dtype=dtype)
        hj_get_target(self.handle, out)
        return out

    def get_value(self, out):
        hj_get_value(self.handle, out)

    def set_value(self, v):
        hj_set_value(self.handle, v)

    @property
    def num_points(self) -> int:
        return hj_get_num_points(self.handle)

    def set_profiling(self, enable: bool):
        hj_set_profiling(self.handle, enable)

    def profile(self) -> dict:
        return hj_get_profile(self.handle)

    def launch_info(self) -> dict:
        return hj_get_launch_info(self.handle)

    def solve_converge(self, threshold: float, max_steps: int) -> dict:
        return hj_solve_converge(self.handle, threshold, max_steps)

    def optimal_control(self, states):
        return hj_optimal_control(self.handle, states)

    def optimal_control_noalloc(self, states):
        return hj_optimal_control_noalloc(self.handle, states)

    def autotune(self):
        hj_autotune(self.handle)

    def set_autotune(self, enable: bool):
        hj_set_autotune(self.handle, enable)


class Batch:
    """Grids solved together (see hj_batch_create); holds references to them."""

    def __init__(self, grids):
        self.grids = list(grids)
        self.handle = hj_batch_create([g.handle for g in self.grids])

    def close(self):
        if getattr(self, "handle", None):
            hj_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, horizons, mode: str = "launches") -> list:
        return hj_batch_solve(self.handle, len(self.grids), horizons, mode)

    def set_tile(self, x_planes: int):
        hj_batch_set_tile(self.handle, x_planes)

    def set_spin_limit(self, polls: int):
        hj_batch_set_spin_limit(self.handle, polls)

    def autotune(self, horizons, mode: str = "launches") -> int:
        return hj_batch_autotune(self.handle, len(self.grids), horizons, mode)

    def info(self) -> dict:
        return hj_batch_get_info(self.handle)


class Server:
    """Continuous-batching re-solve server (see hj_server_create)."""

    def __init__(self, scheme: dict, precision: str = "f32", hbm_budget: int = 0, max_inflight: int = 64,
                 x_planes: int = 0, stream=None, steps_per_tick: int = 0, policy: str = "small_first",
                 age_ms: float = 0.0):
        self.handle = hj_server_create(scheme, precision, hbm_budget, max_inflight, x_planes, stream, steps_per_tick,
                                       policy, age_ms)

    def close(self):
        if getattr(self, "handle", None):
            hj_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, grid: dict, dyn: dict, cylinders, horizon: float) -> int:
        return hj_server_submit(self.handle, grid, dyn, *cylinders, horizon)

    def tick(self) -> int:
        return hj_server_tick(self.handle)

    def poll(self) -> list:
        return hj_server_poll(self.handle)

    def take(self, rid: int, out=None):
        hj_server_take(self.handle, rid, out)

    def stats(self) -> dict:
        return hj_server_get_stats(self.handle)
