"""Benchmark: BRT solves of the 4D car on one MI355X.

One step = one whole BRT re-solve through the C ABI on device-resident
buffers: the cylinder target V0 (and V := V0) for a fresh seeded obstacle set,
then the fixed-horizon time loop (n = ceil(T / dt) steps of the fused
Lax-Friedrichs stage kernel; the CFL step is computed once per grid when the
grid handle is first solved, as its dissipation bounds depend on the grid only).

Workload: 120x120x40x72 (41.5M points), ENO2 + TVD-RK2, FP32, horizon 2 s
(221 steps), 8 seeded cylinders.  Throughput = points x steps / wall time.

Printed: one JSON line with the throughput, the roofline of the dominant
kernel (algorithmic bytes per launch over its average launch time, measured
with HIP events on the stream the kernels run on) and the FP64 CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point updates/s (% HBM roofline); p50/p99 BRT re-solve latency"
UNIT = "grid-point updates/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2012_04011_amd", "csrc", "hj_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_large_120_f32.json")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes_per_launch(npts: int, info: dict, integrator: str) -> float:
    """Bytes a stage must move with ideal on-chip reuse (ghosts excluded),
    from the library's byte model of the mode that ran: each array read once
    and written once per stage.  TVD-RK2: stage 1 reads V^n and writes V^1;
    stage 2 reads V^1 and V^n, reads V0 unless the target is the Nx*Ny table
    of a cylinder target (constant over v, theta), and writes V^(n+1).  Both
    stages run the same kernel, so a launch moves half a step's bytes."""
    launches = 1 if integrator == "euler" else 2
    return info["bytes_per_point_step"] * npts / launches


def measured_traffic(npts_expected: int):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    committed under profiles/, if they were taken on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("points") != npts_expected:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(wl, budget_s: float = 15.0) -> dict:
    """The FP64 oracle on the host cores: whole RK2 steps of the same
    workload from its seed-0 target, as many as fit the time budget."""
    import numpy as np

    import oracle
    from paper_2012_04011_amd import workloads as W

    oracle.build(force=False)
    cx, cy, r = W.cylinders(0, wl.obstacles)
    V0 = oracle.target_cylinders(wl.grid, cx, cy, r)
    dt = oracle.cfl_dt(wl.grid, wl.dyn, wl.scheme["cfl"], wl.horizon)
    V = V0.copy()
    steps, t0 = 0, time.perf_counter()
    while True:
        V = oracle.step(wl.grid, wl.dyn, wl.scheme, V0, V, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el + el / steps > budget_s:
            break
    del V, V0
    return {
        "value": wl.points * steps / el,
        "unit": UNIT,
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"{steps} full ENO2+TVD-RK2 FP64 step(s) of the {'x'.join(map(str, wl.grid['n']))} grid "
                  f"({wl.points * steps / 1e6:.1f}M point-steps, {el:.1f} s)",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); the multi-GPU split is "
              "design-only", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2012_04011_amd import hj
    from paper_2012_04011_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    hj.load_library()
    torch.cuda.set_device(0)
    wl = W.LARGE_120
    stream = torch.cuda.current_stream()
    g = hj.Grid(wl.grid, wl.dyn, wl.scheme, wl.precision, stream)
    npts = g.num_points
    obstacle_sets = [W.cylinders(s, wl.obstacles) for s in range(args.warmup + args.steps)]

    info = None
    for s in range(args.warmup):
        g.set_target_cylinders(*obstacle_sets[s])
        info = g.solve_brt(wl.horizon)
    torch.cuda.synchronize()

    g.set_profiling(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        g.set_target_cylinders(*obstacle_sets[args.warmup + s])
        info = g.solve_brt(wl.horizon)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = g.profile()
    launch = g.launch_info()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    g.close()

    steps_per_solve = info["steps"]
    value = npts * steps_per_solve * args.steps / wall
    bpl = algorithmic_bytes_per_launch(npts, launch, wl.scheme["integrator"])
    avg_launch_s = prof["loop_ms"] / 1e3 / prof["step_launches"]
    achieved = bpl / avg_launch_s / 1e9
    traffic = measured_traffic(npts)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded cylinder obstacles)",
        "config": {
            "workload": "car4d 120x120x40x72 (41.5M points) ENO2+TVD-RK2 FP32, horizon 2 s, 8 cylinders",
            "grid": list(wl.grid["n"]),
            "points": npts,
            "scheme": "eno2+rk2",
            "horizon_s": wl.horizon,
            "steps_per_solve": steps_per_solve,
            "dt": info["dt"],
            "obstacles": wl.obstacles,
            "stage_kernel": launch["kernel"],
            "x_chunks": launch["x_chunks"],
            "target": "xy table (cylinders)" if launch["target_xy"] else "4D V0",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "stage kernel (both TVD-RK2 stages)",
            "bytes_per_launch": bpl,
            "bytes_per_point_step": launch["bytes_per_point_step"],
            "avg_launch_us": avg_launch_s * 1e6,
            "launches_timed": prof["step_launches"],
        },
        "solve_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "min": float(lat.min())},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
