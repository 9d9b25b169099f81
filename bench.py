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

HBM traffic of the stage kernel (the roofline's `traffic`) comes from two
rocprofv3 counter runs of this script (FETCH_SIZE, then WRITE_SIZE), each
scaled by what the same counter reads for a plain device copy of known size:

    python bench.py --copy-calibration          # the copy, under --pmc
    python bench.py --summarize-traffic DIR     # DIR/{stage,copy}_{fetch,write}
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


COPY_MIB = 512


def copy_calibration() -> int:
    """A plain device-to-device copy of COPY_MIB MiB, five times: the known
    byte count that calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    n = COPY_MIB * 2**20 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4, "dispatches": 5}}),
          flush=True)
    return 0


def _counter_rows(run_dir: str, counter: str):
    """(dispatch id, kernel name, value) of one counter from a rocprofv3
    --output-format csv run directory."""
    import csv
    import glob

    out = []
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    out.sort()
    return out


def summarize_traffic(root: str, last: int = 200) -> int:
    """Per-launch HBM bytes of the stage kernel from the counter runs under
    root (stage_fetch, stage_write: this script's default step under
    --pmc FETCH_SIZE / WRITE_SIZE; copy_fetch, copy_write: --copy-calibration).
    Counters are KiB per dispatch; each is scaled by copy bytes / copy counter.
    The last `last` stage dispatches (alternating TVD-RK2 stages 1 and 2 of
    the timed solve) are averaged.  Writes the JSON that the benchmark reads
    and prints a text summary."""
    import numpy as np

    from paper_2012_04011_amd import workloads as W

    copy_bytes = COPY_MIB * 2**20
    res = {}
    for counter, key in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        stage = [r for r in _counter_rows(os.path.join(root, "stage_" + key), counter) if "stage_" in r[1]]
        copy = [r for r in _counter_rows(os.path.join(root, "copy_" + key), counter)
                if "stage_" not in r[1] and "copy" in r[1].lower()]
        if len(stage) < last or not copy:
            print(f"summarize-traffic: {key}: {len(stage)} stage and {len(copy)} copy dispatches found",
                  file=sys.stderr)
            return 1
        v = np.array([r[2] for r in stage[-last:]])
        kib_copy = float(np.median([r[2] for r in copy]))
        factor = copy_bytes / (kib_copy * 1024.0)
        res[key] = {"stage1_kib": float(v[0::2].mean()), "stage2_kib": float(v[1::2].mean()),
                    "copy_kib": kib_copy, "factor": factor, "kernel": stage[-1][1]}
    f, w = res["fetch"], res["write"]
    s1 = (f["stage1_kib"] * f["factor"] + w["stage1_kib"] * w["factor"]) * 1024.0
    s2 = (f["stage2_kib"] * f["factor"] + w["stage2_kib"] * w["factor"]) * 1024.0
    out = {
        "kernel_source_sha256_16": kernel_source_hash(),
        "points": W.LARGE_120.points,
        "bytes_per_launch": (s1 + s2) / 2.0,
        "stage1_bytes": s1,
        "stage2_bytes": s2,
        "fetch": f,
        "write": w,
        "copy_bytes": copy_bytes,
    }
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"kernel: {f['kernel']}")
    print(f"copy of {copy_bytes} B: FETCH_SIZE {f['copy_kib']:.1f} KiB (x{f['factor']:.3f}), "
          f"WRITE_SIZE {w['copy_kib']:.1f} KiB (x{w['factor']:.3f})")
    for i, b in ((1, s1), (2, s2)):
        print(f"stage {i}: FETCH_SIZE {f[f'stage{i}_kib']:.1f} KiB, WRITE_SIZE {w[f'stage{i}_kib']:.1f} KiB "
              f"-> {b / 1e6:.1f} MB per launch (calibrated)")
    print(f"mean per launch: {out['bytes_per_launch'] / 1e6:.1f} MB; wrote {os.path.relpath(TRAFFIC_FILE, ROOT)}")
    return 0


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
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--summarize-traffic", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_traffic:
        return summarize_traffic(args.summarize_traffic)
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
    if args.copy_calibration:
        return copy_calibration()
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
