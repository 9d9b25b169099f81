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
    python bench.py --workload eno60       # the paper's grid, ENO2 + TVD-RK2 with disturbance
    python bench.py --workload batch64     # the uneven 64-instance batch
    python bench.py --workload serve       # the Poisson re-solve stream, served and one at a time
    python bench.py --workload context     # the paper's grid and car, 67 iterations
    python bench.py --precision f64        # the headline workload in FP64

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


def measured_traffic(npts_expected: int, x_chunks: int, plane_rows: int = 1):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    committed under profiles/, if they were taken on the current kernels in
    the same launch configuration (x chunks: each adds halo planes; y rows
    per plane-kernel block: two-row blocks split the plane along v)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("points") != npts_expected or
            t.get("x_chunks") != x_chunks or t.get("plane_rows", 1) != plane_rows):
        return None
    return t.get("bytes_per_launch")


COPY_MIB = 512


def copy_bandwidth_gbs(stream) -> float:
    """Read + write GB/s of a plain 1 GiB device-to-device copy on `stream`
    (best of 5): the practical bandwidth ceiling beside the nominal 8 TB/s."""
    import torch

    n = 2**30 // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    with torch.cuda.stream(stream):
        dst.copy_(src)
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dst.copy_(src)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * n * 4 / best / 1e9


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
    # the launch configuration of the counted runs, from the JSON line each
    # printed
    chunks = set()
    for key in ("fetch", "write"):
        try:
            with open(os.path.join(root, f"stage_{key}.log")) as fh:
                for line in fh:
                    if line.startswith("{"):
                        cfg = json.loads(line)["config"]
                        chunks.add((cfg["x_chunks"], cfg.get("plane_rows", 1)))
        except (OSError, ValueError, KeyError):
            pass
    if len(chunks) != 1:
        print(f"summarize-traffic: the stage runs' launch configurations are not one known value: {sorted(chunks)}",
              file=sys.stderr)
        return 1
    x_chunks, plane_rows = chunks.pop()
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
        "x_chunks": x_chunks,
        "plane_rows": plane_rows,
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


def bench_batch(args) -> int:
    """The uneven 64-instance batch (each grid's launch configuration
    autotuned alone first): every mode of hj_batch_solve beside the
    same solves run one grid at a time, fixed 16-plane tiles beside the
    autotuned tile length, and the launches on the streaming tiles alone
    beside the default mix of batched plane-kernel classes and streaming
    tiles.  One JSON line; throughput is whole-batch point-steps over the
    solve time of the faster of the autotuned graph mode and the
    concurrent-streams mode."""
    import numpy as np
    import torch

    from paper_2012_04011_amd import hj
    from paper_2012_04011_amd import workloads as W

    hj.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    insts = W.batch_instances(**W.BATCH_64)
    H = [i.horizon for i in insts]
    grids = []
    for ins in insts:
        g = hj.Grid(ins.grid, ins.dyn, ins.scheme, "f32", stream)
        g.set_target_cylinders(*ins.cylinders)
        g.autotune()  # each grid's own launch configuration, timed alone before the batch
        grids.append(g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return t

    one = timed(lambda: [g.solve_brt(h) for g, h in zip(grids, H)], max(1, args.steps // 3))
    b = hj.Batch(grids)
    infos = b.solve(H, "launches")
    point_steps = sum(i.points * f["steps"] for i, f in zip(insts, infos))
    res = {}
    b.set_tile(16)
    for mode in ("launches", "graph", "persistent"):
        res[mode] = timed(lambda: b.solve(H, mode), max(1, args.steps // 3))
    tuned = b.autotune(H, "graph")
    res["graph_tuned"] = timed(lambda: b.solve(H, "graph"), args.steps)
    res["streams"] = timed(lambda: b.solve(H, "streams"), args.steps)
    b.solve(H, "graph")
    info = b.info()
    b.close()
    os.environ["HJ_BATCH_KERNEL"] = "stream"  # read when a batch is created
    try:
        bs = hj.Batch(grids)
    finally:
        del os.environ["HJ_BATCH_KERNEL"]
    bs.set_tile(16)
    res["graph_tiles_only"] = timed(lambda: bs.solve(H, "graph"), max(1, args.steps // 3))
    bs.close()
    for g in grids:
        g.close()
    best = min(("graph_tuned", "streams"), key=lambda k: float(np.median(res[k])))
    ms = float(np.median(res[best]))
    value = point_steps / (ms / 1e3)
    bpps = 20.0  # FP32 TVD-RK2 with the cylinder x-y target (see the single-grid byte model)
    achieved = value * bpps / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (64 seeded uneven instances)",
        "config": {
            "workload": "batch: 64 uneven car4d instances 30x30x12x18..80x80x24x48, 1-8 cylinders, horizons "
                        "0.5-2 s, ENO2+TVD-RK2 FP32",
            "points": info["points"], "point_steps": point_steps,
            "mode": "graph" if best == "graph_tuned" else "streams",
            "x_planes_autotuned": tuned, "tiles_per_sweep": info["tiles_per_sweep"],
            "graph_nodes": info["graph_nodes"], "launch_classes": info["classes"],
        },
        "modes_ms": {
            "one_grid_at_a_time": float(np.median(one)),
            "launches_fixed16": float(np.median(res["launches"])),
            "graph_fixed16": float(np.median(res["graph"])),
            "persistent_fixed16": float(np.median(res["persistent"])),
            "graph_autotuned": float(np.median(res["graph_tuned"])),
            "graph_streaming_tiles_only_fixed16": float(np.median(res["graph_tiles_only"])),
            "streams": float(np.median(res["streams"])),
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("batched plane-kernel classes and streaming tiles" if best == "graph_tuned" else
                                "single-grid stage kernels on four concurrent streams") +
                               " (whole solve, both stages)", "bytes_per_point_step": bpps},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    """A Poisson stream of re-solves (20 per second, 70 % on 60x60x20x36 and
    30 % on 100x100x24x48, 1-3 obstacle changes each, horizon 1.5 s) played
    in real time three times: through the continuous-batching server with
    its default policy (small requests first, large ones in arrival order)
    and with every running request stepping every tick (sharing), and one
    request at a time (first in, first out, each solved alone on its class's
    resident grid).
    Latency = completion seen on the host - arrival."""
    import numpy as np
    import torch

    from paper_2012_04011_amd import hj
    from paper_2012_04011_amd import workloads as W

    hj.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n_req = max(20, args.requests)
    sch = W.scheme("eno2", "rk2")

    def play_server(reqs, policy="small_first"):
        lat, done, idmap = [], 0, {}
        with hj.Server(sch, "f32", hbm_budget=args.hbm_budget, max_inflight=64, stream=stream, policy=policy,
                       age_ms=args.age_ms) as srv:
            # warm three slots per class (first-use allocation, table and
            # CFL step: tens of milliseconds once per slot), so that
            # overlapping requests of a class find a resident grid, as the
            # one-at-a-time form always does
            warm = [srv.submit(g, W.car_dynamics(), W.cylinders(70 + c, 3), 0.01)
                    for c, g in enumerate(W.SERVE_GRIDS) for _ in range(3)]
            while warm:
                srv.tick()
                for rid in srv.poll():
                    srv.take(rid)
                    warm.remove(rid)
            t0 = time.perf_counter()
            nxt = 0
            while done < n_req:
                now = time.perf_counter() - t0
                while nxt < n_req and reqs[nxt].arrival <= now:
                    r = reqs[nxt]
                    idmap[srv.submit(r.grid, r.dyn, r.cylinders, r.horizon)] = r.arrival
                    nxt += 1
                st = srv.stats()
                if st["running"] or st["queued"]:
                    srv.tick()
                for rid in srv.poll():
                    lat.append(time.perf_counter() - t0 - idmap.pop(rid))
                    srv.take(rid)
                    done += 1
                if not (st["running"] or st["queued"]) and nxt < n_req:
                    time.sleep(max(0.0, min(0.0005, reqs[nxt].arrival - (time.perf_counter() - t0))))
            wall = time.perf_counter() - t0
            stats = srv.stats()
        return np.array(lat) * 1e3, wall, stats

    def play_alone(reqs):
        grids = [hj.Grid(g, W.car_dynamics(), sch, "f32", stream) for g in W.SERVE_GRIDS]
        for c, g in enumerate(grids):
            g.set_autotune(False)
            g.set_target_cylinders(*W.cylinders(70 + c, 3))
            g.solve_brt(0.01)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for r in reqs:
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(0.0002)
            g = grids[r.cls]
            g.set_target_cylinders(*r.cylinders)
            g.solve_brt(r.horizon)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - r.arrival)
        wall = time.perf_counter() - t0
        for g in grids:
            g.close()
        return np.array(lat) * 1e3, wall

    # the played streams measure the library, not the interpreter: no
    # garbage-collector pauses inside them
    import gc

    gc.collect()
    gc.disable()
    reqs = W.serving_requests(n_req, rate=20.0)
    lat_s, wall_s, stats = play_server(reqs)
    lat_h, wall_h, _ = play_server(reqs, "share")
    lat_a, wall_a = play_alone(reqs)
    # the same stream compressed 6x (120 requests per second): one request
    # at a time then queues, the server batches
    fast = W.serving_requests(n_req, rate=120.0)
    lat_s6, wall_s6, _ = play_server(fast)
    lat_h6, wall_h6, _ = play_server(fast, "share")
    lat_a6, wall_a6 = play_alone(fast)
    gc.enable()
    steps = {0: None, 1: None}
    for c, g in enumerate(W.SERVE_GRIDS):
        with hj.Grid(g, W.car_dynamics(), sch, "f32", stream) as h:
            h.set_target_cylinders(*W.cylinders(70 + c, 3))
            steps[c] = h.solve_brt(1.5)["steps"]
    point_steps = sum(int(np.prod(r.grid["n"])) * steps[r.cls] for r in reqs)
    pct = lambda a, q: float(np.percentile(a, q))
    out = {
        "metric": METRIC, "value": point_steps / wall_s, "unit": UNIT, "n_gpus": 1, "steps": n_req, "warmup": 2,
        "ms_per_step": wall_s / n_req * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded Poisson re-solve stream)",
        "config": {
            "workload": "serving: Poisson 20 req/s, 70/30 mix of 60x60x20x36 (82 steps) and 100x100x24x48 (121 "
                        "steps), 1-3 obstacle changes per request, horizon 1.5 s, ENO2+TVD-RK2 FP32",
            "requests": n_req, "point_steps": point_steps, "hbm_budget": args.hbm_budget,
            "age_ms": args.age_ms or "library default (5)",
        },
        "latency_ms": {
            "server": {"p50": pct(lat_s, 50), "p99": pct(lat_s, 99), "max": float(lat_s.max())},
            "server_share": {"p50": pct(lat_h, 50), "p99": pct(lat_h, 99), "max": float(lat_h.max())},
            "one_at_a_time": {"p50": pct(lat_a, 50), "p99": pct(lat_a, 99), "max": float(lat_a.max())},
            "deadline_ms": 200.0,
            "server_within_deadline": float(np.mean(lat_s <= 200.0)),
        },
        "throughput": {"server_req_per_s": n_req / wall_s, "server_share_req_per_s": n_req / wall_h,
                       "one_at_a_time_req_per_s": n_req / wall_a},
        "stress_120_req_per_s": {
            "server": {"p50": pct(lat_s6, 50), "p99": pct(lat_s6, 99), "req_per_s": n_req / wall_s6},
            "server_share": {"p50": pct(lat_h6, 50), "p99": pct(lat_h6, 99), "req_per_s": n_req / wall_h6},
            "one_at_a_time": {"p50": pct(lat_a6, 50), "p99": pct(lat_a6, 99), "req_per_s": n_req / wall_a6},
        },
        "server_stats": stats,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_context(args) -> int:
    """The paper's own experiment shape beside its FPGA figure: the steering
    car of eq (6) on the 60x60x20x36 grid, first-order upwind + Euler, FP32,
    a BRT solve of 67 iterations (the paper's Table II count; the horizon is
    67 CFL steps of this grid).  GPU-event time per solve, the target already
    on the device.  The FPGA took 0.176 s for its 67 iterations."""
    import numpy as np
    import torch

    from paper_2012_04011_amd import hj
    from paper_2012_04011_amd import workloads as W

    hj.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    grid = W.car_grid(60, 60, 20, 36)
    sch = W.scheme("upwind1", "euler")
    with hj.Grid(grid, W.steer_dynamics(), sch, "f32", stream) as g:
        horizon = 67 * g.cfl_dt()
        sets = [W.cylinders(70 + s, 3) for s in range(args.warmup + args.steps)]
        for s in range(args.warmup):
            g.set_target_cylinders(*sets[s])
            info = g.solve_brt(horizon)
        lat = []
        for s in range(args.steps):
            g.set_target_cylinders(*sets[args.warmup + s])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            info = g.solve_brt(horizon)
            e1.record(stream)
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
        launch = g.launch_info()
    npts = int(np.prod(grid["n"]))
    med = float(np.median(lat))
    out = {
        "metric": "BRT solve latency, 67 iterations (context beside the paper's FPGA)", "value": med,
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": med,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded cylinder obstacles)",
        "config": {"workload": "paper shape: steering car (eq 6), 60x60x20x36, upwind + Euler FP32, 67 iterations",
                   "iterations": info["steps"], "dt": info["dt"], "stage_kernel": launch["kernel"],
                   "x_chunks": launch["x_chunks"]},
        "latency_ms": {"p50": med, "min": float(np.min(lat)), "max": float(np.max(lat))},
        "point_steps_per_s": npts * info["steps"] / (med / 1e3),
        "paper_fpga_s": 0.176,
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_adjacent(args) -> int:
    """The method's adjacent parts on the 120x120x40x72 grid, FP32, beside
    the fixed-horizon solve of the same grid (GPU-event time, the target on
    the device):
      converge     the convergence mode with a zero threshold, so that it runs
                   exactly the n steps of a 2 s solve: the cost of the
                   per-step stop test (eps = max |V_t+1 - V_t|, 8 B per node)
      alpha_range  Algorithm 1's derivative-range dissipation: a range pass
                   over V and a host round trip before every step
      control      the optimal-control query of eq (9) at 2^20 random states
                   on the device, and at one state from the host (latency)"""
    import numpy as np
    import torch

    from paper_2012_04011_amd import hj
    from paper_2012_04011_amd import workloads as W

    hj.load_library()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    wl = W.LARGE_120
    npts = wl.points
    cyl = W.cylinders(0, wl.obstacles)
    reps = max(1, args.steps)

    def timed(fn):
        fn()  # warm-up: autotune, graph capture, first allocations
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        return float(np.median(t))

    out = {"n_gpus": 1, "steps": reps, "warmup": 1, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded cylinder obstacles)"}
    if args.workload == "converge":
        with hj.Grid(wl.grid, wl.dyn, wl.scheme, "f32", stream) as g:
            g.set_target_cylinders(*cyl)
            n = g.solve_brt(wl.horizon)["steps"]
            short = (n - 0.5) * g.cfl_dt()  # n steps, the last one halved
            assert g.solve_brt(short)["steps"] == n
            plain = timed(lambda: g.solve_brt(short))
            info = {}

            def conv():
                info.update(g.solve_converge(0.0, n))

            conv_ms = timed(conv)
        assert info["steps"] == n and not info["converged"]
        extra_us = (conv_ms - plain) / n * 1e3
        out.update({
            "metric": "convergence-mode solve time (eps test every step)", "value": conv_ms, "unit": "ms",
            "ms_per_step": conv_ms / n, "higher_is_better": False,
            "config": {"workload": "car4d 120x120x40x72 ENO2+TVD-RK2 FP32, convergence mode, zero threshold "
                                   f"({n} steps, the 2 s solve's count)", "steps_per_solve": n},
            "fixed_horizon_ms": plain, "stop_test_us_per_step": extra_us,
            "stop_test_bytes_per_step": 8.0 * npts,
            "stop_test_gbs": 8.0 * npts / (extra_us * 1e3) if extra_us > 0 else None,
        })
    elif args.workload == "alpha_range":
        sch = dict(wl.scheme, alpha="deriv_range")
        with hj.Grid(wl.grid, wl.dyn, wl.scheme, "f32", stream) as g0:
            g0.set_target_cylinders(*cyl)
            dt0 = g0.cfl_dt()
            horizon = 20 * dt0
            n0 = g0.solve_brt(horizon)["steps"]
            plain = timed(lambda: g0.solve_brt(horizon))
        info = {}
        with hj.Grid(wl.grid, wl.dyn, sch, "f32", stream) as g:
            g.set_target_cylinders(*cyl)

            def solve():
                info.update(g.solve_brt(horizon))

            rng_ms = timed(solve)
        per = rng_ms / info["steps"]
        out.update({
            "metric": "derivative-range (Algorithm 1) solve time per step", "value": per, "unit": "ms",
            "ms_per_step": per, "higher_is_better": False,
            "config": {"workload": "car4d 120x120x40x72 ENO2+TVD-RK2 FP32, alpha from each step's derivative "
                                   f"range, horizon {horizon:.4f} s", "steps": info["steps"], "first_dt": info["dt"]},
            "state_alpha_ms_per_step": plain / n0, "state_alpha_steps": n0,
            "range_pass_us_per_step": (per - plain / n0) * 1e3,
        })
    elif args.workload == "control":
        m = 1 << 20
        rng = np.random.default_rng(7)
        lo, hi = np.array(wl.grid["lo"]), np.array(wl.grid["hi"])
        z = lo + (hi - lo) * rng.random((m, 4))
        with hj.Grid(wl.grid, wl.dyn, wl.scheme, "f32", stream) as g:
            g.set_target_cylinders(*cyl)
            g.solve_brt(wl.horizon)
            zd = torch.from_numpy(z).to("cuda")
            u = torch.empty((m, 2), dtype=torch.float64, device="cuda")
            val = torch.empty(m, dtype=torch.float64, device="cuda")
            dev_ms = timed(lambda: hj.hj_optimal_control(g.handle, zd, u, val))
            one = []
            for k in range(200):
                t0 = time.perf_counter()
                g.optimal_control(z[k:k + 1])
                one.append((time.perf_counter() - t0) * 1e3)
        out.update({
            "metric": "optimal-control queries/s (eq 9 at arbitrary states)", "value": m / (dev_ms / 1e3),
            "unit": "queries/s", "ms_per_step": dev_ms, "higher_is_better": True, "dtype": "f64",
            "config": {"workload": "car4d 120x120x40x72 FP32 V after a 2 s solve, 2^20 uniform random states, "
                                   "device arrays", "states": m},
            "host_single_query_ms": {"p50": float(np.percentile(one, 50)), "p99": float(np.percentile(one, 99))},
        })
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(wl, budget_s: float = 15.0, coarse=None) -> dict:
    """The FP64 oracle on the host cores: whole RK2 steps of the same
    workload from its seed-0 target, as many as fit the time budget.  With
    `coarse` (the 2x-coarsened companion workload) it also solves that grid
    whole from the same obstacles, timed, and returns its V under the key
    "_coarse_V" (the accuracy report compares the GPU's solves with it; the
    caller removes the key before printing)."""
    import numpy as np

    import oracle
    from paper_2012_04011_amd import workloads as W

    oracle.build(force=False)
    cx, cy, r = W.cylinders(0, wl.obstacles)
    V0 = oracle.target_cylinders(wl.grid, cx, cy, r)
    dt = oracle.cfl_dt(wl.grid, wl.dyn, wl.scheme["cfl"], wl.horizon)
    def sample(budget):
        V = V0.copy()
        steps, t0 = 0, time.perf_counter()
        while True:
            V = oracle.step(wl.grid, wl.dyn, wl.scheme, V0, V, dt)
            steps += 1
            el = time.perf_counter() - t0
            if el + el / steps > budget:
                return steps, el

    cores = oracle.threads()
    steps, el = sample(budget_s)
    # the same on one thread (at least one whole step)
    oracle.set_threads(1)
    try:
        steps1, el1 = sample(0.6 * budget_s)
    finally:
        oracle.set_threads(cores)
    coarse_out = {}
    if coarse is not None:
        V0c = oracle.target_cylinders(coarse.grid, cx, cy, r)
        t0 = time.perf_counter()
        Vc, ic = oracle.solve(coarse.grid, coarse.dyn, coarse.scheme, V0c, coarse.horizon)
        elc = time.perf_counter() - t0
        npc = int(np.prod(coarse.grid["n"]))
        gridc = "x".join(map(str, coarse.grid["n"]))
        coarse_out = {
            "value_coarse_solve": npc * ic["steps"] / elc,
            "sample_coarse_solve": f"the whole {ic['steps']}-step solve of the 2x-coarsened {gridc} grid "
                                   f"({npc * ic['steps'] / 1e6:.1f}M point-steps, {elc:.1f} s)",
            "_coarse_V": Vc,
        }
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    grid = "x".join(map(str, wl.grid["n"]))
    scheme = {"eno2": "ENO2", "upwind1": "upwind"}[wl.scheme["deriv"]] + "+" + \
        {"rk2": "TVD-RK2", "euler": "Euler"}[wl.scheme["integrator"]]
    return {
        "value": wl.points * steps / el,
        "unit": UNIT,
        "cores": cores,
        "kind": "oracle",
        "sample": f"{steps} full {scheme} FP64 step(s) of the {grid} grid "
                  f"({wl.points * steps / 1e6:.1f}M point-steps, {el:.1f} s)",
        "value_1_thread": wl.points * steps1 / el1,
        "sample_1_thread": f"{steps1} step(s) of the same grid on one thread ({el1:.1f} s)",
        "cpu_model": model,
        "nproc": os.cpu_count(),
        **coarse_out,
    }


def accuracy_gpu(wl, stream) -> tuple:
    """The precision report's GPU part (outside the timed loop): the seed-0
    solve of the workload in FP32 and in FP64 on the GPU, compared node by
    node (tol = 1e-4 min(dx, dy): band and all-node max, RMS, membership
    flips), and the FP64 solve of its 2x-coarsened companion.  Returns
    (report, V_fine_f64, V_coarse_f64)."""
    import numpy as np

    from paper_2012_04011_amd import accuracy, hj
    from paper_2012_04011_amd import workloads as W

    cyl = W.cylinders(0, wl.obstacles)
    out = {}
    for prec in ("f32", "f64"):
        with hj.Grid(wl.grid, wl.dyn, wl.scheme, prec, stream) as g:
            g.set_target_cylinders(*cyl)
            g.solve_brt(wl.horizon)
            out[prec] = g.value(np.float32 if prec == "f32" else np.float64)
    wc = W.LARGE_120_COARSE
    with hj.Grid(wc.grid, wc.dyn, wc.scheme, "f64", stream) as g:
        g.set_target_cylinders(*cyl)
        g.solve_brt(wc.horizon)
        Vc = g.value(np.float64)
    m = accuracy.precision_metrics(out["f32"], out["f64"], wl.grid)
    m["within_tol"] = bool(m["max_band"] <= m["tol"] and m["rms"] <= m["tol"] and m["flips_outside"] == 0)
    rep = {"fp32_vs_fp64_gpu": m,
           "note": "seed-0 solves; tol = 1e-4 min(dx, dy) over the band |V| <= 1, RMS over all nodes, flips farther "
                   "than tol from the zero level set"}
    return rep, out["f64"], Vc


def accuracy_small(wl, stream) -> dict:
    """A grid the oracle solves whole in seconds: the seed-0 solve in FP32
    and FP64 on the GPU against the oracle's solve (FP32: tol = 1e-4
    min(dx, dy) over the band, RMS, membership flips; FP64: the largest
    difference)."""
    import numpy as np

    import oracle
    from paper_2012_04011_amd import accuracy, hj
    from paper_2012_04011_amd import workloads as W

    cyl = W.cylinders(0, wl.obstacles)
    V0 = oracle.target_cylinders(wl.grid, *cyl)
    ref, _ = oracle.solve(wl.grid, wl.dyn, wl.scheme, V0, wl.horizon)
    out = {}
    for prec in ("f32", "f64"):
        with hj.Grid(wl.grid, wl.dyn, wl.scheme, prec, stream) as g:
            g.set_target_cylinders(*cyl)
            g.solve_brt(wl.horizon)
            out[prec] = g.value(np.float64)
    m = accuracy.precision_metrics(out["f32"], ref, wl.grid)
    m["within_tol"] = bool(m["max_band"] <= m["tol"] and m["rms"] <= m["tol"] and m["flips_outside"] == 0)
    return {"fp32_gpu_vs_oracle": m, "fp64_gpu_vs_oracle": {"max_abs": float(np.abs(out["f64"] - ref).max())},
            "note": "seed-0 solves against the FP64 oracle; tol = 1e-4 min(dx, dy) over the band |V| <= 1, RMS over "
                    "all nodes, flips farther than tol from the zero level set"}


def accuracy_oracle(rep, wl, V64, Vc_gpu, Vc_oracle) -> None:
    """The precision report's oracle part: the coarse FP64 GPU solve against
    the coarse oracle solve (parity), and the fine FP64 GPU solve sampled
    multilinearly at the coarse nodes against the coarse oracle solve
    (consistency of the two resolutions; flips counted where |V| > 2 dx)."""
    import numpy as np

    from paper_2012_04011_amd import accuracy
    from paper_2012_04011_amd import workloads as W

    rep["fp64_gpu_vs_oracle_coarse"] = {"max_abs": float(np.abs(Vc_gpu - Vc_oracle).max())}
    rep["fine_fp64_gpu_vs_coarse_oracle"] = accuracy.consistency_metrics(V64, wl.grid, Vc_oracle,
                                                                         W.LARGE_120_COARSE.grid)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--workload", choices=["large120", "eno60", "batch64", "serve", "context", "converge",
                                           "alpha_range", "control"], default="large120")
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32",
                    help="large120: arithmetic of the solve (the headline is FP32)")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests in the stream")
    ap.add_argument("--hbm-budget", type=int, default=8 << 30, help="serve: slot memory budget in bytes")
    ap.add_argument("--age-ms", type=float, default=0.0,
                    help="serve: small-first age limit in ms after which requests go first (0: the library's)")
    ap.add_argument("--summarize-traffic", metavar="DIR")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="large120: skip the precision report (FP32 vs FP64 GPU solves, coarse-grid comparison)")
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
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload in ("converge", "alpha_range", "control"):
        return bench_adjacent(args)
    if args.workload == "context":
        return bench_context(args)
    hj.load_library()
    torch.cuda.set_device(0)
    wl = W.ENO_60_DIST if args.workload == "eno60" else W.LARGE_120
    prec = args.precision
    stream = torch.cuda.current_stream()
    g = hj.Grid(wl.grid, wl.dyn, wl.scheme, prec, stream)
    npts = g.num_points
    obstacle_sets = [W.cylinders(s, wl.obstacles) for s in range(args.warmup + args.steps)]

    info = None
    for s in range(args.warmup):
        g.set_target_cylinders(*obstacle_sets[s])
        info = g.solve_brt(wl.horizon)
    torch.cuda.synchronize()

    g.set_profiling(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    import gc

    gc.collect()
    gc.disable()  # no interpreter pauses while the timed solves are enqueued
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        g.set_target_cylinders(*obstacle_sets[args.warmup + s])
        info = g.solve_brt(wl.horizon)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    prof = g.profile()
    launch = g.launch_info()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    g.close()

    steps_per_solve = info["steps"]
    value = npts * steps_per_solve * args.steps / wall
    bpl = algorithmic_bytes_per_launch(npts, launch, wl.scheme["integrator"])
    avg_launch_s = prof["loop_ms"] / 1e3 / prof["step_launches"]
    achieved = bpl / avg_launch_s / 1e9
    traffic = measured_traffic(npts, launch["x_chunks"], launch["plane_rows"]) if prec == "f32" else None
    copy_gbs = copy_bandwidth_gbs(stream)
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
        "dtype": prec,
        "data": "synthetic (seeded cylinder obstacles)",
        "config": {
            "workload": (f"car4d 120x120x40x72 (41.5M points) ENO2+TVD-RK2 {prec.upper()}, horizon 2 s, 8 cylinders"
                         if wl is W.LARGE_120 else
                         f"car4d 60x60x20x36 (2.6M points, the paper's grid) ENO2+TVD-RK2 {prec.upper()}, "
                         "disturbance |d| <= 0.1, horizon 2 s, 5 cylinders"),
            "grid": list(wl.grid["n"]),
            "points": npts,
            "scheme": "eno2+rk2",
            "horizon_s": wl.horizon,
            "steps_per_solve": steps_per_solve,
            "dt": info["dt"],
            "obstacles": wl.obstacles,
            "stage_kernel": launch["kernel"],
            "x_chunks": launch["x_chunks"],
            "plane_rows": launch["plane_rows"],
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
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "solve_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "min": float(lat.min())},
    }
    if wl is not W.LARGE_120:
        # a 2.6M-node grid's arrays (10.4 MB each in FP32) fit in the 256 MB
        # Infinity Cache (MALL), so its stages need not stream from HBM: the
        # fraction of 8 TB/s is a rate, not a proof of an HBM bound
        out["roofline"]["cache_note"] = ("all arrays of a stage (about 31 MB) fit in the 256 MB Infinity Cache; "
                                         "the HBM fraction is a rate on algorithmic bytes")
        if not args.no_accuracy:
            out["accuracy"] = accuracy_small(wl, stream)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        print(json.dumps(out), flush=True)
        return 0
    acc = None
    if prec == "f32" and not args.no_accuracy:
        acc, V64, Vc_gpu = accuracy_gpu(wl, stream)
        out["accuracy"] = acc
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, args.cpu_budget, W.LARGE_120_COARSE if acc is not None else None)
        Vc_oracle = cb.pop("_coarse_V", None)
        if acc is not None and Vc_oracle is not None:
            accuracy_oracle(acc, wl, V64, Vc_gpu, Vc_oracle)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
