"""Host logic of bench.py (no GPU): the one-GPU guard, the byte model and
the traffic bookkeeping that turns rocprofv3 FETCH_SIZE / WRITE_SIZE counters
into HBM bytes per launch."""

from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2012_04011_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_launch():
    n = 1000
    # TVD-RK2 with the cylinder table: 20 B per point-step over two launches
    assert bench.algorithmic_bytes_per_launch(n, {"bytes_per_point_step": 20.0}, "rk2") == 10.0 * n
    # Euler with a 4D target: one launch moves the whole step
    assert bench.algorithmic_bytes_per_launch(n, {"bytes_per_point_step": 12.0}, "euler") == 12.0 * n


def _write_counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, k, c, v in rows:
            f.write(f'{d},"{k}",{c},{v}\n')


def _fake_profile(root, chunks=(2, 2), stage_kib=((100.0, 200.0), (50.0, 50.0)), copy_kib=(262144.0, 524288.0)):
    """Counter runs as rocprofv3 writes them: 200 alternating stage
    dispatches (stage 1, stage 2) after a warm-up, the copy calibration, and
    the JSON line each counted benchmark run printed."""
    kern = "void hj::stage_plane<float, 4, 1, false, false, false>(hj::StreamArgs<float>)"
    for i, (counter, key) in enumerate((("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))):
        s1, s2 = stage_kib[i]
        rows = [(d, kern, counter, 999.0) for d in range(10)]  # warm-up launches, not in the last 200
        rows += [(10 + d, kern, counter, s1 if d % 2 == 0 else s2) for d in range(200)]
        _write_counter_csv(os.path.join(root, f"stage_{key}", "run_counter_collection.csv"), rows)
        _write_counter_csv(os.path.join(root, f"copy_{key}", "run_counter_collection.csv"),
                           [(d, "__amd_rocclr_copyBuffer", counter, copy_kib[i]) for d in range(5)])
        with open(os.path.join(root, f"stage_{key}.log"), "w") as f:
            f.write("some profiler output\n")
            f.write(json.dumps({"metric": "m", "config": {"x_chunks": chunks[i], "plane_rows": 2}}) + "\n")


def test_summarize_traffic_calibration(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    _fake_profile(str(tmp_path))
    assert bench.summarize_traffic(str(tmp_path)) == 0
    t = json.loads(out.read_text())
    copy = bench.COPY_MIB * 2**20
    f_factor, w_factor = copy / (262144.0 * 1024), copy / (524288.0 * 1024)
    assert t["fetch"]["factor"] == pytest.approx(f_factor) and t["write"]["factor"] == pytest.approx(w_factor)
    s1 = (100.0 * f_factor + 50.0 * w_factor) * 1024
    s2 = (200.0 * f_factor + 50.0 * w_factor) * 1024
    assert t["stage1_bytes"] == pytest.approx(s1) and t["stage2_bytes"] == pytest.approx(s2)
    assert t["bytes_per_launch"] == pytest.approx((s1 + s2) / 2)
    assert t["x_chunks"] == 2 and t["plane_rows"] == 2 and t["points"] == W.LARGE_120.points
    assert t["kernel_source_sha256_16"] == bench.kernel_source_hash()
    # the benchmark uses it only for the same kernels, size, chunking and rows per block
    assert bench.measured_traffic(W.LARGE_120.points, 2, 2) == pytest.approx((s1 + s2) / 2)
    assert bench.measured_traffic(W.LARGE_120.points, 2, 1) is None
    assert bench.measured_traffic(W.LARGE_120.points, 4, 2) is None
    assert bench.measured_traffic(W.LARGE_120.points + 1, 2, 2) is None
    t["kernel_source_sha256_16"] = "0" * 16
    out.write_text(json.dumps(t))
    assert bench.measured_traffic(W.LARGE_120.points, 2, 2) is None


def test_summarize_traffic_refuses_mixed_configurations(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    _fake_profile(str(tmp_path), chunks=(4, 6))
    assert bench.summarize_traffic(str(tmp_path)) == 1
    assert not out.exists()


def test_committed_traffic_matches_committed_kernels():
    """The traffic figures under profiles/ were taken on the kernel source in
    this tree (else the benchmark would report traffic as null)."""
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["kernel_source_sha256_16"] == bench.kernel_source_hash()
    assert t["points"] == W.LARGE_120.points and t["x_chunks"] == 2
    assert 1.0 <= t["bytes_per_launch"] / (20.0 * W.LARGE_120.points / 2) < 1.2
