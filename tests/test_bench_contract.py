"""bench.py's output contract: one JSON line with the metric, the roofline
object (traffic from the measured counters while the kernel code matches
them) and the CPU baseline; a request for more than one GPU is refused.
The GPU test runs a short plate400 bench; the CPU tests need no device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_matches_the_current_kernels():
    """Every stored counter figure was taken on the kernel code as it is
    (else bench.py would report the traffic as unknown)."""
    sys.path.insert(0, ROOT)
    import bench
    for w, rec in bench.MEASURED_TRAFFIC.items():
        assert bench.kernel_sha256(rec["sources"]) == rec["sha256"], w
        t = bench.measured_traffic(w, rec["tile"])
        assert t is not None and t > 0, w


def _check_line(d, steps, workload):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["dtype"] == "f64" and d["value"] > 0
    assert d["config"]["name"] == workload and "workload" in d["config"]
    ne = d["config"]["elements"]
    assert d["value"] == pytest.approx(ne * steps / (d["ms_per_step"] * steps * 1e-3), rel=1e-9)
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    # achieved bandwidth from the timed window's time per step; the step
    # kernel alone, timed per launch after the window, is of the same order
    kt = d["kernel_timing"]
    assert rf["kernel_us"] == pytest.approx(d["ms_per_step"] * 1e3)
    assert rf["achieved"] == pytest.approx(rf["bytes_per_launch"] / (d["ms_per_step"] * 1e-3) / 1e9)
    assert 0.3 * rf["kernel_us"] < kt["step_kernel_us"] < 3.0 * rf["kernel_us"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0


@pytest.mark.gpu
def test_bench_json_line():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _bench("--workload", "plate400", "--start", "100", "--steps", "300", "--warmup", "20", "--cpu-seconds", "1")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    _check_line(d, 300, "plate400")
    assert d["config"]["window"] == [120, 420] and not d["config"]["lattice"]


@pytest.mark.gpu
def test_bench_default_batch_line():
    """The default workload (the 256-specimen batch) from a mid-run state,
    on the lattice kernel, with the per-specimen plain comparison."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _bench("--start", "300", "--steps", "40", "--warmup", "8", "--cpu-seconds", "2", timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    _check_line(d, 40, "batch256")
    assert d["config"]["specimens"] == 256 and d["config"]["lattice"] and d["config"]["graph"]
    bp = d["batched_vs_plain"]
    assert bp["identical_crack_sets"] and bp["speedup"] > 1.0
    assert "specimen-parallel" in d["cpu_baseline"]["sample"]


def test_algorithmic_bytes_per_mesh_kind():
    """bytes_per_step: per node 72 B (u, v, 1/m read; u, v written) plus 16 B
    of X, Y unless the grid is a uniform lattice; per element 1 B (split
    code), 8 B more with a Gc field, 12 B (triangle) or 16 B (quadrilateral)
    of node ids on an unstructured mesh; binary32 halves the floating-point
    part."""
    sys.path.insert(0, ROOT)
    import bench
    import numpy as np
    grid = {"nx": 4, "ny": 3, "X": np.zeros(20)}
    gcg = {"nx": 4, "ny": 3, "X": np.zeros(20), "gc_field": np.ones(12)}
    tri = {"conn": np.zeros((7, 3), np.int32), "X": np.zeros(9)}
    quad = {"conn": np.zeros((5, 4), np.int32), "X": np.zeros(11)}
    assert bench.bytes_per_step([grid]) == 88 * 20 + 1 * 12
    assert bench.bytes_per_step([grid], lattice=True) == 72 * 20 + 1 * 12
    assert bench.bytes_per_step([gcg], lattice=True) == 72 * 20 + 9 * 12
    assert bench.bytes_per_step([grid], precision=32) == 44 * 20 + 1 * 12
    assert bench.bytes_per_step([tri]) == 88 * 9 + 13 * 7
    assert bench.bytes_per_step([quad]) == 88 * 11 + 17 * 5
    assert bench.bytes_per_step([grid, tri]) == 88 * 29 + 1 * 12 + 13 * 7
    # the batch of 256 specimens: 81 B per element-update on the lattice
    cfgs = [{"nx": 300, "ny": 200, "X": np.zeros(301 * 201), "gc_field": np.ones(60000)}]
    assert bench.bytes_per_step(cfgs, lattice=True) / 60000 == pytest.approx(81.0, rel=0.02)
