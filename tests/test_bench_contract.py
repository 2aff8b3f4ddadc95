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


@pytest.mark.gpu
def test_bench_json_line():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = _bench("--steps", "300", "--warmup", "20", "--cpu-seconds", "1")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 300 and d["dtype"] == "f64" and d["value"] > 0
    assert d["value"] == pytest.approx(160000 * 300 / (d["ms_per_step"] * 300 * 1e-3), rel=1e-9)
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert rf["traffic"] is not None and rf["traffic"] > rf["bytes_per_launch"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert "workload" in d["config"]


def test_algorithmic_bytes_per_mesh_kind():
    """bytes_per_step: 88 B per node (u, v, X, Y, 1/m read; u, v written) plus
    per element 9 B on the structured grid (split code, area), 13 B for a
    triangle and 17 B for a quadrilateral of an unstructured mesh (split code,
    node ids); binary32 halves the floating-point part."""
    sys.path.insert(0, ROOT)
    import bench
    import numpy as np
    grid = {"nx": 4, "ny": 3, "X": np.zeros(20)}
    tri = {"conn": np.zeros((7, 3), np.int32), "X": np.zeros(9)}
    quad = {"conn": np.zeros((5, 4), np.int32), "X": np.zeros(11)}
    assert bench.bytes_per_step([grid]) == 88 * 20 + 9 * 12
    assert bench.bytes_per_step([grid], precision=32) == 44 * 20 + 5 * 12
    assert bench.bytes_per_step([tri]) == 88 * 9 + 13 * 7
    assert bench.bytes_per_step([quad]) == 88 * 11 + 17 * 5
    assert bench.bytes_per_step([grid, tri]) == 88 * 29 + 9 * 12 + 13 * 7
