"""Benchmark of the MCT-2D-CEM explicit fracture step on one MI355X.

Workload: the 400x400 Q4 mesh of the 100 x 40 mm branching plate
(0.25 x 0.1 mm elements, +/-1% seeded nodal jitter, half-length edge notch,
1 MPa traction on the upper and lower edges), binary64, synthetic inputs.
A bench "step" is one explicit time step: edge stresses, element forces,
coloured scatter, central-difference update, G of every free-surface
candidate, and the multi-tip pick and split.

Timed region: --steps time steps from t = 0 (the state is restored after the
warm-up), inputs resident in HBM, bracketed by device synchronisation.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOADS = {
    "plate400": "branching plate 400x400 Q4, 100x40 mm, jitter 1%, notch 50 mm, 1 MPa",
    "fragment2000": "fragmentation plate 2000x1000 Q4, h 0.1 mm, 5 m/s outward, Weibull(6,3) Gc",
}


def bytes_per_step(nx: int, ny: int) -> int:
    """Algorithmic HBM bytes of one fused step (binary64): per node read u,
    v, X, Y, 1/m and write u, v (11 doubles); per element its split code."""
    nn = (nx + 1) * (ny + 1)
    ne = nx * ny
    return 88 * nn + ne


def cpu_baseline(cfg, steps: int):
    from oracle import oracle
    o = oracle.Oracle(cfg)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    ne = cfg["nx"] * cfg["ny"]
    return {"value": ne * steps / dt, "unit": "element-updates/s", "cores": 1, "kind": "oracle",
            "sample": "first %d time steps of the same 400x400 plate (single-threaded C oracle, %.1f s)"
                      % (steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="plate400", choices=["plate400", "fragment2000"],
                    help="plate400: the 400x400 branching plate (default); fragment2000: the "
                         "2000x1000 Dirichlet fragmentation plate")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (three times), "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 8 * n, "repeats": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_01827_amd import mct2d, workloads as W

    torch.cuda.set_device(0)
    cfg = W.config2() if args.workload == "plate400" else W.config3()
    nx, ny = cfg["nx"], cfg["ny"]
    ne = nx * ny
    stream = torch.cuda.Stream()
    m = mct2d.from_config(cfg, stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
    init = m.checkpoint()
    m.step(args.warmup)
    m.sync()
    m.restore(init)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    m.step(args.steps)
    ev1.record(stream)
    m.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    info = m.info()
    assert info["step"] == args.steps

    ms_per_step = gpu_ms / args.steps
    value = ne * args.steps / (gpu_ms * 1e-3)
    bps = bytes_per_step(nx, ny)
    achieved = bps / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "element-updates/s",
        "value": value,
        "unit": "element-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "elements": ne, "nodes": (nx + 1) * (ny + 1), "time_steps": args.steps,
                   "tile": args.tile, "graph": not args.no_graph},
        "wall_s": wall,
        "splits": info["n_splits"],
        "dissipated_J_per_m": info["dissipated"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bps},
    }
    m.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
