"""Benchmark of the MCT-2D-CEM explicit fracture step on one MI355X.

Default workload: the 400x400 Q4 mesh of the 100 x 40 mm branching plate
(0.25 x 0.1 mm elements, +/-1% seeded nodal jitter, half-length edge notch,
1 MPa traction on the upper and lower edges), binary64, synthetic inputs.
A bench "step" is one explicit time step: edge stresses, element forces,
coloured scatter, central-difference update, G of every free-surface
candidate, and the multi-tip pick and split.

Timed region: --steps time steps from t = 0 (the state is restored after the
warm-up), inputs resident in HBM, bracketed by device synchronisation.
Prints one JSON line.

Other workloads (--workload): fragment2000 (2000 x 1000 fragmentation plate)
and batch256 (256 uneven notched specimens in one launch per step; with
--compare-plain every specimen is also run alone with the plain step and the
crack sets are compared).
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
    "batch256": "256 notched specimens 64..512 x 64..256 Q4, h 1 mm, notch U(0.2,0.6) width, "
                "Weibull(6, U(2,4)) Gc, traction U(0.5,1.5) MPa",
    "screen400": "branching plate 400x400 Q4 (as plate400) with the learned split-screen, exact step every 50",
    "tri320k": "branching plate 100x40 mm on an unstructured CST mesh (Delaunay of 633x254 jittered points, "
               "319792 triangles), notch 50 mm, 1 MPa",
    "cylinder53k": "pressured hollow cylinder r 50/100 mm on an unstructured CST mesh (h 1 mm, ~53000 triangles), "
                   "steel, 400 MPa pulse",
    "quad160k": "branching plate 100x40 mm on an unstructured Q4 mesh (each Delaunay triangle of 259x104 "
                "jittered points split into 3 quadrilaterals, ~160000 elements), notch 50 mm, 1 MPa",
}


def n_elems(c) -> int:
    return len(c["conn"]) if c.get("conn") is not None else c["nx"] * c["ny"]


def n_nodes(c) -> int:
    return len(c["X"])


def bytes_per_step(cfgs, precision: int = 64) -> int:
    """Algorithmic HBM bytes of one step: per node read u, v, X, Y, 1/m and
    write u, v (11 values: 88 bytes in binary64, 44 in binary32); per Q4
    element its split code and its area (9 bytes, 5 in binary32; the
    structured grid needs no connectivity); per element of an unstructured
    mesh its split code and its node ids (13 bytes for a triangle, 17 for a
    quadrilateral)."""
    w = 8 if precision == 64 else 4
    total = 0
    for c in cfgs:
        if c.get("conn") is not None:
            per_elem = 1 + 4 * len(c["conn"][0])
        else:
            per_elem = 1 + w
        total += 11 * w * n_nodes(c) + per_elem * n_elems(c)
    return total


# HBM bytes per time step measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, averaged over the profiled launches and summed
# over the step's kernels), each scaled by the ratio of true to counted bytes
# of a 256 MiB device copy (FETCH_SIZE x 1.99979, WRITE_SIZE x 1.0).  A figure
# holds for the kernel sources it was taken on (their hash) and the tile
# shape; otherwise the traffic is reported as unknown.
Q4_SOURCES = ("mct2d_step.hip", "mct2d_impl.h", "mct2d_device.h")
TRI_SOURCES = ("mct2d_tri.hip", "mct2d_tri.h", "mct2d_front.h", "mct2d_device.h", "mct2d_impl.h")
MEASURED_TRAFFIC = {
    "plate400": {"sources": Q4_SOURCES, "sha256": "a6140c37bbd33d5cff0a1091d3cdfe767eaf756c679d596bb8c541efb07f717e",
                 "tile": 1, "fetch_kib": 5589.8934375, "write_kib": 5044.40625},
    "plate400_f32": {"sources": Q4_SOURCES, "sha256": "a6140c37bbd33d5cff0a1091d3cdfe767eaf756c679d596bb8c541efb07f717e",
                     "tile": 1, "fetch_kib": 2959.135, "write_kib": 2534.78125},
    "batch256": {"sources": Q4_SOURCES, "sha256": "a6140c37bbd33d5cff0a1091d3cdfe767eaf756c679d596bb8c541efb07f717e",
                 "tile": 1, "fetch_kib": 423857.846875, "write_kib": 486074.4453125},
    # two launches per step: k_force (15 006.17 / 14 990.25) + k_node (17 014.01 / 5 024.44)
    "tri320k": {"sources": TRI_SOURCES, "sha256": "9991853dfaedba4f0b5c1afc6731b7505f9e3ec19df83254745b697753d12dde",
                "tile": 1, "fetch_kib": 32020.18375, "write_kib": 20014.6875},
    # one launch per step: k_fused on 64-node patches (the commit, once per 64 steps, is negligible)
    "cylinder53k": {"sources": TRI_SOURCES, "sha256": "9991853dfaedba4f0b5c1afc6731b7505f9e3ec19df83254745b697753d12dde",
                    "tile": 2, "fetch_kib": 5302.3446875, "write_kib": 868.84375},
    # two launches per step: k_qforce (10 982.15 / 9 974.60) + k_node (12 405.03 / 5 005.25)
    "quad160k": {"sources": TRI_SOURCES, "sha256": "9991853dfaedba4f0b5c1afc6731b7505f9e3ec19df83254745b697753d12dde",
                 "tile": 1, "fetch_kib": 23387.1796875, "write_kib": 14979.84984375},
}
FETCH_SCALE, WRITE_SCALE = 262144.0 / 131086.604, 262144.0 / 262144.0


def kernel_sha256(sources) -> str:
    """Hash of the kernel sources' code: comments and blank lines are left
    out, so editing a comment keeps a measurement valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2509_01827_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()


def measured_traffic(workload: str, tile: int):
    rec = MEASURED_TRAFFIC.get(workload)
    if rec is None or rec["fetch_kib"] is None or rec["tile"] != tile or \
            kernel_sha256(rec["sources"]) != rec["sha256"]:
        return None
    return 1024.0 * (rec["fetch_kib"] * FETCH_SCALE + rec["write_kib"] * WRITE_SCALE)


def _oracle_rate(cfg, seconds: float, threads: int):
    """Element-updates/s of the oracle with `threads` OpenMP threads on the
    first time steps of the workload: chunks of 10 steps until `seconds`."""
    from oracle import oracle
    oracle.set_threads(threads)
    o = oracle.Oracle(cfg)  # the binary32 build for a binary32 workload
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds and steps < cfg["steps"]:
        o.step(10)
        steps += 10
    dt = time.perf_counter() - t0
    return n_elems(cfg) * steps / dt, steps, dt


def cpu_baseline(cfg, seconds: float):
    """The oracle on the host's cores (its OpenMP loops, results independent
    of the thread count), and single-threaded beside it, each on a bounded
    sample of the workload's first time steps."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)), 16))
    rate, steps, dt = _oracle_rate(cfg, seconds, cores)
    rate1, steps1, dt1 = _oracle_rate(cfg, seconds, 1)
    ne = n_elems(cfg)
    return {"value": rate, "unit": "element-updates/s", "cores": cores, "kind": "oracle",
            "sample": "first %d time steps of the same %s (%d elements; C oracle, binary%d, %d threads, %.1f s)"
                      % (steps, cfg["name"], ne, int(cfg.get("precision", 64)), cores, dt),
            "single_thread": {"value": rate1, "cores": 1,
                              "sample": "first %d time steps, 1 thread, %.1f s" % (steps1, dt1)}}


def timed_run(m, stream, steps, warmup):
    """Warm up, restore the initial state, time `steps` steps with HIP events
    on the model's stream.  Returns (gpu_ms, wall_s)."""
    import torch
    init = m.checkpoint()
    if warmup:
        m.step(warmup)
        m.sync()
    m.restore(init)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    m.step(steps)
    ev1.record(stream)
    m.sync()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="time steps timed (default: the workload's full run)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="pick tile/order by measurement first")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU-baseline sample: oracle steps from t = 0 for about this long")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="plate400", choices=sorted(WORKLOADS))
    ap.add_argument("--smoothing", default="point", choices=("point", "subcell"),
                    help="Q4 edge smoothing (plain Q4 workloads)")
    ap.add_argument("--front-radius", type=float, default=0.0,
                    help="per-front pick with this competition radius in m (plain workloads; 0: global pick)")
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32),
                    help="32: the binary32 step (plate400 and fragment2000)")
    ap.add_argument("--compare-plain", action="store_true",
                    help="batch256: also run each specimen alone and compare")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="only print the source hashes the measured traffic figures are keyed on")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (three times), "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.kernel_hash:
        print(json.dumps({w: kernel_sha256(r["sources"]) for w, r in MEASURED_TRAFFIC.items()}))
        return
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

    import numpy as np
    import torch
    from paper_2509_01827_amd import mct2d, workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    screen = None
    if args.workload == "batch256":
        cfgs = W.batch_specimens()
        m = mct2d.batch_from_configs(cfgs, stream=stream.cuda_stream, tile=args.tile,
                                     use_graph=not args.no_graph)
    elif args.workload == "screen400":
        cfgs = [W.config2()]
        with open(os.path.join(ROOT, "paper_2509_01827_amd", "screen_weights.json")) as f:
            screen = json.load(f)
        mlp = mct2d.Mlp()
        mlp.set_params(np.asarray(screen["params"], np.float32))
        m = mct2d.from_config(cfgs[0], stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
        m.screen_enable(mlp, screen["tau"], screen["period"])
    else:
        cfgs = [{"plate400": W.config2, "fragment2000": W.config3, "tri320k": W.tri_plate320k,
                 "cylinder53k": lambda: W.tri_cylinder(steps=2000, name="cylinder53k"),
                 "quad160k": W.quad_plate160k}[args.workload]()]
        if args.smoothing != "point":
            cfgs[0]["smoothing"] = args.smoothing
        if args.front_radius > 0:
            cfgs[0]["front_radius"] = args.front_radius
        if args.precision == 32:
            if args.workload not in ("plate400", "fragment2000"):
                print("--precision 32 is for the Q4 workloads plate400 and fragment2000", file=sys.stderr)
                sys.exit(2)
            cfgs[0]["precision"] = 32
        m = mct2d.from_config(cfgs[0], stream=stream.cuda_stream, tile=args.tile,
                              use_graph=not args.no_graph)
    steps = args.steps if args.steps is not None else cfgs[0]["steps"]
    tune = m.autotune(trial_steps=20) if args.autotune else None
    gpu_ms, wall = timed_run(m, stream, steps, args.warmup)
    launch = m.launch()
    ne = sum(n_elems(c) for c in cfgs)
    splits, ud = 0, 0.0
    logs = []
    for s in range(len(cfgs)):
        if len(cfgs) > 1:
            m.select(s)
        inf = m.info()
        assert inf["step"] == steps
        splits += inf["n_splits"]
        ud += inf["dissipated"]
        if args.compare_plain or screen:
            logs.append(m.crack_set())
    screen_stats = m.screen_stats() if screen else None
    ms_per_step = gpu_ms / steps
    value = ne * steps / (gpu_ms * 1e-3)
    bps = bytes_per_step(cfgs, args.precision)
    traffic_key = args.workload + ("_f32" if args.precision == 32 else "")
    achieved = bps / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "element-updates/s",
        "value": value,
        "unit": "element-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "specimens": len(cfgs), "elements": ne,
                   "time_steps": steps, "tile": launch["tile"], "order": launch["order"],
                   "workgroups": launch["workgroups"], "graph": not args.no_graph,
                   "smoothing": args.smoothing, "front_radius": args.front_radius, "precision": args.precision,
                   "autotuned": tune is not None},
        "wall_s": wall,
        "splits": splits,
        "dissipated_J_per_m": ud,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(traffic_key, launch["tile"]), "bytes_per_launch": bps},
    }
    m.close()
    if screen:
        p = mct2d.from_config(cfgs[0], stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
        ms, _ = timed_run(p, stream, steps, args.warmup)
        lg = p.crack_set()
        same = all(np.array_equal(lg[k], logs[0][k]) for k in ("step", "elem", "entry", "exit", "G"))
        p.close()
        out["screened_vs_plain"] = {"speedup": ms / gpu_ms, "plain_ms": ms, "screened_ms": gpu_ms,
                                    "identical_crack_sets": bool(same), "tau": screen["tau"],
                                    "period": screen["period"], "stats": screen_stats}
    if args.compare_plain and len(cfgs) > 1:
        plain_ms = 0.0
        same = True
        for s, cfg in enumerate(cfgs):
            p = mct2d.from_config(cfg, stream=stream.cuda_stream)
            ms, _ = timed_run(p, stream, steps, 0)
            plain_ms += ms
            lg = p.crack_set()
            same = same and all(np.array_equal(lg[k], logs[s][k]) for k in ("step", "elem", "entry", "exit", "G"))
            p.close()
        out["batched_vs_plain"] = {"speedup": plain_ms / gpu_ms, "plain_ms_total": plain_ms,
                                   "batched_ms": gpu_ms, "identical_crack_sets": bool(same)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfgs[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
