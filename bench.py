"""Benchmark of the MCT-2D-CEM explicit fracture step on one MI355X.

Default workload: the batched form, 256 independent notched specimens of
uneven size (64..512 x 64..256 Q4 elements of side 2^-10 m, notch
U(0.2, 0.6) of the width, Weibull(6, U(2, 4) N/m) Gc, traction
U(0.5, 1.5) MPa; 12.8 M elements), binary64, synthetic inputs, one step
launch over all their tiles per time step.  A bench "step" is one explicit
time step of every specimen: edge stresses, element forces, coloured
scatter, central-difference update, G of every free-surface candidate, and
the multi-tip pick and split.

Timed region: the state is advanced untimed from t = 0 to step --start
(default 2500, mid-run: cracks growing, candidates live), then --warmup
untimed steps, then exactly --steps steps (captured graphs) bracketed by
device synchronisation and HIP events on the model's stream; inputs
resident in HBM.  The roofline divides the algorithmic bytes of one step by
that window's time per step (the step kernel plus the per-step pick commit
of a batch), so it is a lower bound of the step kernel's own rate.  As a
cross-check the step kernel alone is then timed with HIP events around each
launch (mct_profile_step, direct launches) over the next steps.  Prints one
JSON line.

Other workloads (--workload): plate400 (400 x 400 jittered branching
plate), fragment2000 (2000 x 1000 fragmentation plate), screen400 (plate400
with the learned split-screen), tri320k / cylinder53k (CST meshes),
quad160k (unstructured Q4).
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
    "batch256": "256 notched specimens 64..512 x 64..256 Q4, h 2^-10 m, notch U(0.2,0.6) width, "
                "Weibull(6, U(2,4)) Gc, traction U(0.5,1.5) MPa",
    "plate400": "branching plate 400x400 Q4, 100x40 mm, jitter 1%, notch 50 mm, 1 MPa",
    "fragment2000": "fragmentation plate 2000x1000 Q4, h 2^-13 m, 5 m/s outward, Weibull(6,3) Gc",
    "screen400": "branching plate 400x400 Q4 (as plate400) with the learned split-screen, exact step every 50",
    "screen2000": "fragmentation plate 2000x1000 Q4 (as fragment2000) with the learned split-screen, exact step "
                  "every 50",
    "tri320k": "branching plate 100x40 mm on an unstructured CST mesh (Delaunay of 633x254 jittered points, "
               "319792 triangles), notch 50 mm, 1 MPa",
    "cylinder53k": "pressured hollow cylinder r 50/100 mm on an unstructured CST mesh (h 1 mm, ~53000 triangles), "
                   "steel, 400 MPa pulse",
    "quad160k": "branching plate 100x40 mm on an unstructured Q4 mesh (each Delaunay triangle of 259x104 "
                "jittered points split into 3 quadrilaterals, ~160000 elements), notch 50 mm, 1 MPa",
}
# untimed steps from t = 0 before the window (mid-run); 0 for the others
DEFAULT_START = {"batch256": 2500, "plate400": 10000, "fragment2000": 5000, "screen400": 10000,
                 "screen2000": 5000, "tri320k": 10000, "quad160k": 10000}


def n_elems(c) -> int:
    return len(c["conn"]) if c.get("conn") is not None else c["nx"] * c["ny"]


def n_nodes(c) -> int:
    return len(c["X"])


def bytes_per_step(cfgs, precision: int = 64, lattice: bool = False) -> int:
    """Algorithmic HBM bytes of one step (what the method must move): per
    node read u, v, 1/m and write u, v (9 values: 72 B in binary64, 36 in
    binary32), plus the reference coordinates X, Y (2 values) where the
    element geometry is recomputed from them (every mesh but a uniform
    lattice, whose elements share one geometry); per element its split code
    (1 B), its Gc where Gc varies per element (one value), and on an
    unstructured mesh its node ids (4 B each)."""
    w = 8 if precision == 64 else 4
    total = 0
    for c in cfgs:
        per_node = (9 + (0 if lattice else 2)) * w
        per_elem = 1 + (w if c.get("gc_field") is not None else 0)
        if c.get("conn") is not None:
            per_elem += 4 * len(c["conn"][0])
        total += per_node * n_nodes(c) + per_elem * n_elems(c)
    return total


# HBM bytes per launch of the dominant kernel measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over the profiled
# launches and summed over the step's kernels), each scaled by the ratio of
# true to counted bytes of a 256 MiB device copy (FETCH_SIZE x 1.99977,
# WRITE_SIZE x 1.0).  A figure holds for the kernel sources it was taken on
# (their hash) and the tile shape; otherwise the traffic is reported as null.
Q4_SOURCES = ("mct2d_step.hip", "mct2d_impl.h", "mct2d_device.h")
TRI_SOURCES = ("mct2d_tri.hip", "mct2d_tri.h", "mct2d_front.h", "mct2d_device.h", "mct2d_impl.h")
MEASURED_TRAFFIC = {
    # the batched lattice step kernel over the timed window (profiles/k_step_batch256_hbm_traffic.md)
    "batch256": {"sources": Q4_SOURCES, "sha256": "0be1dd5dbc91c01e5a3c4180b502f3022bb21a0a5fecd3af32a219a3f8110831",
                 "tile": 1, "fetch_kib": 286603.1083984375, "write_kib": 407268.94677734375},
    # the fused triangle step on its automatic patches (profiles/k_fused_tri320k_hbm_traffic.md)
    "tri320k": {"sources": TRI_SOURCES, "sha256": "806d14d94b3934373738da96454bcb13719769a770e41e96dd202916c26c103e",
                "tile": 5, "fetch_kib": 12160.925545, "write_kib": 5024.832886},
    # the fused quadrilateral step on its automatic patches (profiles/k_fused_quad160k_kernel_trace.md)
    "quad160k": {"sources": TRI_SOURCES, "sha256": "806d14d94b3934373738da96454bcb13719769a770e41e96dd202916c26c103e",
                 "tile": 5, "fetch_kib": 9238.957200, "write_kib": 5005.347145},
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


def host_cores() -> int:
    """The host cores this job may use: its CPU affinity, capped by
    OMP_NUM_THREADS where the machine sets it (the GPU machine sets it to the
    CPU share of one GPU)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        cores = min(cores, int(env))
    return max(1, cores)


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


def _specimen_worker(args):
    """One worker of the specimen-parallel baseline: its specimens (every
    `stride`-th from `first`) one after the other, each for `steps` time
    steps from t = 0 on one thread, until `seconds` are used."""
    first, stride, steps, seconds = args
    from oracle import oracle
    from paper_2509_01827_amd import workloads as W
    oracle.set_threads(1)
    cfgs = W.batch_specimens()
    t0 = time.perf_counter()
    updates, done = 0, 0
    for s in range(first, len(cfgs), stride):
        if time.perf_counter() - t0 >= seconds:
            break
        o = oracle.Oracle(cfgs[s])
        o.step(steps)
        updates += n_elems(cfgs[s]) * steps
        done += 1
    return updates, done


def cpu_baseline(workload, cfgs, seconds: float):
    """The oracle on the host's cores.  Single models: its OpenMP loops
    (results independent of the thread count), and single-threaded beside
    it.  The batch: specimens in parallel, one thread each, over a bounded
    sample (each worker runs its specimens for 20 steps from t = 0 until its
    time is used)."""
    cores = host_cores()
    if workload == "batch256":
        import multiprocessing as mp
        steps = 20
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_specimen_worker, [(w, cores, steps, seconds) for w in range(cores)])
        dt = time.perf_counter() - t0
        updates = sum(r[0] for r in res)
        nspec = sum(r[1] for r in res)
        return {"value": updates / dt, "unit": "element-updates/s", "cores": cores, "kind": "oracle",
                "sample": "%d of the 256 specimens, %d time steps each from t = 0 (C oracle, binary64), "
                          "specimen-parallel on %d processes of one thread, %.1f s wall" % (nspec, steps, cores, dt)}
    cfg = cfgs[0]
    rate, steps, dt = _oracle_rate(cfg, seconds, cores)
    rate1, steps1, dt1 = _oracle_rate(cfg, seconds, 1)
    ne = n_elems(cfg)
    return {"value": rate, "unit": "element-updates/s", "cores": cores, "kind": "oracle",
            "sample": "first %d time steps of the same %s (%d elements; C oracle, binary%d, %d threads, %.1f s)"
                      % (steps, cfg["name"], ne, int(cfg.get("precision", 64)), cores, dt),
            "single_thread": {"value": rate1, "cores": 1,
                              "sample": "first %d time steps, 1 thread, %.1f s" % (steps1, dt1)}}


def total_splits(m, nspec):
    if nspec == 1:
        return m.info()["n_splits"]
    total = 0
    for s in range(nspec):
        m.select(s)
        total += m.info()["n_splits"]
    m.select(0)
    return total


def timed_window(m, stream, start, warmup, steps, nspec):
    """Advance untimed to `start`, run `warmup` untimed steps, then time
    `steps` steps with HIP events on the model's stream.  Returns
    (gpu_ms, wall_s, splits made in the window)."""
    import torch
    if start:
        m.step(start)
    if warmup:
        m.step(warmup)
    m.sync()
    s0 = total_splits(m, nspec)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    m.step(steps)
    ev1.record(stream)
    m.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1), wall, total_splits(m, nspec) - s0


def same_logs(a, b):
    import numpy as np
    return all(np.array_equal(a[k], b[k]) for k in ("step", "elem", "entry", "exit", "G"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="time steps timed")
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--start", type=int, default=None,
                    help="untimed steps from t = 0 before the warm-up (default: mid-run, per workload)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="pick tile/order by measurement first")
    ap.add_argument("--profile-steps", type=int, default=64,
                    help="steps after the window timed per kernel launch (structured grids)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU-baseline sample: about this long per measurement")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch256: skip running each specimen alone with the plain step")
    ap.add_argument("--workload", default="batch256", choices=sorted(WORKLOADS))
    ap.add_argument("--smoothing", default="point", choices=("point", "subcell"),
                    help="Q4 edge smoothing (plain Q4 workloads)")
    ap.add_argument("--front-radius", type=float, default=0.0,
                    help="per-front pick with this competition radius in m (plain workloads; 0: global pick)")
    ap.add_argument("--precision", type=int, default=64, choices=(64, 32),
                    help="32: the binary32 step (plate400 and fragment2000)")
    ap.add_argument("--lattice", default="auto", choices=("auto", "general"),
                    help="general: never the uniform-lattice kernel")
    ap.add_argument("--kernel-hash", action="store_true",
                    help="only print the source hashes the measured traffic figures are keyed on")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (three times), "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.kernel_hash:
        print(json.dumps({"q4": kernel_sha256(Q4_SOURCES), "tri": kernel_sha256(TRI_SOURCES)}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
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

    import numpy as np
    from paper_2509_01827_amd import workloads as W

    screen = None
    if args.workload == "batch256":
        cfgs = W.batch_specimens()
    elif args.workload in ("screen400", "screen2000"):
        cfgs = [W.config2() if args.workload == "screen400" else W.config3()]
        with open(os.path.join(ROOT, "paper_2509_01827_amd", "screen_weights.json")) as f:
            screen = json.load(f)
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
    if args.lattice == "general":
        cfgs = [dict(c, lattice="general") for c in cfgs]
    start = args.start if args.start is not None else DEFAULT_START.get(args.workload, 0)
    if start + args.warmup + args.steps > cfgs[0]["steps"]:
        start = max(0, cfgs[0]["steps"] - args.warmup - args.steps)

    # the CPU baseline first: its worker processes start before this process
    # initialises the GPU
    cpu = None if args.no_cpu else cpu_baseline(args.workload, cfgs, args.cpu_seconds)

    import torch
    from paper_2509_01827_amd import mct2d
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    nspec = len(cfgs)
    if nspec > 1:
        m = mct2d.batch_from_configs(cfgs, stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
    else:
        m = mct2d.from_config(cfgs[0], stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
    if screen:
        mlp = mct2d.Mlp()
        mlp.set_params(np.asarray(screen["params"], np.float32))
        m.screen_enable(mlp, screen["tau"], screen["period"])
    tune = m.autotune(trial_steps=20) if args.autotune else None
    structured = cfgs[0].get("conn") is None
    lattice = structured and m.lattice()
    gpu_ms, wall, splits = timed_window(m, stream, start, args.warmup, args.steps, nspec)
    launch = m.launch()
    logs = []
    if nspec > 1 or screen:
        for s in range(nspec):
            if nspec > 1:
                m.select(s)
            logs.append(m.crack_set())
        if nspec > 1:
            m.select(0)
    ud = 0.0
    for s in range(nspec):
        if nspec > 1:
            m.select(s)
        ud += m.info()["dissipated"]
    screen_stats = m.screen_stats() if screen else None
    kt = None
    if structured and not screen and args.profile_steps > 0:
        kt = m.profile_step(args.profile_steps)
    ne = sum(n_elems(c) for c in cfgs)
    ms_per_step = gpu_ms / args.steps
    value = ne * args.steps / (gpu_ms * 1e-3)
    bps = bytes_per_step(cfgs, args.precision, lattice)
    # the dominant kernel's launch duration, from the timed window: the time
    # per step (step kernel + the batch's pick commit, launch gaps included)
    kern_us = ms_per_step * 1e3
    achieved = bps / (kern_us * 1e-6) / 1e9
    graph_ran = not args.no_graph and not screen
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
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "specimens": nspec, "elements": ne,
                   "start_step": start, "window": [start + args.warmup, start + args.warmup + args.steps],
                   "tile": launch["tile"], "order": launch["order"], "workgroups": launch["workgroups"],
                   "graph": graph_ran, "lattice": lattice, "smoothing": args.smoothing,
                   "front_radius": args.front_radius, "precision": args.precision, "autotuned": tune is not None},
        "wall_s": wall,
        "splits_in_window": splits,
        "dissipated_J_per_m": ud,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload, launch["tile"]),
                     "bytes_per_launch": bps, "kernel": "k_step" if structured else "step",
                     "kernel_us": kern_us, "kernel_us_from": "timed window, per step"},
    }
    if kt:
        out["kernel_timing"] = {"steps": args.profile_steps, "after_step": start + args.warmup + args.steps,
                                "step_kernel_us": kt["step_us"], "pick_commit_us": kt["commit_us"]}
    m.close()
    if screen:
        p = mct2d.from_config(cfgs[0], stream=stream.cuda_stream, tile=args.tile, use_graph=not args.no_graph)
        ms, _, _ = timed_window(p, stream, start, args.warmup, args.steps, 1)
        same = same_logs(p.crack_set(), logs[0])
        p.close()
        out["screened_vs_plain"] = {"speedup": ms / gpu_ms, "plain_ms": ms, "screened_ms": gpu_ms,
                                    "identical_crack_sets": bool(same), "tau": screen["tau"],
                                    "period": screen["period"], "stats": screen_stats}
    if nspec > 1 and not args.no_compare:
        # every specimen alone with the plain step over the same window
        plain_ms = 0.0
        same = True
        for s, cfg in enumerate(cfgs):
            p = mct2d.from_config(cfg, stream=stream.cuda_stream, use_graph=not args.no_graph)
            ms, _, _ = timed_window(p, stream, start, args.warmup, args.steps, 1)
            plain_ms += ms
            same = same and same_logs(p.crack_set(), logs[s])
            p.close()
        out["batched_vs_plain"] = {"speedup": plain_ms / gpu_ms, "plain_ms_total": plain_ms,
                                   "batched_ms": gpu_ms, "identical_crack_sets": bool(same)}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
