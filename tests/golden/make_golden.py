"""Write full-size reference results of the CPU oracle for the GPU parity
tests.  Calls only oracle/ (and the seeded workload generators).

    python tests/golden/make_golden.py plate400 [--threads N]

Output: tests/golden/<name>.json with SHA-256 digests of the full split log
and of the split codes, the first log entries, the dissipated energy, the
tip count, the near-threshold decision log (digest, count and first
records; tolerance NEAR_TOL) and the displacement/velocity of a seeded
sample of nodes; every binary64 value is stored as float.hex() so the
comparison can be exact.  The batch case holds one such record per sampled
specimen (each specimen is an independent model).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_2509_01827_amd import workloads as W  # noqa: E402

NEAR_TOL = 1e-6

CASES = {
    # the 400x400 branching plate, full 20 000-step run
    "plate400": lambda: dict(W.config2(), near_tol=NEAR_TOL),
    # the same plate with the binary32 step (the binary32 build of the oracle)
    "plate400_f32": lambda: dict(W.config2(), precision=32, near_tol=NEAR_TOL),
    # the 2000x1000 fragmentation plate, full 10 000-step run
    "fragment2000": lambda: dict(W.config3(), near_tol=NEAR_TOL),
}


def batch_sample():
    """Indices of the sampled specimens of the 256-specimen batch: the
    largest, the smallest and two seeded random ones."""
    cfgs = W.batch_specimens()
    ne = [c["nx"] * c["ny"] for c in cfgs]
    big, small = int(np.argmax(ne)), int(np.argmin(ne))
    rest = [s for s in range(len(cfgs)) if s not in (big, small)]
    u = W.uniform01(W.BASE_SEED + 98, 2)
    r0 = rest[int(u[0] * len(rest))]
    rest.remove(r0)
    r1 = rest[int(u[1] * len(rest))]
    return cfgs, [big, small, r0, r1]

N_SAMPLE = 512
N_HEAD = 200


def log_digest(step, elem, entry, exit_, G):
    """SHA-256 over the split log: int64 step, elem, entry, exit and the
    binary64 bits of G, little-endian, in log order."""
    h = hashlib.sha256()
    for a in (step, elem, entry, exit_):
        h.update(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes())
    h.update(np.ascontiguousarray(np.asarray(G, dtype="<f8")).tobytes())
    return h.hexdigest()


def codes_digest(split):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(split, dtype=np.uint8)).tobytes()).hexdigest()


def sample_nodes(nn, seed):
    u = W.uniform01(seed, N_SAMPLE)
    return np.unique((u * nn).astype(np.int64))


def near_digest(nl):
    """SHA-256 over the near-threshold log sorted by (step, kind, element,
    tip edge, exit edge): int64 fields, then the binary64 bits of G and ref."""
    order = np.lexsort((nl["k"], nl["a"], nl["elem"], nl["kind"], nl["step"]))
    h = hashlib.sha256()
    for key in ("step", "elem", "a", "kind", "k"):
        h.update(np.ascontiguousarray(np.asarray(nl[key][order], dtype="<i8")).tobytes())
    for key in ("G", "ref"):
        h.update(np.ascontiguousarray(np.asarray(nl[key][order], dtype="<f8")).tobytes())
    return h.hexdigest(), order


def run_case(name, cfg, threads):
    t0 = time.time()
    o = oracle.Oracle(cfg)
    steps = cfg["steps"]
    chunk = 500
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        o.step(n)
        done += n
        print("%s: %d/%d steps, %d splits, %.0f s" % (name, done, steps, o.info()["nlog"],
                                                       time.time() - t0), flush=True)
    inf = o.info()
    st = o.state()
    lg = o.log()
    tips, _ = o.tips()
    nodes = sample_nodes(inf["nn"], W.BASE_SEED + 99)
    h = lambda a: [float(x).hex() for x in a]
    out = {
        "case": name,
        "source": "oracle/mct_oracle.c via tests/golden/make_golden.py",
        "precision": int(cfg.get("precision", 64)),
        "steps": steps,
        "dt": float(inf["dt"]).hex(),
        "Ud": float(inf["Ud"]).hex(),
        "n_tips": int(len(tips)),
        "tips_digest": hashlib.sha256(np.asarray(tips, "<i8").tobytes()).hexdigest(),
        "n_splits": int(len(lg["elem"])),
        "log_digest": log_digest(lg["step"], lg["elem"], lg["entry"], lg["exit"], lg["G"]),
        "codes_digest": codes_digest(st["split"]),
        "log_head": {"step": lg["step"][:N_HEAD].tolist(), "elem": lg["elem"][:N_HEAD].tolist(),
                     "entry": lg["entry"][:N_HEAD].tolist(), "exit": lg["exit"][:N_HEAD].tolist(),
                     "G": h(lg["G"][:N_HEAD])},
        "nodes": nodes.tolist(),
        "ux": h(st["ux"][nodes]), "uy": h(st["uy"][nodes]),
        "vx": h(st["vx"][nodes]), "vy": h(st["vy"][nodes]),
        "split_count": int((st["split"] != 0).sum()),
        "threads": threads,
        "seconds": time.time() - t0,
    }
    if cfg.get("near_tol"):
        nl = o.near_log()
        dig, order = near_digest(nl)
        out["near"] = {"tol": cfg["near_tol"], "count": int(len(nl["kind"])), "digest": dig,
                       "head": {key: nl[key][order][:N_HEAD].tolist() for key in ("step", "elem", "a", "kind", "k")}}
        out["near"]["head"]["G"] = h(nl["G"][order][:N_HEAD])
        out["near"]["head"]["ref"] = h(nl["ref"][order][:N_HEAD])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(CASES) + ["batch256_sample"])
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    if args.name == "batch256_sample":
        cfgs, idx = batch_sample()
        out = {"case": args.name, "source": "oracle/mct_oracle.c via tests/golden/make_golden.py",
               "n_specimens": len(cfgs), "sample": idx,
               "specimens": [run_case("specimen%d" % s, cfgs[s], args.threads) for s in idx]}
    else:
        out = run_case(args.name, CASES[args.name](), args.threads)
    path = os.path.join(HERE, args.name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
