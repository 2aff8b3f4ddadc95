"""Train the learned split-screen and write its parameters.

    python -m paper_2509_01827_amd.screen_train [--out FILE]

Data: seeded runs of the branching-plate set-up (the 400 x 400 jittered
plate with other jitter seeds, and 40 x 40 plates with jitter), stepped
exactly on the GPU; every `period` steps the features of every candidate
are collected.  Label of a row (step k, element f, edge a): f splits with
entry edge a in one of the steps k+1 .. k+period (the steps a screen
computed at step k decides for).  The MLP is trained on the GPU (bfloat16
MFMA, FP32 Adam) on the weighted logistic loss.

Threshold: tau sits just below the smallest logit of any positive training
row (recall 1 on the training set).  For the record, the thresholds at
recall 0.99995 ... 0.999 are also run on a validation plate (another jitter
seed of the 400 x 400 plate) against its plain run.  The benchmark plate
(its own seed, in no other run) is then run plain and screened and the
crack sets compared.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import mct2d
from . import workloads as W

PERIOD = 50


def collect(cfg, steps, period=PERIOD, stream=None):
    """Features and labels of one exact run.  Label of the row of candidate
    (f, a) collected at step k: f splits with entry edge a in one of the
    steps k+1 .. k+period (a split through another edge comes from a
    candidate that is new, hence evaluated anyway)."""
    m = mct2d.from_config(cfg, stream=stream)
    rows, keys = [], []
    k = 0
    while k < steps:
        el, en, F = m.screen_collect()
        rows.append(F)
        keys.append(np.stack([np.full(len(el), k, np.int64), el.astype(np.int64), en.astype(np.int64)], axis=1))
        n = min(period, steps - k)
        m.step(n)
        k += n
    log = m.crack_set()
    m.close()
    X = np.concatenate(rows)
    K = np.concatenate(keys)
    # split step and entry edge of each element (an element splits at most once)
    ne = cfg["nx"] * cfg["ny"]
    split_step = np.full(ne, -1, np.int64)
    split_entry = np.full(ne, -1, np.int64)
    split_step[log["elem"]] = log["step"]
    split_entry[log["elem"]] = log["entry"]
    s = split_step[K[:, 1]]
    y = ((s > K[:, 0]) & (s <= K[:, 0] + period) & (split_entry[K[:, 1]] == K[:, 2])).astype(np.float32)
    return X, y


def training_runs():
    runs = []
    for r in range(3):
        runs.append(W.plate(400, 400, 0.1, 0.04, jitter=0.01, seed=W.BASE_SEED + 5 + r, notch_len=200,
                            steps=20000, name="plate400_seed%d" % r))
    for r in range(8):
        runs.append(W.plate(40, 40, 0.04, 0.04, jitter=0.01, seed=W.BASE_SEED + 15 + r, notch_len=20,
                            steps=2000, name="plate40_seed%d" % r))
    return runs


def train(X, y, *, epochs=6, batch=8192, lr=2e-3, seed=0, stream=None, log=print):
    import torch
    rng = np.random.default_rng(seed)
    n = len(y)
    pos = float(y.sum())
    pos_weight = float(min(max((n - pos) / max(pos, 1.0), 1.0), 50.0))
    mlp = mct2d.Mlp(stream)
    # Kaiming-uniform-like initial weights, zero biases
    p = np.zeros(mct2d.N_PARAMS, np.float32)
    p[0:640] = rng.uniform(-1, 1, 640) * np.sqrt(6.0 / 10.0)
    p[704:4800] = rng.uniform(-1, 1, 4096) * np.sqrt(6.0 / 64.0)
    p[4864:4928] = rng.uniform(-1, 1, 64) * np.sqrt(6.0 / 64.0)
    mlp.set_params(p)
    xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        xs, ys = xd[perm].contiguous(), yd[perm].contiguous()
        lr_e = lr * (0.5 ** max(0, ep - epochs // 2))
        for b0 in range(0, n - batch + 1, batch):
            mlp.train_step(xs[b0:b0 + batch], ys[b0:b0 + batch], pos_weight=pos_weight, lr=lr_e)
        loss, _ = mlp.gradient(xd, yd, pos_weight=pos_weight)
        log("epoch %d lr %.2e loss %.5f" % (ep, lr_e, loss))
    return mlp, pos_weight


def logits_of(mlp, X):
    import torch
    xd = torch.from_numpy(X).cuda()
    out = torch.zeros(len(X), dtype=torch.float32, device="cuda")
    mlp.forward(xd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def evaluate(cfg, mlp, tau, period=PERIOD, stream=None):
    import torch
    res = {}
    runs = {}
    for mode in ("plain", "screened"):
        m = mct2d.from_config(cfg, stream=stream)
        if mode == "screened":
            m.screen_enable(mlp, tau, period)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(cfg["steps"])
        m.sync()
        res[mode + "_s"] = time.perf_counter() - t0
        runs[mode] = m
    a, b = runs["plain"].crack_set(), runs["screened"].crack_set()
    res["identical_crack_sets"] = bool(all(np.array_equal(a[k], b[k]) for k in ("step", "elem", "entry", "exit")))
    res["splits"] = int(len(a["elem"]))
    res["stats"] = runs["screened"].screen_stats()
    for m in runs.values():
        m.close()
    return res


RECALLS = (1.0, 0.99995, 0.9999, 0.9998, 0.9995, 0.999)


def validation_run():
    return W.plate(400, 400, 0.1, 0.04, jitter=0.01, seed=W.BASE_SEED + 8, notch_len=200, steps=20000,
                   name="plate400_validation")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "screen_weights.json"))
    ap.add_argument("--epochs", type=int, default=8)
    args = ap.parse_args()
    t0 = time.perf_counter()
    Xs, ys = [], []
    for cfg in training_runs():
        X, y = collect(cfg, cfg["steps"])
        print("%s: %d rows, %d positive (%.1f s)" % (cfg["name"], len(y), int(y.sum()), time.perf_counter() - t0),
              flush=True)
        Xs.append(X)
        ys.append(y)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    print("features min", X.min(axis=0), "max", X.max(axis=0), flush=True)
    mlp, pos_weight = train(X, y, epochs=args.epochs, log=lambda s: print(s, flush=True))
    z = logits_of(mlp, X)
    zp = np.sort(z[y > 0.5])
    choices = []
    for rec in RECALLS:
        tau = float(zp[int((1.0 - rec) * len(zp))]) - 1e-3
        choices.append(dict(recall=rec, tau=tau, flagged_fraction_train=float((z > tau).mean())))
    print("thresholds:", choices, flush=True)
    val = validation_run()
    for ch in choices:
        ev = evaluate(val, mlp, ch["tau"])
        ch["validation"] = ev
        print("validation recall %.5f tau %.3f: %s" % (ch["recall"], ch["tau"], ev), flush=True)
    chosen = choices[0]  # recall 1 on the training rows
    test = evaluate(W.config2(), mlp, chosen["tau"])
    print("benchmark plate400 with tau %.3f: %s" % (chosen["tau"], test), flush=True)
    out = dict(params=[float(v) for v in mlp.params()], tau=chosen["tau"], period=PERIOD,
               train=dict(rows=int(len(y)), positives=int(y.sum()), pos_weight=pos_weight, epochs=args.epochs,
                          runs=[c["name"] for c in training_runs()], thresholds=choices,
                          chosen_recall=chosen["recall"], validation_run=val["name"]),
               heldout=test)
    with open(args.out, "w") as f:
        json.dump(out, f)
    print("wrote", args.out, "in %.1f s" % (time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
