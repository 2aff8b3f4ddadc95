"""Plain FP64 reference of the learned split-screen (numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by nothing in the product
package.  The screen is an extension of the method, not part of the paper:
it predicts which free-surface candidates of the element-split criterion
(Sec. 2.2, G of the three split topologies against G_c) are worth
evaluating during the next steps; an exact evaluation of every candidate
at a fixed period keeps the final decision with the criterion itself.

Contents
  features()        10 features per candidate (f, a) from an oracle state
  bf16()            round-to-nearest-even to bfloat16 (kept as float64)
  forward()         MLP 10 -> 64 -> 64 -> 1 with GELU
  loss_and_grad()   weighted logistic loss and its exact gradient
  adam()            one Adam update
All arithmetic is float64; the optional bfloat16 rounding is applied at the
points where the device kernels round (inputs, weight copies, hidden
activations and the backpropagated pre-activation gradients).

Parameter vector (4 929 values): W1 [10][64] (input-major), b1 [64],
W2 [64][64], b2 [64], w3 [64], b3 [1].
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H = 10, 64
N_PARAMS = N_IN * N_H + N_H + N_H * N_H + N_H + N_H + 1
TIP_CAP = 64.0


# ---------------------------------------------------------------- features

def _element_edges(o):
    """Edge id of each (element, local edge) from the oracle's edge tables."""
    t = o.tables()
    ne = o.info()["ne"]
    ee = np.full((ne, 4), -1, np.int64)
    for s in range(len(t["edge_elem"])):
        for side in range(2):
            e = t["edge_elem"][s, side]
            if e >= 0:
                ee[e, t["edge_loc"][s, side]] = s
    return ee


def features(o, cfg, g_prev=None):
    """Features of every candidate of the oracle's current state.

    Candidate = intact element f with a free surface across its local edge a
    (the split criterion's candidate set).  Per candidate, with h = sqrt(A_f)
    and sigma_ref = sqrt(E G_c / h):
      0, 1  principal stresses of the mean of the four edge stresses of f,
            over sigma_ref (larger first)
      2     W h / G_c, W = 1/2 sigma:eps of that mean stress (plane stress)
      3     max of the three path G values / G_c (0 when the edge is not
            stretched)
      4     the same quantity at the previous evaluation (g_prev[(f, a)],
            0 when absent)
      5     min(d / h, 64) / 64, d = distance from the midpoint of edge a to
            the nearest crack-path end (reference coordinates): the midpoint
            of an entry or exit edge of a split element whose neighbour
            across that edge is intact; 1 without such ends
      6..9  1 where the neighbour across local edge k = 0..3 is split or
            outside the mesh, else 0
    Returns (elem, a, F [n][10], gnow dict for the next call).
    """
    E, nu = float(cfg["E"]), float(cfg["nu"])
    st = o.state()
    _, _, sig, ok = o.internal_force(st["ux"], st["uy"], with_stress=True)
    cand = o.candidates()
    tabs = o.tables()
    area = tabs["area"]
    ee = _element_edges(o)
    nx, ny = o.nx, o.ny
    split = st["split"]
    X, Y = np.asarray(cfg["X"], float), np.asarray(cfg["Y"], float)
    gcf = cfg.get("gc_field")
    tip_xy = path_ends(nx, ny, X, Y, split)
    n = len(cand["elem"])
    F = np.zeros((n, N_IN))
    gnow = {}
    for r in range(n):
        f, a = int(cand["elem"][r]), int(cand["a"][r])
        gc = float(gcf[f]) if gcf is not None else float(cfg["gc_uniform"])
        h = math.sqrt(area[f])
        sref = math.sqrt(E * gc / h)
        s = np.zeros(3)
        for k in range(4):
            assert ok[ee[f, k]]
            s = s + sig[ee[f, k]]
        s = s / 4.0
        c = 0.5 * (s[0] + s[1])
        rr = math.sqrt((0.5 * (s[0] - s[1])) ** 2 + s[2] ** 2)
        exx = (s[0] - nu * s[1]) / E
        eyy = (s[1] - nu * s[0]) / E
        gxy = 2.0 * (1.0 + nu) * s[2] / E
        W = 0.5 * (s[0] * exx + s[1] * eyy + s[2] * gxy)
        G3 = cand["G"][r]
        gmax = max(G3[0], G3[1], G3[2]) / gc
        i, j = f % nx, f // nx
        nd = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
        p, q = nd[a], nd[(a + 1) % 4]
        mx, my = 0.5 * (X[p] + X[q]), 0.5 * (Y[p] + Y[q])
        if len(tip_xy):
            d = math.sqrt(min((tx - mx) ** 2 + (ty - my) ** 2 for tx, ty in tip_xy))
            fd = min(d / h, TIP_CAP) / TIP_CAP
        else:
            fd = 1.0
        nb = [(i, j - 1), (i + 1, j), (i, j + 1), (i - 1, j)]
        flags = []
        for (bi, bj) in nb:
            if bi < 0 or bi >= nx or bj < 0 or bj >= ny:
                flags.append(1.0)
            else:
                flags.append(1.0 if split[bj * nx + bi] != 0 else 0.0)
        prev = 0.0 if g_prev is None else g_prev.get((f, a), 0.0)
        F[r] = [(c + rr) / sref, (c - rr) / sref, W * h / gc, gmax, prev, fd] + flags
        gnow[(f, a)] = gmax
    return cand["elem"].astype(np.int64), cand["a"].astype(np.int64), F, gnow


def path_ends(nx, ny, X, Y, split):
    """Midpoints of the crack-path ends: entry or exit edges of split
    elements whose neighbour across the edge is an intact element."""
    out = []
    for e in range(nx * ny):
        c = int(split[e])
        if c == 0:
            continue
        i, j = e % nx, e // nx
        nd = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
        for k in ((c >> 2) & 3, c & 3):
            bi, bj = [(i, j - 1), (i + 1, j), (i, j + 1), (i - 1, j)][k]
            if 0 <= bi < nx and 0 <= bj < ny and split[bj * nx + bi] == 0:
                p, q = nd[k], nd[(k + 1) % 4]
                out.append((0.5 * (X[p] + X[q]), 0.5 * (Y[p] + Y[q])))
    return out


# --------------------------------------------------------------- bfloat16

def bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even), first to
    float32 as the device holds them; returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    out = b.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


# -------------------------------------------------------------------- MLP

def unpack(p):
    p = np.asarray(p, np.float64)
    assert p.shape == (N_PARAMS,)
    o = 0
    W1 = p[o:o + N_IN * N_H].reshape(N_IN, N_H); o += N_IN * N_H
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    w3 = p[o:o + N_H]; o += N_H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2, w3, [b3]])


def gelu(z):
    return 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def gelu_prime(z):
    Phi = 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def _round(x, on):
    return bf16(x) if on else np.asarray(x, np.float64)


def forward(p, X, emulate_bf16=True, keep=False):
    """Logits of the rows of X [n][10]."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    R = lambda v: _round(v, emulate_bf16)
    x = R(X)
    z1 = x @ R(W1) + b1
    h1 = R(gelu(z1))
    z2 = h1 @ R(W2) + b2
    h2 = R(gelu(z2))
    z3 = h2 @ R(w3) + b3
    if keep:
        return z3, (x, z1, h1, z2, h2)
    return z3


def loss_and_grad(p, X, y, pos_weight=1.0, emulate_bf16=True):
    """Mean over rows of w_i (softplus(z_i) - y_i z_i), w_i = pos_weight
    where y_i = 1, and its gradient with respect to p (backpropagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    R = lambda v: _round(v, emulate_bf16)
    y = np.asarray(y, np.float64)
    n = len(y)
    z3, (x, z1, h1, z2, h2) = forward(p, X, emulate_bf16, keep=True)
    w = np.where(y > 0.5, pos_weight, 1.0)
    loss = float(np.sum(w * (np.logaddexp(0.0, z3) - y * z3)) / n)
    dz3 = w * (1.0 / (1.0 + np.exp(-z3)) - y) / n
    g_w3 = h2.T @ dz3
    g_b3 = np.sum(dz3)
    dh2 = np.outer(dz3, R(w3))
    dz2 = R(dh2 * gelu_prime(z2))
    g_W2 = h1.T @ dz2
    g_b2 = dz2.sum(axis=0)
    dh1 = dz2 @ R(W2).T
    dz1 = R(dh1 * gelu_prime(z1))
    g_W1 = x.T @ dz1
    g_b1 = dz1.sum(axis=0)
    return loss, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
