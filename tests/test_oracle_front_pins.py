"""Pins of the oracle's per-front pick (a variant of the Sec. 3 pick).

Definition: an accepted candidate c (it passed the element rule) splits iff,
against every other accepted candidate it competes with -- the same element,
or a tip point closer than the radius rho -- it has the better key (larger
G, then lower element id, then lower tip edge) and passes the split-ratio
test G_c > gamma (G_c - G_c').  All picked candidates split in the same step,
logged in key order.

Pinned: rho = infinity reproduces the global pick exactly (Q4 and CST runs);
a rule table on hand-made candidate sets; soundness and completeness of the
picked set against the definition at a state with many candidates; run
invariants (picked splits never compete, key order, U_d); and the physical
point of the variant -- two mirror fronts far apart advance together, so
their splits come in pairs in the same step (the global pick alternates
them).
"""
import math

import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W


def _same_log(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("step", "elem", "entry", "exit", "G"))


@pytest.mark.parametrize("kind", ["q4", "cst", "q4u"])
def test_infinite_radius_is_the_global_pick(oracle_mod, kind):
    if kind == "q4":
        cfg = W.small_cases()["fragment97x45"]
        steps = 300
    elif kind == "q4u":  # the same grid as an unstructured Q4 mesh
        cfg = W.as_unstructured_q4(W.small_cases()["fragment97x45"])
        steps = 300
    else:
        cfg = W.tri_small_cases()["tri_fragment"]
        steps = 300
    g = oracle_mod.run(cfg, steps)
    f = oracle_mod.run(dict(cfg, front_radius=math.inf), steps)
    assert len(g.log()["elem"]) > 20
    assert _same_log(g.log(), f.log())
    assert np.array_equal(g.state()["ux"], f.state()["ux"])


FRONT_CASES = [
    # G, elem, a, x, y, gamma, rho, expected picked (key order)
    ([5.0, 4.0], [10, 20], [0, 0], [0.0, 10.0], [0.0, 0.0], 1.0, 1.0, [0, 1]),   # far apart: both
    ([5.0, 4.0], [10, 20], [0, 0], [0.0, 0.5], [0.0, 0.0], 1.0, 1.0, [0]),      # close: the better
    ([4.0, 5.0], [10, 20], [0, 0], [0.0, 0.5], [0.0, 0.0], 1.0, 1.0, [1]),
    ([5.0, 4.0], [10, 20], [0, 0], [0.0, 0.5], [0.0, 0.0], 6.0, 1.0, []),       # gamma test fails
    ([5.0, 4.0], [10, 10], [0, 2], [0.0, 9.0], [0.0, 0.0], 1.0, 1.0, [0]),      # same element always competes
    ([5.0, 5.0], [11, 10], [0, 0], [0.0, 0.5], [0.0, 0.0], 1.0, 1.0, [1]),      # tie: lower element
    ([5.0, 5.0], [10, 10], [3, 1], [0.0, 0.5], [0.0, 0.0], 1.0, 1.0, [1]),      # tie: lower tip edge
    # chain A > B > C, A-B and B-C compete, A-C do not: C loses to B although
    # B is not picked (no greedy second round)
    ([6.0, 5.0, 4.0], [1, 2, 3], [0, 0, 0], [0.0, 0.8, 1.6], [0.0, 0.0, 0.0], 1.0, 1.0, [0]),
    ([3.0, 7.0, 5.0], [1, 2, 3], [0, 0, 0], [0.0, 5.0, 10.0], [0.0, 0.0, 0.0], 1.0, 1.0, [1, 2, 0]),  # key order
    ([5.0, 4.0], [10, 20], [0, 0], [0.0, 1.0], [0.0, 0.0], 1.0, 1.0, [0, 1]),   # distance == rho: no competition
]


@pytest.mark.parametrize("G,elem,a,x,y,gamma,rho,exp", FRONT_CASES)
def test_front_pick_table(oracle_mod, G, elem, a, x, y, gamma, rho, exp):
    got = oracle_mod.front_pick(G, elem, a, x, y, gamma, rho)
    assert list(got) == exp


def _tip_points(cfg, cand):
    X, Y = cfg["X"], cfg["Y"]
    if cfg.get("conn") is not None:
        T = np.asarray(cfg["conn"])
        nv = T.shape[1]
        nodes = [(T[e, a], T[e, (a + 1) % nv]) for e, a in zip(cand["elem"], cand["a"])]
    else:
        nx = cfg["nx"]
        out = []
        for e, a in zip(cand["elem"], cand["a"]):
            i, j = e % nx, e // nx
            nd = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
            out.append((nd[a], nd[(a + 1) % 4]))
        nodes = out
    x = np.array([0.5 * (X[p] + X[q]) for p, q in nodes])
    y = np.array([0.5 * (Y[p] + Y[q]) for p, q in nodes])
    return x, y


def test_picked_set_is_sound_and_complete(oracle_mod):
    cfg = W.small_cases()["fragment97x45"]
    o = oracle_mod.run(cfg, 120)
    cand = o.candidates()
    acc = cand["dec"] >= 0
    Gsel = np.array([g[d] for g, d in zip(cand["G"], cand["dec"])])[acc]
    el, a = cand["elem"][acc], cand["a"][acc]
    x, y = _tip_points(cfg, cand)
    x, y = x[acc], y[acc]
    assert len(Gsel) > 10
    rho, gamma = 3e-3, cfg["gamma"]
    picked = set(oracle_mod.front_pick(Gsel, el, a, x, y, gamma, rho).tolist())
    assert len(picked) > 1
    for c in range(len(Gsel)):
        wins = True
        for d in range(len(Gsel)):
            if d == c:
                continue
            if el[c] != el[d] and (x[c] - x[d]) ** 2 + (y[c] - y[d]) ** 2 >= rho ** 2:
                continue
            key_c = (-Gsel[c], el[c], a[c])
            key_d = (-Gsel[d], el[d], a[d])
            if not key_c < key_d or not Gsel[c] > gamma * (Gsel[c] - Gsel[d]):
                wins = False
        assert wins == (c in picked), c


@pytest.mark.parametrize("kind", ["q4", "cst", "q4u"])
def test_front_run_invariants(oracle_mod, kind):
    if kind == "q4":
        cfg = dict(W.small_cases()["fragment97x45"], front_radius=3e-3)
    elif kind == "q4u":
        cfg = dict(W.as_unstructured_q4(W.small_cases()["fragment97x45"]), front_radius=3e-3)
    else:
        cfg = dict(W.tri_small_cases()["tri_fragment"], front_radius=3e-3)
    o = oracle_mod.run(cfg, 300)
    lg = o.log()
    steps = lg["step"]
    assert len(steps) > 30
    assert np.any(np.diff(steps) == 0), "several splits in one step"
    # per step: distinct elements, pairwise distance >= rho, key order
    for s in np.unique(steps):
        idx = np.where(steps == s)[0]
        sub = {k: lg[k][idx] for k in lg}
        x, y = _tip_points(cfg, {"elem": sub["elem"], "a": sub["entry"]})
        assert len(set(sub["elem"].tolist())) == len(idx)
        for i in range(len(idx)):
            for j in range(i + 1, len(idx)):
                assert (x[i] - x[j]) ** 2 + (y[i] - y[j]) ** 2 >= cfg["front_radius"] ** 2
                assert (-sub["G"][i], sub["elem"][i], sub["entry"][i]) < (-sub["G"][j], sub["elem"][j], sub["entry"][j])
    gc = cfg.get("gc_field")
    Ud = sum((gc[e] if gc is not None else cfg["gc_uniform"]) * o.path_normal(e, a, k)[2]
             for e, a, k in zip(lg["elem"], lg["entry"], lg["exit"]))
    assert o.info()["Ud"] == pytest.approx(Ud, rel=1e-13)


def _double_notch(nx=40, ny=21, h=1e-3, ln=10, steps=700):
    c = W.plate(nx, ny, nx * h, ny * h, notch_len=None, steps=steps, name="double_notch")
    row = ny // 2
    el = [row * nx + i for i in range(ln)] + [row * nx + nx - 1 - i for i in range(ln)]
    en = [3] * ln + [1] * ln
    ex = [1] * ln + [3] * ln
    c["notch"] = (np.array(el, np.int32), np.array(en, np.uint8), np.array(ex, np.uint8))
    return c


def test_mirror_fronts_advance_together(oracle_mod):
    """Notches from the left and the right edge, mirror-symmetric about the
    vertical centre line: the per-front pick splits both fronts in the same
    step, the global pick alternates them."""
    nx, ny = 40, 21
    base = _double_notch(nx, ny)
    front = oracle_mod.run(dict(base, front_radius=8e-3), base["steps"])
    glob = oracle_mod.run(base, base["steps"])
    lf, lgb = front.log(), glob.log()
    assert len(lf["elem"]) >= 6 and len(lgb["elem"]) >= 6
    # global: one split per step
    assert np.all(np.diff(lgb["step"]) > 0)
    # per front: while the fronts are far apart, every split on the left
    # front has a partner on the right front in the same step: the mirror
    # column, and the same row or its image about the crack line (above /
    # below the crack line is a near-tie that rounding decides per front)
    pairs = 0
    for s in np.unique(lf["step"]):
        idx = np.where(lf["step"] == s)[0]
        cells = [(int(lf["elem"][i]) % nx, int(lf["elem"][i]) // nx) for i in idx]
        if min(abs(i - (nx - 1 - i)) for i, _ in cells) < 8:
            break  # fronts near the centre compete
        left = sorted((i, min(j, ny - 1 - j)) for i, j in cells if i < nx // 2)
        right = sorted((nx - 1 - i, min(j, ny - 1 - j)) for i, j in cells if i >= nx // 2)
        assert left == right, (s, cells)
        pairs += len(left)
    assert pairs >= 3
    # the global pick alternates the two fronts instead
    first = [int(e) % nx < nx // 2 for e in lgb["elem"][:6]]
    assert any(first) and not all(first)
