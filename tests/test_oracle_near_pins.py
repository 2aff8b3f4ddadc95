"""Pins of the oracle's near-threshold decision log (CPU).

The log records every decision whose margin lies within a relative tolerance:
a path G against Gc (kind 1), the gap between the two largest paths above Gc
of one element (2), the element rule's split-ratio margin (3), the gap
between the two largest accepted candidates of a step (4) and the pick's
split-ratio margin (5).  Pinned here by hand-made tables for every kind,
by invariance of the run (recording changes nothing), by monotonicity in the
tolerance and by an independent enumeration over the candidates that the
oracle's candidate query reports before each step.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2509_01827_amd import workloads as W


def _tiny(tol, gamma=1.0):
    cfg = W.plate(4, 3, 0.004, 0.003, notch_len=1, gamma=gamma, steps=1)
    cfg["near_tol"] = tol
    return oracle.Oracle(cfg)


def _cand(o, a, G, Gc):
    o._L.orc_near_candidate(o.h, 5, a, len(G), np.asarray(G, np.float64), float(Gc))
    nl = o.near_log()
    return list(zip(nl["kind"].tolist(), nl["k"].tolist(), nl["G"].tolist(), nl["ref"].tolist()))


@pytest.mark.parametrize("a", [0, 1, 2, 3])
def test_path_near_gc(a):
    o = _tiny(1e-9)
    k0 = (a + 1) % 4
    assert _cand(o, a, [3.0 * (1 + 1e-12), 0.0, 0.0], 3.0) == [(1, k0, 3.0 * (1 + 1e-12), 3.0)]
    o = _tiny(1e-9)
    assert _cand(o, a, [3.0 * (1 + 1e-6), 0.0, 0.0], 3.0) == []
    o = _tiny(1e-9)  # exactly at Gc: the strict rule rejects it, and it is a near decision
    assert _cand(o, a, [0.0, 0.0, 3.0], 3.0) == [(1, (a + 3) % 4, 3.0, 3.0)]


def test_element_gap_and_ties():
    o = _tiny(1e-9)
    g2 = 2.0 * (1 - 1e-12)
    assert _cand(o, 0, [0.5, 2.0, g2], 1.0) == [(2, 2, 2.0, g2)]   # best path 1 (exit edge 2)
    o = _tiny(1e-9)
    assert _cand(o, 1, [3.0, 3.0, 3.0], 1.0) == [(2, 2, 3.0, 3.0)]  # ties: the first path wins
    o = _tiny(1e-9)
    assert _cand(o, 0, [4.0, 2.0, 0.5], 1.0) == []                  # a clear decision


def test_element_ratio_margin_gamma2():
    o = _tiny(1e-9, gamma=2.0)
    gj = 2.0 + 1e-12
    rec = _cand(o, 0, [4.0, gj, 0.0], 1.0)
    # 4 - 2 (4 - gj) = 2e-12 <= 1e-9 * 4: the margin of path 1 (exit edge 2)
    assert rec == [(3, 2, 4.0, gj)]
    o = _tiny(1e-9, gamma=2.0)
    assert _cand(o, 0, [4.0, 2.5, 0.0], 1.0) == []


def _pick(o, G, c, gamma_note=None):
    n = len(G)
    elem = np.arange(10, 10 + n, dtype=np.int32)
    a = np.zeros(n, np.int32)
    k = np.full(n, 2, np.int32)
    o._L.orc_near_pick(o.h, n, np.asarray(G, np.float64), elem, a, k, c)
    nl = o.near_log()
    return list(zip(nl["kind"].tolist(), nl["elem"].tolist(), nl["G"].tolist(), nl["ref"].tolist()))


def test_pick_gap_and_margin():
    o = _tiny(1e-9)
    s = 5.0 * (1 - 1e-12)
    assert _pick(o, [5.0, 3.5, s], 0) == [(4, 10, 5.0, s)]
    o = _tiny(1e-9)
    assert _pick(o, [5.0], 0) == []  # one candidate: no gap, the ratio test is vacuous
    o = _tiny(1e-9, gamma=2.0)
    gm = 2.0 + 1e-12
    assert _pick(o, [4.0, 3.0, gm], 0) == [(5, 10, 4.0, gm)]


def _run(cfg, steps, tol):
    c = dict(cfg)
    if tol:
        c["near_tol"] = tol
    return oracle.run(c, steps)


def test_log_does_not_change_the_run():
    cfg = W.small_cases()["plate70x37_jitter"]
    a = _run(cfg, 700, 0.0)
    b = _run(cfg, 700, 1e-2)
    la, lb = a.log(), b.log()
    assert len(la["elem"]) > 50
    for key in la:
        assert np.array_equal(la[key], lb[key])
    assert np.array_equal(a.state()["ux"], b.state()["ux"])
    assert len(b.near_log()["kind"]) > 0


def test_monotone_in_tolerance():
    cfg = W.small_cases()["fragment97x45"]
    lo = _run(cfg, 150, 1e-4).near_log()
    hi = _run(cfg, 150, 1e-2).near_log()
    key = lambda nl: set(zip(nl["step"].tolist(), nl["elem"].tolist(), nl["a"].tolist(), nl["kind"].tolist(),
                             nl["k"].tolist()))
    assert len(lo["kind"]) < len(hi["kind"])
    assert key(lo) <= key(hi)


def test_enumeration_against_candidate_query():
    """Before every step, the candidate query gives each free-surface
    candidate's three path values and decision; the records the step then
    makes must be exactly the near decisions among them."""
    cfg = dict(W.small_cases()["fragment97x45"], near_tol=2e-2)
    o = oracle.Oracle(cfg)
    tol = cfg["near_tol"]
    gamma = cfg["gamma"]
    gcf = cfg["gc_field"]
    for step in range(60):
        c = o.candidates()
        before = len(o.near_log()["kind"])
        o.step(1)
        nl = o.near_log()
        got = sorted(zip(nl["kind"][before:].tolist(), nl["elem"][before:].tolist(), nl["a"][before:].tolist(),
                         nl["k"][before:].tolist()))
        want = []
        acc = []
        for e, a, G, d in zip(c["elem"], c["a"], c["G"], c["dec"]):
            gc = gcf[e]
            for j in range(3):
                if abs(G[j] - gc) <= tol * gc:
                    want.append((1, e, a, (a + 1 + j) % 4))
            S = [j for j in range(3) if G[j] > gc]
            if len(S) >= 2:
                b = max(S, key=lambda j: (G[j], -j))
                sec = max(G[j] for j in S if j != b)
                if G[b] - sec <= tol * G[b]:
                    want.append((2, e, a, (a + 1 + b) % 4))
                for j in S:
                    if j != b and abs(G[b] - gamma * (G[b] - G[j])) <= tol * G[b]:
                        want.append((3, e, a, (a + 1 + j) % 4))
            if d >= 0:
                acc.append((G[d], e, a, (a + 1 + d) % 4))
        if acc:
            best = min(acc, key=lambda t: (-t[0], t[1], t[2]))
            others = [t[0] for t in acc if t is not best]
            gmin = min(t[0] for t in acc)
            if others and best[0] - max(others) <= tol * best[0]:
                want.append((4, best[1], best[2], best[3]))
            if abs(best[0] - gamma * (best[0] - gmin)) <= tol * best[0]:
                want.append((5, best[1], best[2], best[3]))
        assert got == sorted(want), step
        assert np.all(nl["step"][before:] == step)
