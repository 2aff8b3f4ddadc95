"""Pins of the oracle on unstructured Q4 meshes (general connectivity).

The structured grid is pinned against the paper elsewhere; an unstructured
mesh that is the same grid with nodes and elements renumbered and each
element's node list rotated must give the same mechanics: the same internal
force and edge stresses (to the rounding of a different summation order), the
same run up to the first splits, which map to the same elements and edges.
On a mesh of quadrilaterals split from triangles (irregular valences): rigid
body motions give no force, the stiffness is symmetric positive
semi-definite with exactly three zero modes, energy is conserved to second
order, and the notched plate cracks along its notch line.
"""
import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W


def _maps(c):
    pn, pe, rot = c["perm"]
    inv_n = np.empty_like(pn)
    inv_n[pn] = np.arange(len(pn))
    inv_e = np.empty_like(pe)
    inv_e[pe] = np.arange(len(pe))
    return pn, pe, rot, inv_n, inv_e


def test_renumbered_grid_internal_force(oracle_mod):
    base = W.small_cases()["plate70x37_jitter"]
    u = W.as_unstructured_q4(base)
    pn, pe, rot, inv_n, inv_e = _maps(u)
    ob = oracle_mod.run(base, 700)   # a cracked state
    st = ob.state()
    ou = oracle_mod.Oracle(u)
    codes = np.zeros(len(pe), np.uint8)
    for e_new in range(len(pe)):
        c = st["split"][pe[e_new]]
        if c:
            r = rot[e_new]
            codes[e_new] = 0x80 | ((((c >> 2) & 3) - r) % 4) << 2 | (((c & 3) - r) % 4)
    assert (codes != 0).sum() > 40
    ou.set_split_codes(codes)
    rng = np.random.default_rng(3)
    ux = rng.standard_normal(len(pn)) * 1e-6
    uy = rng.standard_normal(len(pn)) * 1e-6
    fb = ob.internal_force(ux, uy)
    fu = ou.internal_force(ux[pn], uy[pn])
    scale = max(np.abs(fb[0]).max(), np.abs(fb[1]).max())
    assert np.abs(fu[0] - fb[0][pn]).max() <= 1e-13 * scale
    assert np.abs(fu[1] - fb[1][pn]).max() <= 1e-13 * scale


def test_renumbered_grid_run_and_first_splits(oracle_mod):
    base = W.small_cases()["plate70x37_jitter"]
    u = W.as_unstructured_q4(base)
    pn, pe, rot, inv_n, inv_e = _maps(u)
    ob = oracle_mod.run(base, 900)
    ou = oracle_mod.run(u, 900)
    lb, lu = ob.log(), ou.log()
    assert len(lb["elem"]) > 10
    n = 10
    assert np.array_equal(lu["step"][:n], lb["step"][:n])
    assert np.array_equal(pe[lu["elem"][:n]], lb["elem"][:n])
    r = rot[lu["elem"][:n]]
    assert np.array_equal((lu["entry"][:n] + r) % 4, lb["entry"][:n])
    assert np.array_equal((lu["exit"][:n] + r) % 4, lb["exit"][:n])
    np.testing.assert_allclose(lu["G"][:n], lb["G"][:n], rtol=1e-9)
    # fields before the first split agree to the rounding of the sums
    n0 = int(lb["step"][0])
    assert n0 > 50
    ob2 = oracle_mod.run(base, n0)
    ou2 = oracle_mod.run(u, n0)
    sb, su = ob2.state(), ou2.state()
    assert len(ob2.log()["elem"]) == 0
    for k in ("ux", "uy", "vx", "vy"):
        assert np.abs(su[k] - sb[k][pn]).max() <= 1e-10 * np.abs(sb[k]).max(), k


def _stiffness(o, nn):
    K = np.zeros((2 * nn, 2 * nn))
    for d in range(2 * nn):
        v = np.zeros(2 * nn)
        v[d] = 1.0
        fx, fy = o.internal_force(v[0::2].copy(), v[1::2].copy())
        K[0::2, d] = fx
        K[1::2, d] = fy
    return K


def test_split_quads_stiffness_and_rigid_motion(oracle_mod):
    c = W.quad_plate(5, 3, 0.005, 0.003, traction=0.0, notch_len=None)
    o = oracle_mod.Oracle(c)
    nn = len(c["X"])
    K = _stiffness(o, nn)
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    lam = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert (np.abs(lam) < 1e-9 * lam.max()).sum() == 3
    assert lam.min() > -1e-9 * lam.max()
    X, Y = c["X"], c["Y"]
    fmag = np.abs(np.concatenate(o.internal_force(1e-3 * X, 0 * Y))).max()
    for ux, uy in [(np.full_like(X, 1e-4), np.full_like(X, -2e-4)), (-1e-3 * Y, 1e-3 * X)]:
        fx, fy = o.internal_force(ux, uy)
        assert np.abs(np.concatenate([fx, fy])).max() < 1e-11 * fmag


def test_split_quads_energy_conservation(oracle_mod):
    drift = []
    for refine in (1, 2):
        c = W.quad_plate(10, 6, 0.010, 0.006, traction=0.0, notch_len=None, gc=1e12, cfl=0.5 / refine)
        o = oracle_mod.Oracle(c)
        X, Y = c["X"], c["Y"]
        vx = 0.3 * np.sin(np.pi * X / 0.010) * np.cos(np.pi * Y / 0.006)
        vy = -0.2 * np.cos(np.pi * X / 0.010) * np.sin(2 * np.pi * Y / 0.006)
        o.set_state(np.zeros_like(X), np.zeros_like(X), vx, vy)
        e0 = o.energies()
        E0 = e0["kin"] + e0["strain"]
        dev = 0.0
        for _ in range(10):
            o.step(30 * refine)
            e = o.energies()
            dev = max(dev, abs(e["kin"] + e["strain"] - E0) / E0)
        drift.append(dev)
    assert drift[0] < 5e-3 and drift[1] < drift[0] / 2.5


def test_split_quads_plate_cracks_from_the_notch(oracle_mod):
    c = W.quad_small_cases()["quad_plate24x10"]
    o = oracle_mod.run(c, c["steps"])
    lg = o.log()
    assert len(lg["elem"]) > 5
    Q, X, Y = c["conn"], c["X"], c["Y"]
    # the first split is an element touching the notch tip region (right of
    # the notched strip, near its line)
    first = lg["elem"][0]
    cx, cy = X[Q[first]].mean(), Y[Q[first]].mean()
    assert 0.045 < cx < 0.065 and abs(cy - 0.02) < 0.006
