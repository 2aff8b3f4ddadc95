"""Pins of the oracle's sub-cell edge smoothing for Q4 (the alternative to
the point rule: the smoothing domain of an edge is the union of the
triangles (edge, centroid of each intact neighbour), with the displacement
at a centroid the mean of the element's four nodal displacements).

Pinned: on jittered (non-parallelogram) meshes the patch test passes in
full -- exact edge strain *and* zero interior nodal force -- where the point
rule leaves a residual; a static uniaxial solve gives a uniform stress;
the stiffness equals an independent boundary-integral assembly (outward
normals times lengths of the sub-cell sides, shape functions linear along
them); on parallelogram meshes it equals the point rule; symmetry, three
zero modes, rigid-body invariance, the strain-energy identity and
second-order energy conservation; a notched plate cracks.
"""
import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W


def _cfg(nx, ny, lx, ly, *, jitter=0.0, seed=7, notch=0, traction=0.0, X=None, Y=None, subcell=True):
    c = W.plate(nx, ny, lx, ly, traction=traction, jitter=jitter, seed=seed, notch_len=notch or None)
    if traction == 0.0:
        c["traction_nodes"] = np.zeros((0, 2), np.int32)
        c["traction"] = np.zeros((0, 2))
    if X is not None:
        c["X"], c["Y"] = X, Y
    if subcell:
        c["smoothing"] = "subcell"
    return c


def _interior(nx, ny):
    i = np.tile(np.arange(nx + 1), ny + 1)
    j = np.repeat(np.arange(ny + 1), nx + 1)
    return (i > 0) & (i < nx) & (j > 0) & (j < ny)


def _stiffness(o):
    nn = o.info()["nn"]
    K = np.zeros((2 * nn, 2 * nn))
    for d in range(2 * nn):
        u = np.zeros(2 * nn)
        u[d] = 1.0
        fx, fy = o.internal_force(u[0::2].copy(), u[1::2].copy())
        K[0::2, d] = fx
        K[1::2, d] = fy
    return K


def _D(c):
    E, nu = c["E"], c["nu"]
    return E / (1 - nu * nu) * np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]])


def _linear(c):
    X, Y = c["X"], c["Y"]
    a = (1e-4, 2e-3, -3e-3)
    b = (-2e-4, 1.5e-3, 4e-3)
    return a[0] + a[1] * X + a[2] * Y, b[0] + b[1] * X + b[2] * Y, np.array([a[1], b[2], a[2] + b[1]])


@pytest.mark.parametrize("jitter", [0.01, 0.2, 0.35])
def test_full_patch_test_on_jittered_meshes(oracle_mod, jitter):
    nx, ny = 9, 7
    for subcell in (True, False):
        c = _cfg(nx, ny, 0.009, 0.007, jitter=jitter, seed=21, subcell=subcell)
        o = oracle_mod.Oracle(c)
        ux, uy, eps = _linear(c)
        fx, fy, sig, ok = o.internal_force(ux, uy, with_stress=True)
        s_exp = _D(c) @ eps
        np.testing.assert_allclose(sig, np.broadcast_to(s_exp, sig.shape), rtol=1e-9, atol=1e-9 * np.abs(s_exp).max())
        inner = _interior(nx, ny)
        scale = np.abs(np.concatenate([fx, fy])).max()
        resid = max(np.abs(fx[inner]).max(), np.abs(fy[inner]).max()) / scale
        if subcell:
            assert resid < 1e-11, resid
        else:
            assert resid > 1e-5  # the point rule is not consistent on these meshes


def test_uniform_stress_from_static_solve(oracle_mod):
    nx, ny, sig0 = 7, 5, 1.0e6
    c = _cfg(nx, ny, 0.007, 0.005, jitter=0.25, seed=9, traction=sig0)
    o = oracle_mod.Oracle(c)
    K = _stiffness(o)
    f = o.tables()["fext"].reshape(-1)
    fix = [0, 1, 2 * nx + 1]  # corner (0, 0) and y at (lx, 0)
    free = np.setdiff1d(np.arange(len(f)), fix)
    u = np.zeros(len(f))
    u[free] = np.linalg.solve(K[np.ix_(free, free)], f[free])
    _, _, sig, ok = o.internal_force(u[0::2].copy(), u[1::2].copy(), with_stress=True)
    assert ok.all()
    np.testing.assert_allclose(sig[:, 1], sig0, rtol=1e-8)
    assert np.abs(sig[:, [0, 2]]).max() < 1e-8 * sig0


def test_stiffness_equals_boundary_integral_assembly(oracle_mod):
    nx, ny = 5, 4
    c = _cfg(nx, ny, 0.005, 0.004, jitter=0.3, seed=4)
    o = oracle_mod.Oracle(c)
    K = _stiffness(o)
    X, Y = c["X"], c["Y"]
    nn = len(X)
    D = _D(c)
    # sub-cell sides: for each element e and local edge k, the triangle
    # (n_k, n_k+1, centroid); shape-function values linear along each side
    # (nodes: Kronecker, centroid: 1/4 of each node of e)
    edges = {}
    for j in range(ny):
        for i in range(nx):
            e = j * nx + i
            nd = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
            cx, cy = X[nd].mean(), Y[nd].mean()
            for k in range(4):
                a, b = nd[k], nd[(k + 1) % 4]
                key = (min(a, b), max(a, b))
                # corner points and their nodal weight vectors
                Nc = np.zeros(nn)
                Nc[nd] = 0.25
                Na = np.zeros(nn)
                Na[a] = 1.0
                Nb = np.zeros(nn)
                Nb[b] = 1.0
                P = [(X[a], Y[a], Na), (X[b], Y[b], Nb), (cx, cy, Nc)]
                area = 0.5 * ((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]))
                gx = np.zeros(nn)
                gy = np.zeros(nn)
                for s in range(3):  # counter-clockwise sides: outward normal (dy, -dx)
                    p0, p1 = P[s], P[(s + 1) % 3]
                    nxl, nyl = p1[1] - p0[1], -(p1[0] - p0[0])
                    Nmid = 0.5 * (p0[2] + p1[2])
                    gx += Nmid * nxl
                    gy += Nmid * nyl
                ent = edges.setdefault(key, [0.0, np.zeros(nn), np.zeros(nn)])
                ent[0] += area
                ent[1] += gx
                ent[2] += gy
    Kr = np.zeros((2 * nn, 2 * nn))
    for As, gx, gy in edges.values():
        Bs = np.zeros((3, 2 * nn))
        Bs[0, 0::2] = gx / As
        Bs[1, 1::2] = gy / As
        Bs[2, 0::2] = gy / As
        Bs[2, 1::2] = gx / As
        Kr += As * Bs.T @ D @ Bs
    assert np.abs(K - Kr).max() <= 1e-11 * np.abs(Kr).max()
    lam = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert (np.abs(lam) < 1e-9 * lam.max()).sum() == 3
    assert lam.min() > -1e-9 * lam.max()


def test_equals_point_rule_on_parallelograms(oracle_mod):
    nx, ny = 7, 5
    i = np.tile(np.arange(nx + 1, dtype=float), ny + 1)
    j = np.repeat(np.arange(ny + 1, dtype=float), nx + 1)
    X = 1e-3 * (1.0 * i + 0.35 * j)
    Y = 1e-3 * (0.2 * i + 0.8 * j)
    Ks = _stiffness(oracle_mod.Oracle(_cfg(nx, ny, 1, 1, X=X, Y=Y, notch=3)))
    Kp = _stiffness(oracle_mod.Oracle(_cfg(nx, ny, 1, 1, X=X, Y=Y, notch=3, subcell=False)))
    assert np.abs(Ks - Kp).max() <= 1e-12 * np.abs(Kp).max()


def test_rigid_body_and_energy_identity(oracle_mod):
    c = _cfg(9, 7, 0.009, 0.007, jitter=0.2, seed=5, notch=4)
    o = oracle_mod.Oracle(c)
    X, Y = c["X"], c["Y"]
    fmag = np.abs(np.concatenate(o.internal_force(1e-3 * X, 0 * Y))).max()
    for ux, uy in [(np.full_like(X, 1e-4), np.full_like(X, -2e-4)), (-1e-3 * (Y - 0.003), 1e-3 * (X - 0.004))]:
        fx, fy = o.internal_force(ux, uy)
        assert np.abs(np.concatenate([fx, fy])).max() < 1e-11 * fmag
    rng = np.random.default_rng(2)
    ux = rng.standard_normal(len(X)) * 1e-6
    uy = rng.standard_normal(len(X)) * 1e-6
    o.set_state(ux, uy, np.zeros_like(ux), np.zeros_like(ux))
    fx, fy = o.internal_force(ux, uy)
    assert o.energies()["strain"] == pytest.approx(0.5 * (ux @ fx + uy @ fy), rel=1e-12)


def test_energy_conservation_and_cracking(oracle_mod):
    drift = []
    for refine in (1, 2):
        c = _cfg(12, 8, 0.012, 0.008, jitter=0.2, seed=6)
        c["cfl"] = 0.5 / refine
        c["gc_uniform"] = 1e12
        o = oracle_mod.Oracle(c)
        X, Y = c["X"], c["Y"]
        vx = 0.3 * np.sin(np.pi * X / 0.012) * np.cos(np.pi * Y / 0.008)
        vy = -0.2 * np.cos(np.pi * X / 0.012) * np.sin(2 * np.pi * Y / 0.008)
        o.set_state(np.zeros_like(X), np.zeros_like(X), vx, vy)
        e0 = o.energies()
        E0 = e0["kin"] + e0["strain"]
        dev = 0.0
        for _ in range(10):
            o.step(40 * refine)
            e = o.energies()
            dev = max(dev, abs(e["kin"] + e["strain"] - E0) / E0)
        drift.append(dev)
    assert drift[0] < 5e-3 and drift[1] < drift[0] / 2.5
    c = dict(W.small_cases()["plate70x37_jitter"], smoothing="subcell")
    o = oracle_mod.run(c, 800)
    assert len(o.log()["elem"]) > 5
