"""Pins of the split-screen reference (oracle/screen.py) against closed
forms, brute force and finite differences.  CPU only."""
import math

import numpy as np
import pytest

from oracle import screen as S
from paper_2509_01827_amd import workloads as W


# ---------------------------------------------------------------- bfloat16

def test_bf16_round_to_nearest_even():
    one = 1.0
    assert S.bf16(one) == 1.0
    assert S.bf16(1.0 + 2.0 ** -8) == 1.0                      # tie -> even (mantissa 0)
    assert S.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (mantissa 2)
    assert S.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert S.bf16(-1.5) == -1.5
    x = np.array([0.1, -7.3, 1e-3, 12345.678])
    r = S.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)      # half an ulp of an 8-bit mantissa
    assert np.array_equal(S.bf16(r), r)                        # idempotent


# -------------------------------------------------------------------- MLP

def test_gelu_closed_forms():
    assert S.gelu(np.array([0.0]))[0] == 0.0
    assert S.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)  # Phi(1)
    assert S.gelu(np.array([-1.0]))[0] == pytest.approx(-(1 - 0.8413447460685429), rel=1e-14)
    assert S.gelu(np.array([40.0]))[0] == 40.0
    assert S.gelu(np.array([-40.0]))[0] == pytest.approx(0.0, abs=1e-300)
    assert S.gelu_prime(np.array([0.0]))[0] == 0.5
    z = np.array([-2.0, -0.3, 0.7, 3.0])
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_prime(z), fd, rtol=1e-8)


def _rand_params(rng, scale=0.3):
    return rng.normal(0.0, scale, S.N_PARAMS)


def test_forward_matches_neuron_loops():
    """Brute force: every neuron of every layer written out with scalar loops."""
    rng = np.random.default_rng(1)
    p = _rand_params(rng)
    X = rng.normal(size=(3, S.N_IN))
    W1, b1, W2, b2, w3, b3 = S.unpack(p)
    gelu = lambda z: 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))
    want = []
    for r in range(3):
        h1 = [gelu(sum(X[r, i] * W1[i, j] for i in range(S.N_IN)) + b1[j]) for j in range(S.N_H)]
        h2 = [gelu(sum(h1[i] * W2[i, j] for i in range(S.N_H)) + b2[j]) for j in range(S.N_H)]
        want.append(sum(h2[i] * w3[i] for i in range(S.N_H)) + b3)
    np.testing.assert_allclose(S.forward(p, X, emulate_bf16=False), want, rtol=1e-12)


def test_loss_at_zero_logit():
    p = np.zeros(S.N_PARAMS)
    X = np.ones((4, S.N_IN))
    y = np.array([1.0, 0.0, 0.0, 1.0])
    loss, g = S.loss_and_grad(p, X, y, pos_weight=3.0, emulate_bf16=False)
    assert loss == pytest.approx((3 + 1 + 1 + 3) / 4 * math.log(2.0), rel=1e-15)
    # d/db3 = mean(w (sigmoid(0) - y))
    assert g[-1] == pytest.approx((3 * -0.5 + 0.5 + 0.5 + 3 * -0.5) / 4, rel=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = _rand_params(rng)
    X = rng.normal(size=(7, S.N_IN))
    y = (rng.random(7) < 0.4).astype(float)
    _, g = S.loss_and_grad(p, X, y, pos_weight=2.5, emulate_bf16=False)
    idx = np.concatenate([rng.choice(S.N_PARAMS, 60, replace=False), [S.N_PARAMS - 1, 0, 640, 704]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (S.loss_and_grad(pp, X, y, 2.5, False)[0] - S.loss_and_grad(pm, X, y, 2.5, False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=2e-6, abs=1e-10), i


def test_bf16_emulation_changes_little():
    rng = np.random.default_rng(3)
    p = _rand_params(rng)
    X = rng.normal(size=(50, S.N_IN))
    a = S.forward(p, X, emulate_bf16=False)
    b = S.forward(p, X, emulate_bf16=True)
    assert np.abs(a - b).max() < 0.05 * np.abs(a).max()
    assert not np.array_equal(a, b)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(size=S.N_PARAMS)
    g = rng.normal(size=S.N_PARAMS)
    z = np.zeros(S.N_PARAMS)
    p1, m, v = S.adam(p, g, z, z, 1, lr=1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


# ---------------------------------------------------------------- features

def _plate(nx=8, ny=6):
    return W.plate(nx, ny, nx * 1e-3, ny * 1e-3, traction=0.0)


def _set_u(o, ux, uy):
    z = np.zeros_like(ux)
    o.set_state(ux, uy, z, z)


def test_features_uniaxial_tension_closed_form(oracle_mod):
    c = _plate()
    o = oracle_mod.Oracle(c)
    E, nu, gc = c["E"], c["nu"], c["gc_uniform"]
    eps = 1e-4
    X, Y = c["X"], c["Y"]
    _set_u(o, eps * X, -nu * eps * Y)           # sigma_xx = E eps, sigma_yy = 0
    elem, a, F, _ = S.features(o, c)
    assert len(elem) == 2 * (8 + 6)             # the domain boundary only
    h = 1e-3
    sref = math.sqrt(E * gc / h)
    np.testing.assert_allclose(F[:, 0], E * eps / sref, rtol=1e-9)
    np.testing.assert_allclose(F[:, 1], 0.0, atol=1e-9 * E * eps / sref)
    np.testing.assert_allclose(F[:, 2], 0.5 * E * eps * eps * h / gc, rtol=1e-9)
    # edges along y (a = 1, 3) are shortened (Poisson) -> not stretched: G = 0
    assert np.all(F[(a == 1) | (a == 3), 3] == 0.0)
    assert np.all(F[(a == 0) | (a == 2), 3] != 0.0)
    assert np.all(F[:, 4] == 0.0)
    assert np.all(F[:, 5] == 1.0)               # no crack tips
    # the outward flags: element 0 has the outside below and left
    r0 = np.where((elem == 0) & (a == 0))[0][0]
    assert list(F[r0, 6:]) == [1.0, 0.0, 0.0, 1.0]


def test_features_pure_shear_closed_form(oracle_mod):
    c = _plate()
    o = oracle_mod.Oracle(c)
    E, nu, gc = c["E"], c["nu"], c["gc_uniform"]
    g = 2e-4
    X, Y = c["X"], c["Y"]
    _set_u(o, 0.5 * g * Y, 0.5 * g * X)         # gamma_xy = g
    _, _, F, _ = S.features(o, c)
    tau = E / (2 * (1 + nu)) * g
    sref = math.sqrt(E * gc / 1e-3)
    np.testing.assert_allclose(F[:, 0], tau / sref, rtol=1e-9)
    np.testing.assert_allclose(F[:, 1], -tau / sref, rtol=1e-9)
    np.testing.assert_allclose(F[:, 2], tau * tau * (1 + nu) / E * 1e-3 / gc, rtol=1e-9)


def test_features_tips_flags_and_history(oracle_mod):
    nx, ny = 8, 6
    c = _plate(nx, ny)
    o = oracle_mod.Oracle(c)
    codes = np.zeros(nx * ny, np.uint8)
    i0, j0 = 5, 2
    codes[j0 * nx + i0] = 0x80 | (3 << 2) | 1   # split left -> right
    o.set_split_codes(codes)
    X, Y = c["X"], c["Y"]
    _set_u(o, 1e-4 * X, 1e-4 * Y)
    elem, a, F, g1 = S.features(o, c)
    key = {(int(e), int(k)): r for r, (e, k) in enumerate(zip(elem, a))}
    # path ends: the left and right edges of the split element (entry 3,
    # exit 1), midpoints (5h, 2.5h) and (6h, 2.5h)
    h = 1e-3
    np.testing.assert_allclose(S.path_ends(nx, ny, c["X"], c["Y"], codes), [(5 * h, 2.5 * h), (6 * h, 2.5 * h)],
                               rtol=1e-14)
    # the four neighbours of the split element see it across the facing edge
    for (ni, nj, k, dist) in ((i0, j0 - 1, 2, math.sqrt(0.5)), (i0 + 1, j0, 3, 0.0),
                              (i0, j0 + 1, 0, math.sqrt(0.5)), (i0 - 1, j0, 1, 0.0)):
        r = key[(nj * nx + ni, k)]
        assert F[r, 5] == pytest.approx(dist / 64.0, rel=1e-12, abs=1e-15)
        assert F[r, 6 + k] == 1.0
    # element 0, bottom edge midpoint (0.5h, 0); nearest end (5h, 2.5h)
    r = key[(0, 0)]
    assert F[r, 5] == pytest.approx(math.hypot(4.5, 2.5) / 64.0, rel=1e-12)
    # a crack reaching the domain boundary has no end there
    codes2 = np.zeros(nx * ny, np.uint8)
    codes2[0] = 0x80 | (3 << 2) | 1            # element 0, left (boundary) -> right
    assert len(S.path_ends(nx, ny, c["X"], c["Y"], codes2)) == 1
    # the previous-evaluation feature carries the last call's G / Gc
    _, _, F2, _ = S.features(o, c, g_prev=g1)
    np.testing.assert_array_equal(F2[:, 4], F[:, 3])
