"""Pins of the oracle's binary32 build: the same C source compiled with the
step in binary32 (state, strains, stresses, forces, G, the element rule and
the pick), reading the binary64 set-up values (areas, masses, nodal forces,
D, dt) rounded once; times and the load factor stay binary64.

The binary64 oracle is pinned against the paper and closed forms elsewhere;
here the binary32 build is pinned against it and against the mathematics at
binary32 accuracy:
  - it is the binary32 build, and its state and logged G are binary32 values;
  - on identical binary32 inputs (coordinates and displacements rounded to
    binary32, given to both builds) its internal force is the binary64 force
    within a few binary32 rounding errors -- and not equal to it (the step
    really runs in binary32);
  - the patch test holds to binary32 accuracy (uniform edge stress, zero
    interior force on a parallelogram mesh);
  - an uncracked run stays within binary32 drift of the binary64 run, and
    energy is conserved as in binary64;
  - the first splits of the 40 x 40 notched plate are the binary64 ones;
  - the element rule and pick tables decide as in binary64 on values exact
    in binary32.
"""
import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _is_f32(a):
    return np.array_equal(_f32(a), np.asarray(a))


def test_library_is_the_binary32_build(oracle_mod):
    assert oracle_mod.lib(32).orc_precision() == 32
    assert oracle_mod.lib(64).orc_precision() == 64


def test_state_and_log_are_binary32_values(oracle_mod):
    o = oracle_mod.run(dict(W.config1(), precision=32), 600)
    st, lg = o.state(), o.log()
    assert len(lg["elem"]) > 0
    for k in ("ux", "uy", "vx", "vy"):
        assert _is_f32(st[k]), k
    assert _is_f32(lg["G"])
    assert np.abs(st["uy"]).max() > 0


@pytest.mark.parametrize("smooth", [False, True])
def test_internal_force_within_binary32_error(oracle_mod, smooth):
    """Both builds on the same binary32 inputs (the binary64 build gets the
    rounded coordinates): |f32 - f64| <= 5e-5 max|f64|.  Derivation: each
    force is a short sum (4 edges x 2 products) of products of a gradient, a
    stress (3-term fma chains over 4-node strains) and an area; each stage
    adds a few units of 2^-24 = 6e-8 relative to its own magnitude, and the
    cancellation of a smooth field (strain much smaller than |grad||u|)
    multiplies it by about the element count across the field's wavelength
    (here < 100): bound 100 x 8 x 6e-8 = 5e-5.  A cracked state (split
    pieces) is included."""
    cfg = W.small_cases()["plate70x37_jitter"]
    o32 = oracle_mod.Oracle(dict(cfg, precision=32))
    o64 = oracle_mod.Oracle(dict(cfg, X=_f32(cfg["X"]), Y=_f32(cfg["Y"])))
    crack = oracle_mod.run(cfg, 900).state()["split"]
    assert (crack != 0).sum() > 40
    o32.set_split_codes(crack)
    o64.set_split_codes(crack)
    X, Y = cfg["X"], cfg["Y"]
    if smooth:
        ux = _f32(1e-6 * np.sin(3 * X / X.max()))
        uy = _f32(2e-6 * np.cos(2 * Y / Y.max()))
    else:
        rng = np.random.default_rng(1)
        ux = _f32(rng.standard_normal(len(X)) * 1e-6)
        uy = _f32(rng.standard_normal(len(X)) * 1e-6)
    a = o32.internal_force(ux, uy)
    b = o64.internal_force(ux, uy)
    scale = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    err = max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) / scale
    assert err < 5e-5
    assert err > 1e-9  # binary32 arithmetic, not binary64
    assert _is_f32(a[0]) and _is_f32(a[1])


def test_patch_test_to_binary32_accuracy(oracle_mod):
    """Parallelogram mesh (where the point rule is exact): a linear
    displacement gives the exact uniform stress at every edge and zero
    interior force, to binary32 accuracy."""
    nx, ny = 9, 7
    i = np.tile(np.arange(nx + 1, dtype=float), ny + 1)
    j = np.repeat(np.arange(ny + 1, dtype=float), nx + 1)
    X = 1e-3 * (1.0 * i + 0.35 * j)
    Y = 1e-3 * (0.2 * i + 0.8 * j)
    c = W.plate(nx, ny, 1, 1, traction=0.0, notch_len=None)
    c["X"], c["Y"] = X, Y
    c["traction_nodes"] = np.zeros((0, 2), np.int32)
    c["traction"] = np.zeros((0, 2))
    o = oracle_mod.Oracle(dict(c, precision=32))
    ux = 1e-4 + 2e-3 * X - 3e-3 * Y
    uy = -2e-4 + 1.5e-3 * X + 4e-3 * Y
    fx, fy, sig, ok = o.internal_force(ux, uy, with_stress=True)
    E, nu = c["E"], c["nu"]
    D = E / (1 - nu * nu) * np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]])
    s_exp = D @ np.array([2e-3, 4e-3, -3e-3 + 1.5e-3])
    np.testing.assert_allclose(sig, np.broadcast_to(s_exp, sig.shape), rtol=0, atol=2e-5 * np.abs(s_exp).max())
    inner = (i > 0) & (i < nx) & (j > 0) & (j < ny)
    scale = max(np.abs(fx).max(), np.abs(fy).max())
    assert max(np.abs(fx[inner]).max(), np.abs(fy[inner]).max()) < 1e-4 * scale


def test_uncracked_run_tracks_binary64(oracle_mod):
    """Without cracking (Gc huge) the binary32 run stays within binary32
    drift of the binary64 run on the same rounded coordinates: after 500
    steps |u32 - u64| < 1e-4 max|u64| and |v32 - v64| < 1e-3 max|v64|
    (per-step rounding of about 1e-6 of the force, accumulated over the
    steps the wave has travelled)."""
    c = dict(W.config1(), gc_uniform=1e30)
    r32 = oracle_mod.run(dict(c, precision=32), 500)
    r64 = oracle_mod.run(dict(c, X=_f32(c["X"]), Y=_f32(c["Y"])), 500)
    s32, s64 = r32.state(), r64.state()
    assert len(r32.log()["elem"]) == 0
    for k, tol in (("ux", 1e-4), ("uy", 1e-4), ("vx", 1e-3), ("vy", 1e-3)):
        assert np.abs(s32[k] - s64[k]).max() <= tol * np.abs(s64[k]).max(), k


def test_energy_conservation_binary32(oracle_mod):
    c = W.plate(10, 8, 0.010, 0.008, traction=0.0, jitter=0.05, seed=11, gc=1e30, cfl=0.4, notch_len=None)
    c["traction_nodes"] = np.zeros((0, 2), np.int32)
    c["traction"] = np.zeros((0, 2))
    o = oracle_mod.Oracle(dict(c, precision=32))
    X, Y = c["X"], c["Y"]
    bump = np.exp(-((X - 0.004) ** 2 + (Y - 0.005) ** 2) / (2 * 0.002 ** 2))
    o.set_state(1e-7 * bump, -2e-7 * bump, 0 * X, 0 * X)
    e0 = o.energies()
    E0 = e0["kin"] + e0["strain"]
    dev = 0.0
    for _ in range(20):
        o.step(10)
        e = o.energies()
        dev = max(dev, abs(e["kin"] + e["strain"] - E0))
    assert dev / E0 < 3e-2


def test_first_splits_match_binary64(oracle_mod):
    """The notched 40 x 40 plate: the first 40 splits (step, element, entry,
    exit) are the binary64 ones and their G agree to 1e-4 (the fields drift
    apart by about 1e-5 relative over the first few hundred steps, and G is
    a product of displacement and stress); later near-ties may be decided
    differently by the two precisions."""
    c = W.config1()
    l32 = oracle_mod.run(dict(c, precision=32), 2000).log()
    l64 = oracle_mod.run(c, 2000).log()
    assert len(l32["elem"]) > 100 and len(l64["elem"]) > 100
    for k in ("step", "elem", "entry", "exit"):
        assert np.array_equal(l32[k][:40], l64[k][:40]), k
    np.testing.assert_allclose(l32["G"][:40], l64["G"][:40], rtol=1e-4)


RULES = [((4.0, 1.0, 2.0), 3.0, 2.0, 0), ((3.1, 6.2, 1.0), 3.0, 2.0, -1), ((3.25, 6.25, 1.0), 3.0, 2.0, 1),
         ((4.0, 5.0, 9.0), 3.0, 2.0, -1), ((8.0, 5.0, 9.0), 3.0, 2.0, 2), ((1.0, 2.0, 2.5), 3.0, 1.0, -1)]
PICKS = [([4.0, 6.0, 5.0], [1, 2, 3], [0, 0, 0], 1.0, 1), ([6.0, 6.0, 5.0], [9, 2, 3], [0, 0, 0], 1.0, 1),
         ([6.0, 6.0], [4, 4], [3, 1], 1.0, 1), ([3.125, 7.0, 5.0], [1, 2, 3], [0, 0, 0], 2.0, -1)]


def test_rule_and_pick_tables_binary32(oracle_mod):
    for G, Gc, gamma, exp in RULES:
        assert oracle_mod.element_rule(G, Gc, gamma, precision=32) == exp
        assert oracle_mod.element_rule(G, Gc, gamma, precision=64) == exp
    for G, el, a, gamma, exp in PICKS:
        assert oracle_mod.mct_pick(G, el, a, gamma, precision=32) == exp
        assert oracle_mod.mct_pick(G, el, a, gamma, precision=64) == exp


def test_subcell_internal_force_within_binary32_error(oracle_mod):
    """Sub-cell smoothing in the binary32 build: on the same binary32 inputs
    its internal force is the binary64 build's within 5e-5 max|f| (the
    derivation of the point-rule bound applies: short sums of products of
    gradients, stresses and areas), and not equal to it."""
    cfg = dict(W.small_cases()["plate70x37_jitter"], smoothing="subcell")
    o32 = oracle_mod.Oracle(dict(cfg, precision=32))
    o64 = oracle_mod.Oracle(dict(cfg, X=_f32(cfg["X"]), Y=_f32(cfg["Y"])))
    crack = oracle_mod.run(cfg, 900).state()["split"]
    assert (crack != 0).sum() > 40
    o32.set_split_codes(crack)
    o64.set_split_codes(crack)
    rng = np.random.default_rng(4)
    ux = _f32(rng.standard_normal(len(cfg["X"])) * 1e-6)
    uy = _f32(rng.standard_normal(len(cfg["X"])) * 1e-6)
    a = o32.internal_force(ux, uy)
    b = o64.internal_force(ux, uy)
    scale = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    err = max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) / scale
    assert 1e-9 < err < 5e-5
    assert _is_f32(a[0]) and _is_f32(a[1])
