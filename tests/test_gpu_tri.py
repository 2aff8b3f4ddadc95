"""CST (unstructured triangle mesh) path on the GPU against the CPU oracle.

Bar: the split log, split codes, tips and the displacement / velocity
fields bit-identical to the oracle's after every checked step count, with
and without HIP graphs, in both tracking modes; queried forces and stresses
to 1e-12 relative, energies (sums in another order) to 1e-12 relative; the
stability limit against a dense eigenvalue computation."""
import math

import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_01827_amd import mct2d
    mct2d.load()
    return mct2d


def _same(m, o, label):
    lg, ol = m.crack_set(), o.log()
    for k in ("step", "elem", "entry", "exit"):
        assert np.array_equal(lg[k].astype(np.int64), ol[k].astype(np.int64)), (label, k)
    assert np.array_equal(lg["G"], ol["G"]), label
    st = o.state()
    assert np.array_equal(m.split_codes(), st["split"]), label
    (ux, uy), (vx, vy) = m.field(0), m.field(1)
    for a, b, name in ((ux, st["ux"], "ux"), (uy, st["uy"], "uy"), (vx, st["vx"], "vx"), (vy, st["vy"], "vy")):
        assert np.array_equal(a, b), (label, name, np.abs(a - b).max())
    inf = m.info()
    assert inf["n_splits"] == len(ol["elem"])
    assert inf["dissipated"] == o.info()["Ud"], label


@pytest.mark.parametrize("name", sorted(W.tri_small_cases()))
def test_tri_matches_oracle(gpu, oracle_mod, name, monkeypatch):
    cfg = W.tri_small_cases()[name]
    o = oracle_mod.Oracle(cfg)
    # split step kernels (1), fused on 64-, 128-, 256-node patches (2, 3, 4)
    models = [gpu.from_config(cfg, tile=t, use_graph=g) for t in (1, 2, 3, 4) for g in (True, False)]
    assert [m.launch()["tile"] for m in models] == [1, 1, 2, 2, 3, 3, 4, 4]
    # fused on 77-node patches (not a multiple of the wavefront, the last one
    # ragged), and on patches of the size the library finds
    nn = models[0].info()["n_nodes"]
    monkeypatch.setenv("MCT_PATCH_NODES", "77")
    sized = [gpu.from_config(cfg, tile=5, use_graph=g) for g in (True, False)]
    monkeypatch.delenv("MCT_PATCH_NODES")
    for m in sized:
        lau = m.launch()
        assert lau["tile"] == 5 and lau["workgroups"] == -(-nn // 77), lau
    auto = gpu.from_config(cfg)
    assert auto.launch()["tile"] in (2, 3, 5), auto.launch()
    print(name, "automatic patches", auto.launch(), flush=True)
    models += sized + [auto]
    inf = models[0].info()
    assert (inf["n_nodes"], inf["n_elems"], inf["n_edges"]) == (o.info()["nn"], o.info()["ne"], o.info()["ns"])
    assert inf["dt"] == o.info()["dt"]
    done = 0
    for chunk in (1, 63, 136, 400):
        o.step(chunk)
        done += chunk
        for m in models:
            m.step(chunk)
            m.sync()
            _same(m, o, (name, done, m.launch()["tile"]))
    e, xy = models[0].tips()
    oe, oxy = o.tips()
    assert np.array_equal(e, oe) and np.array_equal(xy, oxy)
    assert len(o.log()["elem"]) > 5, "the case should crack within the checked steps"
    print(name, "splits", len(o.log()["elem"]), flush=True)


def _shuffled_nodes(cfg, seed):
    """The same mesh with its node ids in a seeded random order (element ids
    and each triangle's node order kept)."""
    nn = len(cfg["X"])
    pn = np.argsort(W.uniform01(seed, nn), kind="stable")  # new id -> old id
    inv = np.empty(nn, np.int64)
    inv[pn] = np.arange(nn)
    vn, vm, vv = cfg["vbc"]
    return dict(cfg, name=cfg["name"] + "_shuffled", X=np.ascontiguousarray(cfg["X"][pn]),
                Y=np.ascontiguousarray(cfg["Y"][pn]),
                conn=np.ascontiguousarray(inv[np.asarray(cfg["conn"], np.int64)].astype(np.int32)),
                traction_nodes=np.ascontiguousarray(inv[np.asarray(cfg["traction_nodes"], np.int64)].astype(np.int32)),
                vbc=(np.ascontiguousarray(inv[np.asarray(vn, np.int64)].astype(np.int32)), vm, vv))


def test_tri_shuffled_nodes(gpu, oracle_mod, monkeypatch):
    """Node ids without locality: the fused kernel's patches of consecutive
    nodes scatter, their rings and staged node lists overflow what the
    shared-strain kernel holds, and every launch choice falls back (to the
    kernel that re-derives neighbour strains, or to the split kernels) with
    results still equal to the oracle's on the same mesh."""
    cfg = _shuffled_nodes(W.tri_small_cases()["tri_plate40x16"], W.BASE_SEED + 120)
    o = oracle_mod.Oracle(cfg)
    models = [gpu.from_config(cfg, tile=t) for t in (0, 1, 2)]
    monkeypatch.setenv("MCT_PATCH_NODES", "16")  # small patches: 512-slot kernel or the shared one
    models.append(gpu.from_config(cfg, tile=5))
    monkeypatch.delenv("MCT_PATCH_NODES")
    print("launches", [m.launch() for m in models], flush=True)
    for chunk in (1, 299, 700):
        o.step(chunk)
        for m in models:
            m.step(chunk)
            _same(m, o, ("shuffled", chunk, m.launch()))
    assert len(o.log()["elem"]) > 3


def test_tri_sct_matches_oracle(gpu, oracle_mod):
    cfg = dict(W.tri_small_cases()["tri_plate40x16"], tracking=("sct", -1, 0))
    o = oracle_mod.Oracle(cfg)
    models = [gpu.from_config(cfg, tile=t) for t in (0, 1)]
    assert models[0].tip() == o.tip() and o.tip() is not None
    for chunk in (100, 501, 900):
        o.step(chunk)
        for m in models:
            m.step(chunk)
            _same(m, o, ("sct", chunk, m.launch()["tile"]))
            assert m.tip() == o.tip()
    assert len(o.log()["elem"]) > 3


def test_tri_checkpoint_restore(gpu):
    cfg = W.tri_small_cases()["tri_cylinder_coarse"]
    a = gpu.from_config(cfg)
    a.step(151)  # odd: the state sits in the second displacement buffer
    ck = a.checkpoint()
    a.step(200)
    b = gpu.from_config(cfg, tile=1)  # split step kernels resume the fused run
    b.restore(ck)
    b.step(77)
    b.set_launch(3)  # and hand over to the fused kernel mid-run
    b.step(123)
    assert b.launch()["tile"] == 3
    la, lb = a.crack_set(), b.crack_set()
    for k in ("step", "elem", "entry", "exit", "G"):
        assert np.array_equal(la[k], lb[k])
    assert np.array_equal(a.field(0)[0], b.field(0)[0]) and np.array_equal(a.field(1)[1], b.field(1)[1])
    assert a.info()["dissipated"] == b.info()["dissipated"]
    with pytest.raises(gpu.MctError):
        gpu.from_config(W.tri_small_cases()["tri_fragment"]).restore(ck)


def _edge_index(tabs, ne):
    ee = np.full((ne, 3), -1, np.int64)
    for s in range(len(tabs["edge_elem"])):
        for side in range(2):
            e = tabs["edge_elem"][s, side]
            if e >= 0:
                ee[e, tabs["edge_loc"][s, side]] = s
    return ee


@pytest.mark.parametrize("name", ["tri_plate40x16", "tri_cylinder_coarse", "tri_fragment"])
def test_tri_fields_and_energies(gpu, oracle_mod, name):
    cfg = W.tri_small_cases()[name]
    steps = 300
    m = gpu.from_config(cfg)
    o = oracle_mod.Oracle(cfg)
    m.step(steps)
    o.step(steps)
    st = o.state()
    fx, fy, sig, ok = o.internal_force(st["ux"], st["uy"], with_stress=True)
    scale = max(np.abs(fx).max(), np.abs(fy).max())
    gx, gy = m.field(gpu.FIELD_FINT)
    assert np.abs(gx - fx).max() <= 1e-12 * scale and np.abs(gy - fy).max() <= 1e-12 * scale
    gs = m.field(gpu.FIELD_SIGMA_EDGE)
    okb = ok.astype(bool)
    assert np.all(np.isnan(gs[~okb]))
    smax = np.abs(sig[okb]).max()
    assert np.abs(gs[okb] - sig[okb]).max() <= 1e-12 * smax
    tabs = o.tables()
    phi = o.load_factor(steps * o.info()["dt"])
    fe = tabs["fext"]
    ax = (phi * fe[:, 0] - fx) / tabs["mass"]
    ay = (phi * fe[:, 1] - fy) / tabs["mass"]
    nodes, masks, _ = cfg["vbc"]
    for n, mk in zip(nodes, masks):
        if mk & 1:
            ax[n] = 0.0
        if mk & 2:
            ay[n] = 0.0
    ga, gb = m.field(gpu.FIELD_A)
    amax = max(np.abs(ax).max(), np.abs(ay).max())
    assert np.abs(ga - ax).max() <= 1e-11 * amax and np.abs(gb - ay).max() <= 1e-11 * amax
    ne = o.info()["ne"]
    ee = _edge_index(tabs, ne)
    split = st["split"]
    gp = m.field(gpu.FIELD_PRINCIPAL)
    assert np.all(np.isnan(gp[split != 0]))
    intact = np.where(split == 0)[0]
    mean = sig[ee[intact]].sum(axis=1) / 3.0
    c = 0.5 * (mean[:, 0] + mean[:, 1])
    r = np.sqrt((0.5 * (mean[:, 0] - mean[:, 1])) ** 2 + mean[:, 2] ** 2)
    np.testing.assert_allclose(gp[intact], c + r, rtol=1e-12, atol=1e-12 * smax)
    ge, oe = m.energies(), o.energies()
    print(name, ge, oe, flush=True)
    for k in ("kin", "strain", "wext"):
        assert ge[k] == pytest.approx(oe[k], rel=1e-12, abs=1e-300), k
    assert ge["Ud"] == pytest.approx(oe["Ud"], rel=1e-12)


def _dense_limit(oracle_mod, cfg):
    o = oracle_mod.Oracle(cfg)
    nn = o.info()["nn"]
    mass = o.tables()["mass"]
    free = np.ones(2 * nn, bool)
    nodes, masks, _ = cfg["vbc"]
    for n, mk in zip(nodes, masks):
        if mk & 1:
            free[n] = False
        if mk & 2:
            free[nn + n] = False
    K = np.zeros((2 * nn, 2 * nn))
    for col in range(2 * nn):
        u = np.zeros(2 * nn)
        u[col] = 1.0
        fx, fy = o.internal_force(u[:nn], u[nn:])
        K[:, col] = np.concatenate([fx, fy])
    minv = 1.0 / np.concatenate([mass, mass])
    A = (minv[:, None] * K)[np.ix_(free, free)]
    lam = np.max(np.real(np.linalg.eigvals(A)))
    return 2.0 / math.sqrt(lam)


@pytest.mark.parametrize("kind", ["notched", "velocity_bc"])
def test_tri_stability_limit(gpu, oracle_mod, kind):
    if kind == "notched":
        cfg = W.tri_plate(9, 6, 0.009, 0.006, notch_len=0.004, steps=10)
    else:
        cfg = W.tri_fragment(8, 6, 1e-3, steps=10)
    want = _dense_limit(oracle_mod, cfg)
    m = gpu.from_config(cfg)
    got = m.info()["dt_limit"]
    print(kind, "dt", m.info()["dt"], "limit", got, "dense", want, flush=True)
    assert got == pytest.approx(want, rel=2e-3)
    assert got >= want * (1 - 1e-9)
    with pytest.raises(gpu.MctError, match="stability"):
        gpu.from_config(dict(cfg, dt=1.02 * want))
    gpu.from_config(dict(cfg, dt=0.97 * want)).close()


def test_tri_invalid_meshes(gpu):
    X = np.array([0.0, 1.0, 1.0, 0.0, 0.5])
    Y = np.array([0.0, 0.0, 1.0, 1.0, 0.5])
    good = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32)
    m = gpu.Model()
    m.set_mesh_tri(X, Y, good)
    for conn in (good[:, [0, 2, 1]], np.array([[0, 1, 1], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32),
                 np.array([[0, 1, 4], [0, 1, 4], [2, 3, 4], [3, 0, 4]], np.int32),
                 np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4], [0, 1, 2]], np.int32),
                 np.array([[0, 1, 5], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32)):
        with pytest.raises(gpu.MctError):
            m.set_mesh_tri(X, Y, conn)
    with pytest.raises(gpu.MctError):  # a node in no triangle
        m.set_mesh_tri(np.append(X, 2.0), np.append(Y, 2.0), good)
    m.set_mesh_tri(X, Y, good)
    for bad in (-1, 6):  # step kernel choices are 0..5
        with pytest.raises(gpu.MctError):
            m.set_launch(bad, True)
    with pytest.raises(gpu.MctError):  # notch local edges are 0..2
        m.set_notch(np.array([0], np.int32), np.array([3], np.uint8), np.array([1], np.uint8))
    with pytest.raises(gpu.MctError):  # no batches of triangle meshes
        b = gpu.Model(n_specimens=2)
        b.set_mesh_tri(X, Y, good)


def test_tri_fullsize_plate_sampled(gpu, oracle_mod):
    """The CST benchmark mesh (Delaunay plate of 633 x 254 points, 320 000
    triangles) for 300 steps: bit-identical fields."""
    cfg = W.tri_plate320k()
    o = oracle_mod.Oracle(cfg)
    m = gpu.from_config(cfg)
    # the automatic choice (the fused kernel on its largest patches of at most
    # 256 elements), as timed
    assert m.launch()["tile"] == 5, m.launch()
    s = gpu.from_config(cfg, tile=1)  # the split kernels
    f = gpu.from_config(cfg, tile=2)  # the fused kernel on 64-node patches
    assert s.launch()["tile"] == 1 and f.launch()["tile"] == 2
    o.step(300)
    for x in (m, s, f):
        x.step(300)
    _same(m, o, "tri_plate320k sized patches")
    _same(s, o, "tri_plate320k split")
    _same(f, o, "tri_plate320k fused")
