"""Unstructured Q4 path (mct_set_mesh_q4) on the GPU against the CPU oracle.

Bar (as for the triangle path): the split log, split codes, tips and the
displacement / velocity fields bit-identical to the oracle's after every
checked step count, with and without HIP graphs, in both tracking modes and
with the per-front pick; queried forces, stresses and accelerations to
1e-12 relative, energies (sums in another order) to 1e-12 relative.  A
structured grid written as an unstructured mesh (renumbered, node lists
rotated) runs the structured path's crack sequence."""
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


@pytest.mark.parametrize("name", sorted(W.quad_small_cases()))
def test_q4u_matches_oracle(gpu, oracle_mod, name, monkeypatch):
    cfg = W.quad_small_cases()[name]
    print("case", name, flush=True)
    o = oracle_mod.Oracle(cfg)
    # the element kernel plus the node kernel (1), the fused kernel on 64-,
    # 128-, 256-node patches (2, 3, 4), on 77-node patches (not a multiple of
    # the wavefront, the last one ragged) and on patches of the size the
    # library finds
    models = [gpu.from_config(cfg, tile=t, use_graph=g) for t, g in ((1, False), (2, True), (3, False), (4, True))]
    assert [m.launch()["tile"] for m in models] == [1, 2, 3, 4]
    nn = models[0].info()["n_nodes"]
    monkeypatch.setenv("MCT_PATCH_NODES", "77")
    sized = gpu.from_config(cfg, tile=5, use_graph=True)
    monkeypatch.delenv("MCT_PATCH_NODES")
    assert sized.launch()["tile"] == 5 and sized.launch()["workgroups"] == -(-nn // 77), sized.launch()
    auto = gpu.from_config(cfg, tile=5, use_graph=False)
    assert auto.launch()["tile"] in (2, 3, 4, 5), auto.launch()
    print(name, "automatic patches", auto.launch(), flush=True)
    models += [sized, auto]
    assert gpu.from_config(cfg).launch() == auto.launch()  # the automatic choice
    inf = models[0].info()
    assert (inf["n_nodes"], inf["n_elems"], inf["n_edges"]) == (o.info()["nn"], o.info()["ne"], o.info()["ns"])
    assert inf["dt"] == o.info()["dt"]
    done = 0
    for chunk in (1, 63, 136, 400, 600):
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


def test_q4u_sct_and_front_pick(gpu, oracle_mod):
    base = W.quad_small_cases()["grid70x37_unstructured"]
    for cfg, label in ((dict(base, tracking=("sct", -1, 0)), "sct"), (dict(base, front_radius=2.5e-3), "front")):
        print("case", label, flush=True)
        o = oracle_mod.Oracle(cfg)
        # the element plus node kernels, and the fused kernel (whose step is
        # then followed by the pick's own launch)
        models = [gpu.from_config(cfg, tile=t) for t in (1, 5)]
        assert [m.launch()["tile"] for m in models][0] == 1 and models[1].launch()["tile"] != 1
        if label == "sct":
            assert all(m.tip() == o.tip() for m in models) and o.tip() is not None
        for chunk in (100, 501, 599):
            o.step(chunk)
            for m in models:
                m.step(chunk)
                _same(m, o, (label, chunk, m.launch()["tile"]))
                if label == "sct":
                    assert m.tip() == o.tip()
        assert len(o.log()["elem"]) > 3, label


def test_q4u_is_the_structured_grid(gpu):
    """The renumbered grid cracks like the structured grid: the same steps,
    elements (through the permutation), local edges (through the rotation)
    and G to 1e-9 (sums of another order)."""
    base = W.small_cases()["plate70x37_jitter"]
    u = W.as_unstructured_q4(base)
    pn, pe, rot = u["perm"]
    a = gpu.from_config(base)
    b = gpu.from_config(u)
    a.step(900)
    b.step(900)
    la, lb = a.crack_set(), b.crack_set()
    n = 10
    assert len(la["elem"]) > n
    assert np.array_equal(lb["step"][:n], la["step"][:n])
    assert np.array_equal(pe[lb["elem"][:n]], la["elem"][:n])
    r = rot[lb["elem"][:n]]
    assert np.array_equal((lb["entry"][:n].astype(np.int64) + r) % 4, la["entry"][:n])
    assert np.array_equal((lb["exit"][:n].astype(np.int64) + r) % 4, la["exit"][:n])
    np.testing.assert_allclose(lb["G"][:n], la["G"][:n], rtol=1e-9)


def _edge_index(tabs, ne):
    ee = np.full((ne, 4), -1, np.int64)
    for s in range(len(tabs["edge_elem"])):
        for side in range(2):
            e = tabs["edge_elem"][s, side]
            if e >= 0:
                ee[e, tabs["edge_loc"][s, side]] = s
    return ee


@pytest.mark.parametrize("name", sorted(W.quad_small_cases()))
def test_q4u_fields_and_energies(gpu, oracle_mod, name):
    cfg = W.quad_small_cases()[name]
    steps = 800
    m = gpu.from_config(cfg)
    o = oracle_mod.Oracle(cfg)
    m.step(steps)
    o.step(steps)
    st = o.state()
    assert (st["split"] != 0).sum() > len(cfg["notch"][0])  # a cracked state
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
    mean = sig[ee[intact]].sum(axis=1) / 4.0
    c = 0.5 * (mean[:, 0] + mean[:, 1])
    r = np.sqrt((0.5 * (mean[:, 0] - mean[:, 1])) ** 2 + mean[:, 2] ** 2)
    np.testing.assert_allclose(gp[intact], c + r, rtol=1e-12, atol=1e-12 * smax)
    ge, oe = m.energies(), o.energies()
    print(name, ge, oe, flush=True)
    for k in ("kin", "strain", "wext"):
        assert ge[k] == pytest.approx(oe[k], rel=1e-12, abs=1e-300), k
    assert ge["Ud"] == pytest.approx(oe["Ud"], rel=1e-12)


def test_q4u_checkpoint_restore(gpu):
    cfg = W.quad_small_cases()["quad_plate24x10"]
    a = gpu.from_config(cfg)
    a.step(451)  # odd: the state sits in the second displacement buffer
    ck = a.checkpoint()
    a.step(400)
    b = gpu.from_config(cfg, use_graph=False)
    b.restore(ck)
    b.step(400)
    la, lb = a.crack_set(), b.crack_set()
    for k in ("step", "elem", "entry", "exit", "G"):
        assert np.array_equal(la[k], lb[k])
    assert np.array_equal(a.field(0)[0], b.field(0)[0]) and np.array_equal(a.field(1)[1], b.field(1)[1])
    assert a.info()["dissipated"] == b.info()["dissipated"]
    # the fused kernel takes the same checkpoint and continues alike, and its
    # own checkpoint restores into the split kernels
    f = gpu.from_config(cfg, tile=5)
    f.restore(ck)
    f.step(200)
    ckf = f.checkpoint()
    f.step(200)
    g = gpu.from_config(cfg, tile=1)
    g.restore(ckf)
    g.step(200)
    for m in (f, g):
        lm = m.crack_set()
        for k in ("step", "elem", "entry", "exit", "G"):
            assert np.array_equal(la[k], lm[k]), (m.launch(), k)
        assert np.array_equal(a.field(0)[0], m.field(0)[0]) and np.array_equal(a.field(1)[1], m.field(1)[1])
        assert a.info()["dissipated"] == m.info()["dissipated"]
    # another mesh does not take it
    with pytest.raises(gpu.MctError):
        gpu.from_config(W.quad_small_cases()["grid70x37_unstructured"]).restore(ck)


def test_q4u_invalid_meshes(gpu):
    X = np.array([0.0, 1.0, 2.0, 0.0, 1.0, 2.0])
    Y = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    good = np.array([[0, 1, 4, 3], [1, 2, 5, 4]], np.int32)
    m = gpu.Model()
    m.set_mesh_q4(X, Y, good)
    # a dart: positive area, but it turns right at its third corner
    dart = (np.array([0.0, 2.0, 0.5, 0.0]), np.array([0.0, 0.0, 0.5, 2.0]), np.array([[0, 1, 2, 3]], np.int32))
    for xx, yy, conn in ((X, Y, good[:, [0, 3, 2, 1]]),  # clockwise
                         (X, Y, np.array([[0, 1, 1, 3], [1, 2, 5, 4]], np.int32)),  # repeated node
                         (X, Y, np.array([[0, 1, 4, 3], [1, 2, 5, 6]], np.int32)),  # out of range
                         (X, Y, np.array([[0, 1, 4, 3], [0, 1, 4, 3]], np.int32)),  # edges reused one way
                         dart):  # not convex
        with pytest.raises(gpu.MctError):
            m.set_mesh_q4(xx, yy, conn)
    with pytest.raises(gpu.MctError):  # a node in no element
        m.set_mesh_q4(np.append(X, 3.0), np.append(Y, 3.0), good)
    m.set_mesh_q4(X, Y, good)
    m.set_notch(np.array([0], np.int32), np.array([3], np.uint8), np.array([1], np.uint8))  # edges 0..3
    with pytest.raises(gpu.MctError):
        m.set_notch(np.array([0], np.int32), np.array([4], np.uint8), np.array([1], np.uint8))
    with pytest.raises(gpu.MctError):  # sub-cell smoothing: structured grids only
        m.set_smoothing("subcell")
    with pytest.raises(gpu.MctError):  # plain binary64 contexts only
        gpu.Model(precision=32).set_mesh_q4(X, Y, good)
    with pytest.raises(gpu.MctError):
        gpu.Model(n_specimens=2).set_mesh_q4(X, Y, good)


def test_q4u_fullsize_plate(gpu, oracle_mod):
    """The unstructured Q4 benchmark mesh (about 160 000 quadrilaterals split
    from Delaunay triangles) for 300 steps, as timed: bit-identical fields."""
    cfg = W.quad_plate160k()
    o = oracle_mod.Oracle(cfg)
    m = gpu.from_config(cfg)
    # the automatic choice (the fused kernel on patches it sizes), as timed
    assert m.launch()["tile"] == 5, m.launch()
    s = gpu.from_config(cfg, tile=1)  # the element kernel plus the node kernel
    f = gpu.from_config(cfg, tile=4)  # the fused kernel that re-derives neighbour strains
    assert s.launch()["tile"] == 1 and f.launch()["tile"] == 4
    o.step(300)
    for x in (m, s, f):
        x.step(300)
    _same(m, o, "quad_plate160k fused, shared strains")
    _same(s, o, "quad_plate160k split")
    _same(f, o, "quad_plate160k fused, 256-node patches")


@pytest.mark.parametrize("kind", ["q4u", "tri"])
def test_unstructured_path_geometry_bitwise(gpu, oracle_mod, kind):
    """mct_get_path_geometry on unstructured meshes: every path of sampled
    elements equals the oracle's normal and length bit for bit; paths a
    triangle does not have are NaN."""
    cfg = (W.quad_small_cases()["quad_plate24x10"] if kind == "q4u"
           else W.tri_small_cases()["tri_plate40x16"])
    nv = np.asarray(cfg["conn"]).shape[1]
    m = gpu.from_config(cfg)
    o = oracle_mod.Oracle(cfg)
    ne = len(cfg["conn"])
    elems = np.unique(np.linspace(0, ne - 1, 97).astype(np.int32))
    g = m.path_geometry(elems)
    for i, e in enumerate(elems):
        for a in range(4):
            for j in range(3):
                if a >= nv or j >= nv - 1:
                    assert np.all(np.isnan(g[i, a, j])), (e, a, j)
                    continue
                k = (a + 1 + j) % nv
                assert np.array_equal(g[i, a, j], o.path_normal(int(e), a, k)), (kind, e, a, k)
    with pytest.raises(gpu.MctError):
        m.path_geometry(np.array([ne], np.int32))


@pytest.mark.parametrize("kind", ["q4u", "tri"])
def test_unstructured_autotune(gpu, oracle_mod, kind):
    """The autotuner of an unstructured mesh times its step-kernel choices,
    keeps the fastest and leaves the state as it was: the run continues
    bit-identical to the oracle."""
    cfg = (W.quad_small_cases()["quad_plate24x10"] if kind == "q4u"
           else W.tri_small_cases()["tri_cylinder_coarse"])
    m = gpu.from_config(cfg)
    o = oracle_mod.Oracle(cfg)
    m.step(400)
    o.step(400)
    r = m.autotune(trial_steps=30)
    print(kind, r, flush=True)
    assert r["tile"] in (1, 2, 3, 4, 5) and r["us_per_step"] > 0
    assert m.launch()["tile"] == r["tile"]
    assert m.info()["step"] == 400
    _same(m, o, (kind, "after autotune"))
    m.step(300)
    o.step(300)
    _same(m, o, (kind, "continued"))


@pytest.mark.parametrize("kind", ["fragment_ramp_weibull", "pulse_curve"])
def test_q4u_loading_variants(gpu, oracle_mod, kind):
    """Renumbered grids under the other loadings: outward edge velocities
    with a ramp and a Weibull Gc field (fragmentation), and a traction
    pulse given by a load curve; bit-identical to the oracle."""
    if kind == "fragment_ramp_weibull":
        base = dict(W.fragmentation(61, 33, 1e-3, seed=W.BASE_SEED + 17, steps=400), t_ramp=5e-6)
    else:
        base = W.pulse_plate(48, 32, 0.048, 0.032, peak=2e6, steps=900, t0=2e-5, tau=4e-5)
    cfg = W.as_unstructured_q4(base)
    o = oracle_mod.Oracle(cfg)
    m = gpu.from_config(cfg)
    done = 0
    for chunk in (1, 99, 300, 500):
        o.step(chunk)
        m.step(chunk)
        done += chunk
        _same(m, o, (kind, done))
    assert len(o.log()["elem"]) > 0, kind
    print(kind, "splits", len(o.log()["elem"]), flush=True)


@pytest.mark.parametrize("nodes", [1, 3, 256])
def test_fused_patch_extremes(gpu, oracle_mod, monkeypatch, nodes):
    """Patch sizes at the ends of the fused kernel's range (one node per
    patch; a few; 256, whose patches take the 512- or 1024-slot kernel), on
    a small triangle and a small quadrilateral case: bit-identical to the
    oracle."""
    for cfg in (W.tri_small_cases()["tri_plate40x16"], W.quad_small_cases()["quad_plate24x10"]):
        o = oracle_mod.Oracle(cfg)
        monkeypatch.setenv("MCT_PATCH_NODES", str(nodes))
        m = gpu.from_config(cfg, tile=5)
        monkeypatch.delenv("MCT_PATCH_NODES")
        nn = m.info()["n_nodes"]
        lau = m.launch()
        assert lau["workgroups"] == -(-nn // nodes), (cfg["name"], lau)
        for chunk in (1, 150, 450):
            o.step(chunk)
            m.step(chunk)
            _same(m, o, (cfg["name"], nodes, chunk))
