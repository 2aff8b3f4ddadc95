"""Per-front pick on the GPU against the CPU oracle (Q4 grid and CST mesh,
the one-workgroup pick of small models and the pick over the whole GPU of
models from 16 384 elements on): split logs, codes and fields
bit-identical, with graph and direct launches;
rho = infinity equals the global pick; errors for the combinations the
variant excludes."""
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
    for k in ("step", "elem", "entry", "exit", "G"):
        assert np.array_equal(lg[k], ol[k].astype(lg[k].dtype)), (label, k)
    st = o.state()
    assert np.array_equal(m.split_codes(), st["split"]), label
    (ux, uy), (vx, vy) = m.field(0), m.field(1)
    assert np.array_equal(ux, st["ux"]) and np.array_equal(uy, st["uy"]), label
    assert np.array_equal(vx, st["vx"]) and np.array_equal(vy, st["vy"]), label
    assert m.info()["dissipated"] == o.info()["Ud"], label


def _double_notch(nx=40, ny=21, h=1e-3, ln=10, steps=700):
    c = W.plate(nx, ny, nx * h, ny * h, steps=steps, name="double_notch")
    row = ny // 2
    el = [row * nx + i for i in range(ln)] + [row * nx + nx - 1 - i for i in range(ln)]
    c["notch"] = (np.array(el, np.int32), np.array([3] * ln + [1] * ln, np.uint8),
                  np.array([1] * ln + [3] * ln, np.uint8))
    return c


CASES = {
    "q4_fragment": (lambda: dict(W.small_cases()["fragment97x45"], front_radius=3e-3), (1, 99, 200)),
    "q4_double_notch": (lambda: dict(_double_notch(), front_radius=8e-3), (64, 300, 336)),
    "cst_fragment": (lambda: dict(W.tri_small_cases()["tri_fragment"], front_radius=3e-3), (1, 99, 200)),
    "cst_cylinder": (lambda: dict(W.tri_small_cases()["tri_cylinder_coarse"], front_radius=2e-2), (64, 136, 200)),
    # from 16 384 elements on the pick runs over the whole GPU (bucket lists
    # in a global table, one thread per candidate): up to 145 splits per step
    "q4_fragment_grid": (lambda: dict(W.fragmentation(200, 100, 1.0e-3, seed=W.BASE_SEED + 13, steps=300,
                                                      name="fragment200x100"), front_radius=3e-3), (1, 99, 200)),
    "cst_fragment_grid": (lambda: dict(W.tri_fragment(96, 90, 1.0e-3, steps=300, name="tri_fragment96x90"),
                                       front_radius=3e-3), (1, 99, 200)),
    # a radius of a quarter of the plate: a few cells hold thousands of
    # accepted candidates, so the 64-slot bucket rows overflow into lists
    "q4_fragment_grid_wide": (lambda: dict(W.fragmentation(200, 100, 1.0e-3, seed=W.BASE_SEED + 13, steps=300,
                                                           name="fragment200x100"), front_radius=5e-2), (1, 99, 200)),
    "cst_fragment_grid_wide": (lambda: dict(W.tri_fragment(96, 90, 1.0e-3, steps=300, name="tri_fragment96x90"),
                                            front_radius=5e-2), (1, 99, 200)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_front_pick_matches_oracle(gpu, oracle_mod, name):
    make, chunks = CASES[name]
    cfg = make()
    o = oracle_mod.Oracle(cfg)
    models = [gpu.from_config(cfg, use_graph=g) for g in (True, False)]
    done = 0
    for ch in chunks:
        o.step(ch)
        done += ch
        for m in models:
            m.step(ch)
            m.sync()
            _same(m, o, (name, done))
    lg = o.log()
    assert len(lg["elem"]) > 5
    assert np.any(np.diff(lg["step"]) == 0), "several splits in one step"
    print(name, "splits", len(lg["elem"]), "steps with splits", len(np.unique(lg["step"])), flush=True)


@pytest.mark.parametrize("name", ["q4_fragment_grid", "cst_fragment_grid"])
@pytest.mark.parametrize("limits", [("0", "2048"), ("4", "16")], ids=["lds_sort", "all_paths"])
def test_front_pick_close_paths(gpu, oracle_mod, monkeypatch, name, limits):
    """The pick's close takes three paths by the number of picked candidates
    of a step: ranking by counting (up to 256), a sort in LDS, a sort in the
    scratch arrays (global memory).  The testing knobs MCT_FRONT_RANK_MAX and
    MCT_FRONT_SORT_LDS_MAX, read when the model is finalised, lower the
    limits so that small steps take the other paths: every step sorts in
    LDS, or steps with up to 4 picks count, up to 16 sort in LDS and more
    sort in global memory."""
    monkeypatch.setenv("MCT_FRONT_RANK_MAX", limits[0])
    monkeypatch.setenv("MCT_FRONT_SORT_LDS_MAX", limits[1])
    make, chunks = CASES[name]
    cfg = make()
    o = oracle_mod.Oracle(cfg)
    m = gpu.from_config(cfg)
    for ch in chunks:
        o.step(ch)
        m.step(ch)
        m.sync()
        _same(m, o, (name, limits))
    per_step = np.bincount(o.log()["step"])
    assert per_step.max() > 16 and np.any((per_step > 4) & (per_step <= 16))


@pytest.mark.parametrize("kind", ["q4", "cst"])
def test_infinite_radius_is_the_global_pick(gpu, oracle_mod, kind):
    cfg = W.small_cases()["fragment97x45"] if kind == "q4" else W.tri_small_cases()["tri_fragment"]
    g = gpu.from_config(cfg)
    f = gpu.from_config(dict(cfg, front_radius=math.inf))
    g.step(300)
    f.step(300)
    lg, lf = g.crack_set(), f.crack_set()
    assert len(lg["elem"]) > 20
    for k in ("step", "elem", "entry", "exit", "G"):
        assert np.array_equal(lg[k], lf[k])
    assert np.array_equal(g.field(0)[0], f.field(0)[0])


@pytest.mark.parametrize("name", ["q4_fragment", "q4_fragment_grid", "cst_fragment_grid"])
def test_front_pick_checkpoint(gpu, name):
    """Restored into a fresh model and into the same one (an odd number of
    steps after the checkpoint, so that the grid pick's table of the next
    step is the one the last step left in use)."""
    cfg = CASES[name][0]()
    a = gpu.from_config(cfg)
    a.step(100)
    ck = a.checkpoint()
    a.step(151)
    la = a.crack_set()
    fa = a.field(0)[1]
    assert len(la["elem"]) > 0
    b = gpu.from_config(cfg)
    b.restore(ck)
    b.step(151)
    a.restore(ck)
    a.step(151)
    for m in (a, b):
        lm = m.crack_set()
        for k in ("step", "elem", "entry", "exit", "G"):
            assert np.array_equal(la[k], lm[k]), k
        assert np.array_equal(fa, m.field(0)[1])


def test_front_pick_errors(gpu):
    cfg = W.config1()
    m = gpu.Model()
    m.set_mesh_grid(cfg["nx"], cfg["ny"], cfg["X"], cfg["Y"])
    with pytest.raises(gpu.MctError):
        m.set_front_pick(-1.0)
    with pytest.raises(gpu.MctError, match="single-tip"):
        gpu.from_config(dict(cfg, front_radius=1e-3, tracking=("sct", -1, 0)))
    with pytest.raises(gpu.MctError, match="single-tip"):
        gpu.from_config(dict(W.tri_small_cases()["tri_plate40x16"], front_radius=1e-3, tracking=("sct", -1, 0)))
    b = gpu.Model(n_specimens=2)
    b.set_mesh_grid(cfg["nx"], cfg["ny"], cfg["X"], cfg["Y"])
    with pytest.raises(gpu.MctError):
        b.set_front_pick(1e-3)
