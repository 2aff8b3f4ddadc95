"""GPU: the near-threshold decision log against the oracle's.

Both sides record the decisions whose margin lies within a relative
tolerance (paths near Gc, element argmax gaps and split-ratio margins, the
pick's gap and margin), evaluated in the step's precision.  The library
sorts its records by (step, kind, element, a, k); the oracle's are sorted the
same way here, and the two must agree exactly, values included.  A large
tolerance (1e-2) makes the logs long enough to exercise every kind.
"""
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


def _sorted(nl):
    order = np.lexsort((nl["k"], nl["a"], nl["elem"], nl["kind"], nl["step"]))
    return {k: np.asarray(v)[order] for k, v in nl.items()}


def _equal(g, o, label):
    o = _sorted(o)
    assert len(g["kind"]) == len(o["kind"]), (label, len(g["kind"]), len(o["kind"]))
    for k in ("step", "elem", "a", "kind", "k"):
        assert np.array_equal(np.asarray(g[k], np.int64), np.asarray(o[k], np.int64)), (label, k)
    for k in ("G", "ref"):
        assert np.array_equal(g[k], o[k]), (label, k)


def _cases():
    sc = W.small_cases()
    return {
        "plate70x37_jitter": sc["plate70x37_jitter"],
        "plate64x48_gamma2": sc["plate64x48_gamma2"],
        "fragment97x45": dict(sc["fragment97x45"], steps=250),
        "fragment_lattice": W.fragmentation(97, 45, W.H_BATCH, seed=W.BASE_SEED + 13, steps=250),
        "plate40x40_f32": dict(sc["plate40x40"], precision=32, steps=900),
        "sct_plate40x40": dict(sc["plate40x40"], tracking=("sct", -1, 0), steps=900),
    }


@pytest.mark.parametrize("name", sorted(_cases()))
def test_near_log_matches_oracle(gpu, oracle_mod, name):
    cfg = dict(_cases()[name], near_tol=1e-2)
    steps = cfg["steps"]
    print("near case", name, steps, flush=True)
    o = oracle_mod.run(cfg, steps)
    m = gpu.from_config(cfg, use_graph=True)
    done = 0
    for chunk in (1, 100, steps - 101):  # graph segments and direct launches
        m.step(chunk)
        done += chunk
    m.sync()
    lg, ol = m.crack_set(), o.log()
    assert np.array_equal(lg["elem"], ol["elem"]) and np.array_equal(lg["G"], ol["G"])
    g = m.near_log()
    assert len(g["kind"]) > 0
    _equal(g, o.near_log(), name)
    if name.startswith("fragment"):  # heavy fragmentation exercises the rule's and the pick's kinds
        assert set(np.unique(g["kind"]).tolist()) >= {1, 2, 3, 4}


def test_near_log_off_and_refused(gpu):
    m = gpu.from_config(W.small_cases()["plate40x40"])
    m.step(300)
    assert len(m.near_log()["kind"]) == 0
    b = gpu.Model(n_specimens=2)
    with pytest.raises(gpu.MctError):
        b.set_near_log(1e-6)
    with pytest.raises(gpu.MctError):
        m.set_near_log(-1.0)


def test_near_log_capacity(gpu):
    cfg = dict(W.small_cases()["fragment97x45"], near_tol=1e-2, near_cap=10, steps=100)
    m = gpu.from_config(cfg)
    m.step(100)
    with pytest.raises(gpu.MctError, match="overflow"):
        m.near_log()
