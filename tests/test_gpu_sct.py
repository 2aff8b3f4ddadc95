"""Single crack-tip tracking on the GPU against the CPU oracle (same bar as
the multi-tip step: exact split log and codes, bit-identical fields, the
same tip), for every tile shape and launch mode, in a batch next to
multi-tip specimens, and across a checkpoint."""
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


def _sct(cfg, elem=-1, edge=0):
    c = dict(cfg)
    c["tracking"] = ("sct", elem, edge)
    return c


def _same(m, o):
    lg, ol = m.crack_set(), o.log()
    for k in ("step", "elem", "entry", "exit"):
        if not np.array_equal(lg[k].astype(np.int64), ol[k].astype(np.int64)):
            return False
    st = o.state()
    return (np.array_equal(lg["G"], ol["G"]) and np.array_equal(m.split_codes(), st["split"])
            and all(np.array_equal(a, b) for a, b in zip(m.field(0) + m.field(1),
                                                        (st["ux"], st["uy"], st["vx"], st["vy"])))
            and m.tip() == o.tip())


def test_sct_matches_oracle_all_tiles(gpu, oracle_mod):
    cfg = _sct(W.small_cases()["plate70x37_jitter"])
    o = oracle_mod.Oracle(cfg)
    models = [gpu.from_config(cfg, tile=t, use_graph=g) for t in (1, 2, 3) for g in (True, False)]
    assert all(m.tip() == o.tip() for m in models)
    done = 0
    for chunk in (1, 64, 300, 835):
        o.step(chunk)
        done += chunk
        for m in models:
            m.step(chunk)
            m.sync()
            assert _same(m, o), ("step", done, m.launch())
    assert len(o.log()["elem"]) > 10


def test_sct_explicit_start_and_boundary_end(gpu, oracle_mod):
    cfg = _sct(W.config1(), 20 * 40 + 20, 3)
    o = oracle_mod.run(cfg, 2000)
    m = gpu.from_config(cfg)
    m.step(2000)
    assert _same(m, o)
    assert m.tip() is None  # the crack reached the boundary


def test_sct_in_a_batch_with_mct(gpu, oracle_mod):
    cfgs = W.small_batch(6, steps=500)
    cfgs = [(_sct(c) if s % 2 == 0 else c) for s, c in enumerate(cfgs)]
    m = gpu.batch_from_configs(cfgs)
    m.step(500)
    for s, cfg in enumerate(cfgs):
        m.select(s)
        o = oracle_mod.run(cfg, 500)
        assert _same(m, o), s


def test_sct_checkpoint_restore(gpu):
    cfg = _sct(W.small_cases()["plate64x48_gamma2"])
    a = gpu.from_config(cfg)
    a.step(333)
    ck = a.checkpoint()
    a.step(400)
    b = gpu.from_config(cfg)
    b.restore(ck)
    assert b.tip() is not None or a.tip() is None
    b.step(400)
    la, lb = a.crack_set(), b.crack_set()
    assert np.array_equal(la["elem"], lb["elem"]) and np.array_equal(la["step"], lb["step"])
    assert a.tip() == b.tip()
    assert np.array_equal(a.field(0)[0], b.field(0)[0])


def test_sct_needs_a_start_tip(gpu):
    cfg = _sct(W.small_cases()["fragment97x45"])  # no pre-notch
    with pytest.raises(gpu.MctError, match="start tip"):
        gpu.from_config(cfg)
    with pytest.raises(gpu.MctError):
        gpu.from_config(_sct(W.config1(), 1600, 0))
