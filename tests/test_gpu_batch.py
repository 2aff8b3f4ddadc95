"""Batched form: many independent, uneven specimens in one launch per step.

Every specimen of the batch must equal the CPU oracle run of that specimen
alone (same bar as the plain step: exact split log, codes and tips, fields
bit-identical), whatever the tile shape, work-unit order or launch mode, and
the autotuner must leave the state as it found it.
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


def _snapshot(m, s):
    m.select(s)
    lg = m.crack_set()
    return dict(log=lg, codes=m.split_codes(), u=m.field(0), v=m.field(1), tips=m.tips()[0],
                info=m.info())


def _same(a, b):
    for k in ("step", "elem", "entry", "exit", "G"):
        if not np.array_equal(a["log"][k], b["log"][k]):
            return False
    return (np.array_equal(a["codes"], b["codes"]) and np.array_equal(a["tips"], b["tips"])
            and all(np.array_equal(x, y) for x, y in zip(a["u"] + a["v"], b["u"] + b["v"]))
            and a["info"]["dissipated"] == b["info"]["dissipated"])


def test_batch_matches_oracle_per_specimen(gpu, oracle_mod):
    cfgs = W.small_batch(12, steps=600)
    m = gpu.batch_from_configs(cfgs)
    m.step(600)
    m.sync()
    total_splits = 0
    for s, cfg in enumerate(cfgs):
        print("specimen", s, cfg["nx"], cfg["ny"], flush=True)
        o = oracle_mod.run(cfg, 600)
        got = _snapshot(m, s)
        ol, st = o.log(), o.state()
        for k in ("step", "elem", "entry", "exit"):
            assert np.array_equal(got["log"][k].astype(np.int64), ol[k].astype(np.int64)), (s, k)
        assert np.array_equal(got["log"]["G"], ol["G"]), s
        assert np.array_equal(got["codes"], st["split"]), s
        for a, b in zip(got["u"] + got["v"], (st["ux"], st["uy"], st["vx"], st["vy"])):
            assert np.array_equal(a, b), s
        assert np.array_equal(got["tips"], o.tips()[0]), s
        assert got["info"]["dissipated"] == pytest.approx(o.info()["Ud"], rel=1e-12)
        assert got["info"]["step"] == 600
        total_splits += len(ol["elem"])
    assert total_splits > 0


def test_batch_invariant_to_tiles_orders_and_graphs(gpu):
    cfgs = W.small_batch(7, steps=300)
    ref = None
    for tile in (1, 2, 3):
        for order in (0, 1, 2):
            for graph in ((True, False) if tile == 2 else (True,)):
                print("tile", tile, "order", order, "graph", graph, flush=True)
                m = gpu.batch_from_configs(cfgs, tile=tile, order=order, use_graph=graph)
                m.step(130)
                snaps = [_snapshot(m, s) for s in range(len(cfgs))]
                if ref is None:
                    ref = snaps
                else:
                    assert all(_same(a, b) for a, b in zip(ref, snaps)), (tile, order, graph)
                m.close()


def test_autotune_keeps_state(gpu):
    cfgs = W.small_batch(9, steps=300)
    a = gpu.batch_from_configs(cfgs)
    a.step(100)
    choice = a.autotune(trial_steps=5)
    assert 1 <= choice["tile"] <= 3 and 0 <= choice["order"] <= 2 and choice["us_per_step"] > 0
    lau = a.launch()
    assert lau["tile"] == choice["tile"] and lau["order"] == choice["order"]
    a.step(100)
    b = gpu.batch_from_configs(cfgs)
    b.step(200)
    for s in range(len(cfgs)):
        assert _same(_snapshot(a, s), _snapshot(b, s)), s


def test_plain_autotune(gpu):
    cfg = W.small_cases()["plate70x37_jitter"]
    m = gpu.from_config(cfg)
    m.step(50)
    choice = m.autotune(trial_steps=5)
    assert 1 <= choice["tile"] <= 3 and choice["order"] == 0
    m.step(50)
    r = gpu.from_config(cfg)
    r.step(100)
    assert np.array_equal(m.field(0)[0], r.field(0)[0])
    assert np.array_equal(m.split_codes(), r.split_codes())


def test_batch_checkpoint_restore(gpu):
    cfgs = W.small_batch(5, steps=200)
    a = gpu.batch_from_configs(cfgs)
    a.step(100)
    ck = a.checkpoint()
    a.step(100)
    b = gpu.batch_from_configs(cfgs)
    b.restore(ck)
    b.step(100)
    for s in range(len(cfgs)):
        assert _same(_snapshot(a, s), _snapshot(b, s)), s


def test_batch_select_out_of_range(gpu):
    m = gpu.Model(n_specimens=3)
    with pytest.raises(gpu.MctError):
        m.select(3)
    with pytest.raises(gpu.MctError):
        m.finalize()  # specimens not set up


def test_batch_with_different_time_steps(gpu, oracle_mod):
    """Specimens with different element sizes, materials and loads step with
    their own dt in one launch."""
    cfgs = [W.plate(20, 14, 0.02, 0.014, jitter=0.02, seed=W.BASE_SEED + 51, notch_len=8, steps=400),
            W.plate(17, 23, 0.034, 0.023, jitter=0.01, seed=W.BASE_SEED + 52, notch_len=7, traction=1.4e6,
                    steps=400),
            W.fragmentation(25, 12, 2.5e-3, seed=W.BASE_SEED + 53, steps=400)]
    m = gpu.batch_from_configs(cfgs)
    m.step(400)
    dts = set()
    for s, cfg in enumerate(cfgs):
        o = oracle_mod.run(cfg, 400)
        snap = _snapshot(m, s)
        dts.add(snap["info"]["dt"])
        assert snap["info"]["dt"] == o.info()["dt"]
        ol, st = o.log(), o.state()
        for k in ("step", "elem", "entry", "exit"):
            assert np.array_equal(snap["log"][k].astype(np.int64), ol[k].astype(np.int64)), (s, k)
        assert np.array_equal(snap["codes"], st["split"]), s
        for a, b in zip(snap["u"] + snap["v"], (st["ux"], st["uy"], st["vx"], st["vy"])):
            assert np.array_equal(a, b), s
    assert len(dts) == 3
