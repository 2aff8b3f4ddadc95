"""Full-size GPU parity against stored oracle results.

The reference files under tests/golden/ were written by
tests/golden/make_golden.py, which runs only the CPU oracle.  The GPU runs
the same workload through the C ABI in the launch configuration bench.py
times (automatic tile and kernel choice, captured graphs) over the
workload's whole run and must reproduce the whole split log and the split
codes bit for bit (SHA-256 over the arrays), the tip set, U_d, the
near-threshold decision log and the sampled nodal fields (within 1e-9
relative; expected bitwise).  Cases: the 400 x 400 branching plate in
binary64 (20 000 steps) and in binary32 (20 000 steps), the 2000 x 1000
fragmentation plate (10 000 steps), and four specimens of the 256-specimen
batch (the largest, the smallest and two seeded ones), run inside the full
batch launch for its 5 000 steps.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2509_01827_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
NEAR_TOL = 1e-6


def _log_digest(step, elem, entry, exit_, G):
    h = hashlib.sha256()
    for a in (step, elem, entry, exit_):
        h.update(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes())
    h.update(np.ascontiguousarray(np.asarray(G, dtype="<f8")).tobytes())
    return h.hexdigest()


def _near_digest(nl):
    """The library returns the records sorted by (step, kind, element, a, k)."""
    h = hashlib.sha256()
    for key in ("step", "elem", "a", "kind", "k"):
        h.update(np.ascontiguousarray(np.asarray(nl[key], dtype="<i8")).tobytes())
    for key in ("G", "ref"):
        h.update(np.ascontiguousarray(np.asarray(nl[key], dtype="<f8")).tobytes())
    return h.hexdigest()


def _unhex(v):
    return np.array([float.fromhex(x) for x in v])


def _golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip("reference %s not generated" % name)
    return json.load(open(path))


def _check(m, ref, *, label, near=True):
    inf = m.info()
    assert inf["step"] == ref["steps"], label
    assert inf["dt"] == float.fromhex(ref["dt"]), label
    lg = m.crack_set()
    assert len(lg["elem"]) == ref["n_splits"], label
    head = ref["log_head"]
    nh = len(head["elem"])
    assert np.array_equal(lg["step"][:nh], head["step"]), label
    assert np.array_equal(lg["elem"][:nh], head["elem"]), label
    assert np.array_equal(lg["entry"][:nh], head["entry"]), label
    assert np.array_equal(lg["exit"][:nh], head["exit"]), label
    np.testing.assert_allclose(lg["G"][:nh], _unhex(head["G"]), rtol=1e-9, atol=0)
    assert _log_digest(lg["step"], lg["elem"], lg["entry"], lg["exit"], lg["G"]) == ref["log_digest"], label
    codes = m.split_codes()
    assert hashlib.sha256(codes.tobytes()).hexdigest() == ref["codes_digest"], label
    tips, _ = m.tips()
    assert len(tips) == ref["n_tips"], label
    assert hashlib.sha256(np.asarray(tips, "<i8").tobytes()).hexdigest() == ref["tips_digest"], label
    assert inf["dissipated"] == pytest.approx(float.fromhex(ref["Ud"]), rel=1e-12), label
    nodes = np.asarray(ref["nodes"])
    ux, uy = m.field(0)
    vx, vy = m.field(1)
    for got, key in ((ux, "ux"), (uy, "uy"), (vx, "vx"), (vy, "vy")):
        want = _unhex(ref[key])
        scale = max(np.abs(want).max(), 1e-300)
        assert np.abs(got[nodes] - want).max() <= 1e-9 * scale, (label, key)
        assert np.array_equal(got[nodes], want), (label, key + " not bit-identical")
    if near and "near" in ref:
        nl = m.near_log()
        assert len(nl["kind"]) == ref["near"]["count"], label
        assert _near_digest(nl) == ref["near"]["digest"], label


CASES = {
    "plate400": lambda: W.config2(),
    "plate400_f32": lambda: dict(W.config2(), precision=32),
    "fragment2000": lambda: W.config3(),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fullsize_against_oracle(name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref = _golden(name)
    from paper_2509_01827_amd import mct2d
    cfg = dict(CASES[name](), near_tol=ref["near"]["tol"])
    print("full-size case", name, cfg["nx"], cfg["ny"], cfg["steps"], flush=True)
    s = torch.cuda.Stream()
    m = mct2d.from_config(cfg, stream=s.cuda_stream)
    m.step(cfg["steps"])
    m.sync()
    _check(m, ref, label=name)


@pytest.mark.parametrize("name", ["plate400", "fragment2000"])
def test_fullsize_without_near_log(name):
    """The launch bench.py times (no near-threshold log: the plain kernels,
    the lattice kernel on the fragmentation plate) reproduces the same run."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref = _golden(name)
    from paper_2509_01827_amd import mct2d
    cfg = CASES[name]()
    s = torch.cuda.Stream()
    m = mct2d.from_config(cfg, stream=s.cuda_stream)
    assert m.lattice() == (name == "fragment2000")
    m.step(cfg["steps"])
    m.sync()
    _check(m, ref, label=name, near=False)


def test_batch_specimens_at_full_size():
    """Four specimens of the 256-specimen batch (the largest 479 x 245, the
    smallest 64 x 74, two seeded ones) run inside the whole batch launch for
    the full 5 000 steps and equal their own oracle runs."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref = _golden("batch256_sample")
    from paper_2509_01827_amd import mct2d
    cfgs = W.batch_specimens()
    assert len(cfgs) == ref["n_specimens"]
    print("batch of", len(cfgs), "specimens,", cfgs[0]["steps"], "steps", flush=True)
    s = torch.cuda.Stream()
    b = mct2d.batch_from_configs(cfgs, stream=s.cuda_stream)
    assert b.lattice()
    b.step(cfgs[0]["steps"])
    b.sync()
    for spec, r in zip(ref["sample"], ref["specimens"]):
        b.select(spec)
        _check(b, r, label="specimen %d" % spec)
