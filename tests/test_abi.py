"""Host-side checks of the C ABI that need no GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2509_01827_amd import mct2d, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mct2d.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mct_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_binding_names():
    assert sorted(mct2d.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = mct2d.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # extern "C": no C++ mangling for the ABI
    out = os.popen("nm -D --defined-only %s" % mct2d.LIB_PATH).read()
    for name in _declared():
        assert re.search(r"\bT %s\b" % name, out), name


def test_null_handles_are_rejected():
    lib = mct2d.load()
    assert lib.mct_destroy(None) == 0
    assert lib.mct_step(None, 1) == -1
    assert lib.mct_finalize(None) == -1
    assert lib.mct_create(None, 64, None) == -1
    h = ctypes.c_void_p()
    assert lib.mct_create(ctypes.byref(h), 16, None) == -6   # precisions are 64 and 32
    assert lib.mct_batch_create(ctypes.byref(h), 2, 32, None) == -6  # binary32: plain contexts only
    assert b"null" in lib.mct_last_error(None)


def test_workload_generators_are_seeded_and_shaped():
    c1 = W.config2(steps=1)
    c2 = W.config2(steps=1)
    assert np.array_equal(c1["X"], c2["X"]) and np.array_equal(c1["Y"], c2["Y"])
    nx, ny = c1["nx"], c1["ny"]
    X = c1["X"].reshape(ny + 1, nx + 1)
    Y = c1["Y"].reshape(ny + 1, nx + 1)
    # rectangular plate: boundary nodes only slide along their edge
    assert np.all(X[:, 0] == 0.0) and np.allclose(X[:, -1], 0.1, rtol=0, atol=1e-15)
    assert np.all(Y[0, :] == 0.0) and np.allclose(Y[-1, :], 0.04, rtol=0, atol=1e-15)
    hx = 0.1 / nx
    dev = np.abs(X - np.arange(nx + 1) * hx).max()
    assert 0.009 * hx < dev <= 0.01 * hx
    g = W.weibull_gc(W.BASE_SEED + 3, 100000, 6.0, 3.0)
    # Weibull(k=6, lambda=3): mean = 3 Gamma(1 + 1/6)
    assert g.mean() == pytest.approx(3.0 * 0.9277193336, rel=5e-3)
    # SplitMix64 reference value (seed 0, first output)
    assert int(W.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_device_views_refuse_bad_arrays():
    """Caller-owned state arrays are checked before the library sees them:
    CPU, wrong-dtype, strided, short or aliased tensors, mixed kinds and raw
    addresses without a length are refused."""
    import torch
    nn = 50
    ok = [torch.zeros(nn, dtype=torch.float64) for _ in range(6)]
    with pytest.raises(mct2d.MctError, match="device tensors"):
        mct2d.device_views(ok, None, nn)  # host tensors
    with pytest.raises(mct2d.MctError, match="six arrays"):
        mct2d.device_views(ok[:5] + [None], None, nn)
    with pytest.raises(mct2d.MctError, match="length n"):
        mct2d.device_views([1, 2, 3, 4, 5, 6], None, nn)
    with pytest.raises(mct2d.MctError, match="distinct"):
        mct2d.device_views([8, 8, 16, 24, 32, 40], nn, nn)
    with pytest.raises(mct2d.MctError, match="non-null"):
        mct2d.device_views([0, 8, 16, 24, 32, 40], nn, nn)
    with pytest.raises(mct2d.MctError, match="nodes"):
        mct2d.device_views([8, 16, 24, 32, 40, 48], nn - 1, nn)
    with pytest.raises(mct2d.MctError, match="not mixed"):
        mct2d.device_views([8, 16, 24, 32, 40, ok[0]], nn, nn)
    ptr, length = mct2d.device_views([8, 16, 24, 32, 40, 48], nn + 3, nn)
    assert ptr == [8, 16, 24, 32, 40, 48] and length == nn + 3
    # the C side checks the same at finalize against the mesh (GPU tests)
    assert "int64_t n;" in open(HEADER).read()
