"""GPU: the tip query that allocates nothing (mct_get_tips_noalloc), through
the C ABI, against the allocating query (mct_get_tips): two calls in a row
on the same GPU, the second on a smaller model, each bit for bit equal; a
capacity below the count writes only that many and reports the count; sizes
beyond the static scratch are refused."""
import ctypes

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


def _noalloc_tips(gpu, m, cap, stream):
    import torch
    edge = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    xy = torch.full((max(2 * cap, 2),), -7.0, dtype=torch.float64, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = m._L.mct_get_tips_noalloc(m._h, cap, ctypes.c_void_p(edge.data_ptr()), ctypes.c_void_p(xy.data_ptr()),
                                   ctypes.c_void_p(cnt.data_ptr()))
    assert rc == 0, m._L.mct_last_error(m._h)
    stream.synchronize()
    torch.cuda.synchronize()
    return edge.cpu().numpy(), xy.cpu().numpy().reshape(-1, 2), int(cnt.cpu().numpy()[0])


def test_noalloc_tips_match_the_allocating_query(gpu):
    import torch
    st = torch.cuda.Stream()
    big = gpu.from_config(W.config2(steps=4000), stream=st.cuda_stream)
    big.step(4000)
    small = gpu.from_config(W.small_cases()["plate70x37_jitter"], stream=st.cuda_stream)
    small.step(900)
    for m in (big, small):  # two calls in a row, the second smaller
        m.sync()
        want_e, want_xy = m.tips()
        print("tips", len(want_e), flush=True)
        assert len(want_e) > 0
        e, xy, n = _noalloc_tips(gpu, m, len(want_e) + 5, st)
        assert n == len(want_e)
        assert np.array_equal(e[:n], want_e) and np.array_equal(xy[:n], want_xy)
        assert np.all(e[n:] == -7)  # nothing written past the count
    # a capacity below the count: the first cap tips, the full count
    want_e, want_xy = big.tips()
    e, xy, n = _noalloc_tips(gpu, big, 10, st)
    assert n == len(want_e) and np.array_equal(e[:10], want_e[:10]) and np.array_equal(xy[:10], want_xy[:10])
    # capacity 0: only the count
    _, _, n0 = _noalloc_tips(gpu, small, 0, st)
    assert n0 == len(small.tips()[0])


def test_noalloc_tips_refusals(gpu):
    import torch
    m = gpu.from_config(W.small_cases()["plate40x40"])
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert m._L.mct_get_tips_noalloc(m._h, 4, None, None, ctypes.c_void_p(cnt.data_ptr())) == -1
    assert m._L.mct_get_tips_noalloc(m._h, 0, None, None, None) == -1
    t = gpu.from_config(W.tri_small_cases()["tri_plate40x16"])
    assert t._L.mct_get_tips_noalloc(t._h, 0, None, None, ctypes.c_void_p(cnt.data_ptr())) == -6
    # a mesh beyond the static scratch (2^24 edges) is refused before any launch
    nx, ny = 4097, 2049  # 2 nx ny + nx + ny > 2^24
    X, Y = W.grid_coords(nx, ny, nx * 1e-3, ny * 1e-3)
    h = gpu.Model()
    h.set_mesh_grid(nx, ny, X, Y)
    h.set_material(32e9, 0.2, 2450.0, None, 3.0, 1.0)
    h.finalize()
    rc = h._L.mct_get_tips_noalloc(h._h, 0, None, None, ctypes.c_void_p(cnt.data_ptr()))
    assert rc == -1 and b"at most" in h._L.mct_last_error(h._h)
