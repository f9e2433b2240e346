"""The allocation-free finite min/max (svr_minmax_noalloc) against svr_minmax, called through
the C ABI on two calls in a row, the second with a smaller input whose range lies inside the
first's (so partials left over from the first call would show)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pair_minmax(L, v):
    out = (C.c_float * 2)()
    st = L.svr_minmax(C.byref(v), out, None)
    assert st == 0, L.svr_last_error()
    return np.array(out[:], dtype=np.float32)


def _pair_noalloc(L, v, torch):
    dev = torch.full((2,), 7.0, dtype=torch.float32, device="cuda")
    st = L.svr_minmax_noalloc(C.byref(v), C.c_void_p(dev.data_ptr()), None)
    assert st == 0, L.svr_last_error()
    return dev.cpu().numpy()


def _same(a, b):
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_minmax_noalloc_matches_minmax_on_two_calls():
    import torch

    import paper_1707_00442_amd as svr
    from paper_1707_00442_amd import _capi
    L = _capi.load()
    rng = np.random.default_rng(11)
    # call 1: a float32 cube large enough for the full 2048-workgroup reduction, with wide
    # extremes and non-finite values (ignored)
    big = rng.standard_normal((257, 300, 200)).astype(np.float32)
    big[3, 4, 5], big[200, 100, 7] = -1.0e6, 1.0e6
    big[0, 0, 0], big[1, 2, 3], big[5, 6, 7] = np.nan, np.inf, -np.inf
    tb = torch.from_numpy(big).cuda()
    print("call 1: float32 257x300x200 contiguous", flush=True)
    ref1 = _pair_minmax(L, svr.cube_view(tb))
    got1 = _pair_noalloc(L, svr.cube_view(tb), torch)
    assert ref1[0] == -1.0e6 and ref1[1] == 1.0e6
    assert _same(got1, ref1), (got1, ref1)
    # call 2: a smaller strided float16 view with values inside (-1, 1)
    small = (rng.random((40, 33, 50)) * 1.8 - 0.9).astype(np.float16)
    ts = torch.from_numpy(small).cuda()[::2, 1:, ::3]
    print("call 2: float16 strided view", tuple(ts.shape), flush=True)
    ref2 = _pair_minmax(L, svr.cube_view(ts))
    got2 = _pair_noalloc(L, svr.cube_view(ts), torch)
    expect = small[::2, 1:, ::3].astype(np.float32)
    assert ref2[0] == expect.min() and ref2[1] == expect.max()
    assert _same(got2, ref2), (got2, ref2)
    # call 3: one element, and a cube with no finite value (NaN pair on both sides)
    one = torch.tensor([[[0.25]]], dtype=torch.float32, device="cuda")
    assert _same(_pair_noalloc(L, svr.cube_view(one), torch), _pair_minmax(L, svr.cube_view(one)))
    nan = torch.full((3, 4, 5), float("nan"), dtype=torch.float32, device="cuda")
    g, r = _pair_noalloc(L, svr.cube_view(nan), torch), _pair_minmax(L, svr.cube_view(nan))
    assert np.isnan(g).all() and np.isnan(r).all()
    # the binding (same entry point) on the first cube again
    out = torch.empty(2, dtype=torch.float32, device="cuda")
    svr.svr_minmax_noalloc(tb, out)
    assert _same(out.cpu().numpy(), ref1)


def test_minmax_noalloc_rejects_bad_arguments():
    import paper_1707_00442_amd as svr
    from paper_1707_00442_amd import _capi
    import torch
    L = _capi.load()
    t = torch.zeros((2, 2, 2), dtype=torch.float32, device="cuda")
    assert L.svr_minmax_noalloc(C.byref(svr.cube_view(t)), None, None) == _capi.SVR_EINVAL
    v = svr.cube_view(t)
    v.nx = 0
    out = torch.empty(2, dtype=torch.float32, device="cuda")
    assert L.svr_minmax_noalloc(C.byref(v), C.c_void_p(out.data_ptr()), None) == _capi.SVR_EINVAL
