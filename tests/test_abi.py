"""The C-ABI library loads without a GPU, exports every symbol include/svr.h declares, and
rejects invalid arguments on the host before touching any device memory."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_1707_00442_amd import _capi
    return _capi


def test_header_and_library_agree(capi):
    hdr = open(os.path.join(ROOT, "include", "svr.h")).read()
    declared = set(re.findall(r"\b(svr_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(capi.EXPORTS)
    L = capi.load()
    for name in declared:
        assert hasattr(L, name), name
    assert L.svr_version().startswith(b"svr")


def _fake_view(capi, **kw):
    v = capi.CubeView()
    v.data, v.dtype, v.nx, v.ny, v.nz, v.sx, v.sy, v.sz = 0x1000, 0, 8, 8, 8, 0, 0, 0
    for k, x in kw.items():
        setattr(v, k, x)
    return v


def test_view_validation(capi):
    L = capi.load()
    out = (C.c_float * 2)()
    assert L.svr_minmax(C.byref(_fake_view(capi, data=0)), out, None) == capi.SVR_EINVAL
    assert L.svr_minmax(C.byref(_fake_view(capi, nx=0)), out, None) == capi.SVR_EINVAL
    assert L.svr_minmax(C.byref(_fake_view(capi, dtype=7)), out, None) == capi.SVR_EINVAL
    assert L.svr_minmax(C.byref(_fake_view(capi, sx=1)), out, None) == capi.SVR_EINVAL
    h = C.c_void_p()
    assert L.svr_volume_create(C.byref(_fake_view(capi)), 5, 8, math.nan, None,
                               C.byref(h)) == capi.SVR_EINVAL
    assert L.svr_volume_create(C.byref(_fake_view(capi)), 0, 12, math.nan, None,
                               C.byref(h)) == capi.SVR_EINVAL
    assert b"brick" in L.svr_last_error()


def _cam(capi, **kw):
    c = capi.Camera()
    c.type, c.width, c.height = 1, 16, 16
    c.eye[:] = [0, 0, -10]
    c.U[:] = [0.3, 0, 0]
    c.V[:] = [0, 0.3, 0]
    c.W[:] = [0, 0, 1]
    for k, x in kw.items():
        setattr(c, k, x)
    return c


def test_render_validation(capi):
    import paper_1707_00442_amd as svr
    L = capi.load()
    vol = C.c_void_p(0)  # null volume is rejected first
    lut = capi.Lut()
    lut.rgba, lut.n = 0x1000, 16
    p = svr.params_struct(mode="avip0")
    out = C.c_void_p(0x2000)
    assert L.svr_render(vol, None, C.byref(_cam(capi)), C.byref(lut), C.byref(p), out, None,
                        None) == capi.SVR_EINVAL
    # parameter checks run before any device access, so a fake handle never gets touched
    cases = [
        dict(mode=9), dict(filter=5), dict(box_arm=99), dict(k=1.5), dict(k=-0.1),
        dict(min_val=0.0), dict(dt=0.0), dict(dt=math.nan), dict(filter="scale", min_t=2.0, max_t=1.0),
        dict(ratio=1, mode="avip0"), dict(ratio=1, box_arm=2), dict(mip_alpha=3),
        dict(min_t=math.nan), dict(clim_lo=0.0, clim_hi=math.inf),
    ]
    for c in cases:
        q = svr.params_struct(c)
        assert L.svr_params_validate(C.byref(q)) == capi.SVR_EINVAL, c
    good = [dict(), dict(mode="mip1", filter="clip", min_t=1.0), dict(ratio=2, filter="clip"),
            dict(filter="scale", min_t=0.0, max_t=1.0), dict(box_arm=15, mode="aviprgb"),
            dict(clim_lo=1.0, clim_hi=1.0), dict(k=0.0), dict(k=1.0, ert=2.0)]
    for c in good:
        assert L.svr_params_validate(C.byref(svr.params_struct(c))) == capi.SVR_OK, c
    bad_cams = [dict(type=3), dict(width=0), dict(height=40000)]
    for c in bad_cams:
        assert L.svr_render(C.c_void_p(0x10), None, C.byref(_cam(capi, **c)), C.byref(lut),
                            C.byref(p), out, None, None) == capi.SVR_EINVAL, c
    cam = _cam(capi)
    cam.W[:] = [0, 0, 0]
    assert L.svr_render(C.c_void_p(0x10), None, C.byref(cam), C.byref(lut), C.byref(p), out,
                        None, None) == capi.SVR_EINVAL
    lut.n = 1
    assert L.svr_render(C.c_void_p(0x10), None, C.byref(_cam(capi)), C.byref(lut), C.byref(p),
                        out, None, None) == capi.SVR_EINVAL


def test_smooth_and_ratio_validation(capi):
    L = capi.load()
    v = _fake_view(capi)
    taps = (C.c_float * 4)(0.25, 0.25, 0.25, 0.25)
    n = C.c_size_t()
    assert L.svr_smooth_workspace(C.byref(v), 3, C.byref(n)) == capi.SVR_OK
    assert n.value == 2 * 8 * 8 * 8 * 4
    # the fused tap counts need no workspace (and accept none)
    for T in (5, 7, 9, 13, 19):
        m = C.c_size_t(123)
        assert L.svr_smooth_workspace(C.byref(v), T, C.byref(m)) == capi.SVR_OK
        assert m.value == 0
    assert L.svr_smooth_workspace(C.byref(v), 4, C.byref(n)) == capi.SVR_EINVAL
    taps7 = (C.c_float * 7)(*([1.0 / 7] * 7))
    assert L.svr_smooth(C.byref(v), taps7, 7, None, None, 0, None) == capi.SVR_EINVAL
    assert L.svr_smooth(C.byref(v), taps7, 7, C.c_void_p(0x1000), None, 0,
                        None) == capi.SVR_EINVAL  # output aliases the input
    n.value = 2 * 8 * 8 * 8 * 4
    assert L.svr_smooth(C.byref(v), taps, 4, C.c_void_p(0x5000), C.c_void_p(0x6000), n.value,
                        None) == capi.SVR_EINVAL  # even tap count
    taps3 = (C.c_float * 3)(0.25, 0.5, 0.25)
    assert L.svr_smooth(C.byref(v), taps3, 3, C.c_void_p(0x5000), C.c_void_p(0x6000), 16,
                        None) == capi.SVR_ENOMEM  # workspace too small
    assert L.svr_smooth(C.byref(_fake_view(capi, sx=1, sy=8, sz=64)), taps3, 3,
                        C.c_void_p(0x5000), C.c_void_p(0x6000), n.value,
                        None) == capi.SVR_EUNSUPPORTED
    assert L.svr_line_ratio(C.byref(v), 0, 4, 5, 0.0, 0.0, -1.0, C.c_void_p(0x5000),
                            None) == capi.SVR_EINVAL  # window 4..9 leaves the cube
    assert L.svr_line_ratio(C.byref(v), 0, 4, 4, math.nan, 0.0, -1.0, C.c_void_p(0x5000),
                            None) == capi.SVR_EINVAL
    # window starts near INT32_MAX: the end is checked in 64 bits (no overflow)
    big = 2 ** 31 - 2
    assert L.svr_line_ratio(C.byref(v), big, 0, 4, 0.0, 0.0, -1.0, C.c_void_p(0x5000),
                            None) == capi.SVR_EINVAL
    assert L.svr_line_ratio(C.byref(v), 0, big, 4, 0.0, 0.0, -1.0, C.c_void_p(0x5000),
                            None) == capi.SVR_EINVAL
    assert L.svr_moments(C.byref(v), big, 4, 1.0, -math.inf, math.inf, C.c_void_p(0x5000),
                         None, None, None) == capi.SVR_EINVAL


def test_status_strings(capi):
    L = capi.load()
    for s in range(5):
        assert L.svr_status_string(s).startswith(b"SVR_")


def test_moments_validation(capi):
    """svr_moments rejects bad windows and arguments on the host (fake device pointers are
    never touched)."""
    L = capi.load()
    v = C.byref(_fake_view(capi))
    p = C.c_void_p(0x2000)
    inf = math.inf
    assert L.svr_moments(v, 0, 9, 1.0, -inf, inf, p, p, p, None) == capi.SVR_EINVAL  # nz = 8
    assert L.svr_moments(v, -1, 4, 1.0, -inf, inf, p, p, p, None) == capi.SVR_EINVAL
    assert L.svr_moments(v, 0, 0, 1.0, -inf, inf, p, p, p, None) == capi.SVR_EINVAL
    assert L.svr_moments(v, 0, 8, math.nan, -inf, inf, p, p, p, None) == capi.SVR_EINVAL
    assert L.svr_moments(v, 0, 8, 1.0, 2.0, 1.0, p, p, p, None) == capi.SVR_EINVAL
    assert L.svr_moments(v, 0, 8, 1.0, -inf, inf, None, None, None, None) == capi.SVR_EINVAL
    assert b"svr_moments" in L.svr_last_error()
