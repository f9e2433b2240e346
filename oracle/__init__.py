"""FP64 CPU oracle for the ray-cast colouring/filtering path (Vohl et al. 2017).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product (the HIP library and its binding) never
does, and this package never imports the product.  It is plain and slow on purpose.

Contents
  * ``render`` / ``render_grad`` / ``smooth`` / ``smooth_at`` / ``line_ratio`` / ``moments``: ctypes
    wrappers over ``oracle.c`` (double precision, one ray at a time).
  * ``taps``: binomial, Gaussian and the paper's linear-sampling 9-tap kernels.
  * ``quant``: float16 / bfloat16 round-to-nearest-even, finite min/max.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import quant, taps  # noqa: F401
from .build import library_path, build

MIP0, MIP1, MIPRGB, AVIP0, AVIP1, AVIPRGB = range(6)
MODES = {"mip0": MIP0, "mip1": MIP1, "miprgb": MIPRGB, "avip0": AVIP0, "avip1": AVIP1,
         "aviprgb": AVIPRGB}
FILTERS = {"none": 0, "clip": 1, "scale": 2}


class _Camera(C.Structure):
    _fields_ = [("type", C.c_int32), ("eye", C.c_double * 3), ("U", C.c_double * 3),
                ("V", C.c_double * 3), ("W", C.c_double * 3), ("width", C.c_int32),
                ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("filter", C.c_int32), ("box_arm", C.c_int32),
                ("mip_alpha", C.c_int32), ("ratio", C.c_int32),
                ("opacity_from_lut", C.c_int32),
                ("k", C.c_double), ("min_val", C.c_double), ("ert", C.c_double),
                ("lo", C.c_double), ("hi", C.c_double), ("dt", C.c_double),
                ("min_t", C.c_double), ("max_t", C.c_double),
                ("min_t2", C.c_double), ("max_t2", C.c_double),
                ("ratio_lo", C.c_double), ("ratio_hi", C.c_double),
                ("star_n", C.c_int32), ("star_c0", C.c_double),
                ("star_off", C.c_double * 4), ("star_w", C.c_double * 4)]


class _Margins(C.Structure):
    _fields_ = [("ds", C.c_double), ("dv", C.c_double), ("da", C.c_double),
                ("dn", C.c_double), ("dr", C.c_double), ("pv", C.c_double),
                ("pt", C.c_double), ("pp", C.c_double)]


FRAG_COUNT, FRAG_ARGMAX, FRAG_ERT, FRAG_THRESHOLD, FRAG_RATIO, FRAG_COND = 1, 2, 4, 8, 16, 32
NOT_CANDIDATE = 64


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        P = C.POINTER
        L.orc_render.argtypes = [P(C.c_double), P(C.c_double), C.c_int32, C.c_int32, C.c_int32,
                                 P(_Camera), P(C.c_double), C.c_int32, P(_Params), P(_Margins),
                                 C.c_int64, P(C.c_int64), P(C.c_int32), P(C.c_double),
                                 P(C.c_uint8), P(C.c_int32), C.c_int32]
        L.orc_render_grad.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32,
                                      P(_Camera), P(C.c_double), C.c_int32, P(_Params),
                                      C.c_int64, P(C.c_int64), P(C.c_double), P(C.c_double),
                                      P(C.c_double), P(C.c_double)]
        L.orc_smooth.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32, P(C.c_double),
                                 C.c_int32, P(C.c_double), P(C.c_double), C.c_int32]
        L.orc_smooth_at.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32,
                                    P(C.c_double), C.c_int32, C.c_int64, P(C.c_int64),
                                    P(C.c_double)]
        L.orc_line_ratio.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                     P(C.c_double)]
        L.orc_moments.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_double, C.c_double, C.c_double, P(C.c_double),
                                  P(C.c_double), P(C.c_int32)]
        L.orc_pixel_ray.argtypes = [P(_Camera), C.c_int32, C.c_int32, P(C.c_double),
                                    P(C.c_double)]
        L.orc_ray_box.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(C.c_double), P(C.c_double),
                                  P(C.c_double), P(C.c_double)]
        L.orc_trilinear.argtypes = [P(C.c_double), C.c_int32, C.c_int32, C.c_int32,
                                    P(C.c_double)]
        L.orc_trilinear.restype = C.c_double
        for f in ("orc_render", "orc_render_grad", "orc_smooth", "orc_smooth_at",
                  "orc_line_ratio", "orc_moments", "orc_ray_box"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _cube64(cube):
    a = np.ascontiguousarray(cube, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("cube must be 3-D [z][y][x]")
    return a


def camera_struct(cam):
    c = _Camera()
    c.type = int(cam.type)
    for name in ("eye", "U", "V", "W"):
        getattr(c, name)[:] = [float(v) for v in getattr(cam, name)]
    c.width, c.height = int(cam.width), int(cam.height)
    return c


DEFAULTS = dict(mode="mip0", filter="none", box_arm=0, mip_alpha=0, ratio=0,
                opacity_from_lut=0, k=0.22, min_val=1e-6, ert=0.99, lo=0.0, hi=1.0, dt=0.5,
                min_t=-np.inf, max_t=np.inf, min_t2=-np.inf, max_t2=np.inf,
                ratio_lo=0.0, ratio_hi=1.0)


def params_struct(params):
    q = dict(DEFAULTS)
    q.update(params)
    p = _Params()
    p.mode = MODES[q["mode"]] if isinstance(q["mode"], str) else int(q["mode"])
    p.filter = FILTERS[q["filter"]] if isinstance(q["filter"], str) else int(q["filter"])
    for name in ("box_arm", "mip_alpha", "ratio", "opacity_from_lut"):
        setattr(p, name, int(q[name]))
    for name in ("k", "min_val", "ert", "lo", "hi", "dt", "min_t", "max_t", "min_t2",
                 "max_t2", "ratio_lo", "ratio_hi"):
        setattr(p, name, float(q[name]))
    # in-ray Gaussian (Section 4.2): star = (c0, [(off_1, w_1), ...]) or None
    if q.get("star"):
        c0, pairs = q["star"]
        p.star_n = len(pairs)
        p.star_c0 = float(c0)
        for i, (o, w) in enumerate(pairs):
            p.star_off[i] = float(o)
            p.star_w[i] = float(w)
    return p


DEFAULT_MARGINS = dict(ds=1e-5, dv=1e-5, da=2e-6, dn=1e-9, dr=0.0, pv=0.0, pt=5e-6, pp=0.0)


def render(cube, camera, lut, params, cube2=None, pixels=None, margins=None, nthreads=0,
           forced_n=None, bits=False):
    """FP64 render.  Returns (rgba[npix,4] float64, fragile[npix], nsamples[npix]);
    fragile is boolean, or the FRAG_* bit mask when bits=True.  forced_n[npix] (>= 0)
    makes AVIP rays composite exactly that many samples, and MIP1 / MIP_RGB rays take that
    sample as the arg-max (NOT_CANDIDATE set when it is not within ds of the maximum)."""
    V = _cube64(cube)
    V2 = _cube64(cube2) if cube2 is not None else None
    if V2 is not None and V2.shape != V.shape:
        raise ValueError("the two cubes of a ratio must share one grid")
    nz, ny, nx = V.shape
    L = np.ascontiguousarray(lut, dtype=np.float64).reshape(-1, 4)
    m = dict(DEFAULT_MARGINS)
    m.update(margins or {})
    mg = _Margins(**m)
    cam = camera_struct(camera)
    p = params_struct(params)
    if pixels is None:
        npix, pix = camera.width * camera.height, None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pix.size
    rgba = np.zeros((npix, 4), dtype=np.float64)
    frag = np.zeros(npix, dtype=np.uint8)
    ns = np.zeros(npix, dtype=np.int32)
    fn = None
    if forced_n is not None:
        fn = np.ascontiguousarray(forced_n, dtype=np.int32).reshape(-1)
        assert fn.size == npix
    rc = lib().orc_render(_dp(V), _dp(V2) if V2 is not None else None, nx, ny, nz,
                          C.byref(cam), _dp(L), L.shape[0], C.byref(p), C.byref(mg), npix,
                          pix.ctypes.data_as(C.POINTER(C.c_int64)) if pix is not None else None,
                          fn.ctypes.data_as(C.POINTER(C.c_int32)) if fn is not None else None,
                          _dp(rgba), frag.ctypes.data_as(C.POINTER(C.c_uint8)),
                          ns.ctypes.data_as(C.POINTER(C.c_int32)), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_render rejected its arguments (code {rc})")
    return rgba, (frag if bits else frag.astype(bool)), ns


def render_grad(cube, camera, tf, params, grad_rgba, pixels=None, want_vox=True):
    """FP64 AVIP0 render with table opacity and its exact reverse-mode derivative."""
    V = _cube64(cube)
    nz, ny, nx = V.shape
    T = np.ascontiguousarray(tf, dtype=np.float64).reshape(-1, 4)
    cam = camera_struct(camera)
    q = dict(params)
    q.setdefault("mode", "avip0")
    q["opacity_from_lut"] = 1
    p = params_struct(q)
    if pixels is None:
        npix, pix = camera.width * camera.height, None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pix.size
    g = np.ascontiguousarray(grad_rgba, dtype=np.float64).reshape(npix, 4)
    rgba = np.zeros((npix, 4))
    gtf = np.zeros_like(T)
    gvox = np.zeros(V.shape) if want_vox else None
    rc = lib().orc_render_grad(_dp(V), nx, ny, nz, C.byref(cam), _dp(T), T.shape[0],
                               C.byref(p), npix,
                               pix.ctypes.data_as(C.POINTER(C.c_int64)) if pix is not None
                               else None, _dp(g), _dp(rgba), _dp(gtf),
                               _dp(gvox) if gvox is not None else None)
    if rc != 0:
        raise ValueError(f"orc_render_grad rejected its arguments (code {rc})")
    return rgba, gtf, gvox


def smooth(cube, g, nthreads=0):
    V = _cube64(cube)
    nz, ny, nx = V.shape
    gg = np.ascontiguousarray(g, dtype=np.float64)
    out = np.empty_like(V)
    tmp = np.empty_like(V)
    if lib().orc_smooth(_dp(V), nx, ny, nz, _dp(gg), gg.size, _dp(out), _dp(tmp),
                        int(nthreads)) != 0:
        raise ValueError("orc_smooth rejected its arguments")
    return out


def smooth_at(cube, g, idx):
    V = _cube64(cube)
    nz, ny, nx = V.shape
    gg = np.ascontiguousarray(g, dtype=np.float64)
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(ii.size)
    if lib().orc_smooth_at(_dp(V), nx, ny, nz, _dp(gg), gg.size, ii.size,
                           ii.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out)) != 0:
        raise ValueError("orc_smooth_at rejected its arguments")
    return out


def line_ratio(cube, z0a, z0b, nzw, min_t_a=-np.inf, min_t_b=-np.inf, datamin=0.0):
    V = _cube64(cube)
    nz, ny, nx = V.shape
    out = np.empty((nzw, ny, nx))
    if lib().orc_line_ratio(_dp(V), nx, ny, nz, z0a, z0b, nzw, float(min_t_a), float(min_t_b),
                            float(datamin), _dp(out)) != 0:
        raise ValueError("orc_line_ratio rejected its arguments")
    return out


def moments(cube, z0=0, nzw=None, dv=1.0, min_t=-np.inf, max_t=np.inf):
    """Moment maps (Section 2.2, Eq. mom0 / Eq. mom1 and the argmax variant) of each spectrum
    over channels [z0, z0 + nzw): (m0, m1, argmax), each [ny, nx]."""
    V = _cube64(cube)
    nz, ny, nx = V.shape
    nzw = nz - z0 if nzw is None else nzw
    m0 = np.empty((ny, nx))
    m1 = np.empty((ny, nx))
    am = np.empty((ny, nx), dtype=np.int32)
    if lib().orc_moments(_dp(V), nx, ny, nz, z0, nzw, float(dv), float(min_t), float(max_t),
                         _dp(m0), _dp(m1), am.ctypes.data_as(C.POINTER(C.c_int32))) != 0:
        raise ValueError("orc_moments rejected its arguments")
    return m0, m1, am


def pixel_ray(camera, px, py):
    cam = camera_struct(camera)
    o = np.zeros(3)
    d = np.zeros(3)
    lib().orc_pixel_ray(C.byref(cam), px, py, _dp(o), _dp(d))
    return o, d


def ray_box(shape_zyx, o, d):
    nz, ny, nx = shape_zyx
    t0 = C.c_double()
    t1 = C.c_double()
    oo = np.ascontiguousarray(o, dtype=np.float64)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    hit = lib().orc_ray_box(nx, ny, nz, _dp(oo), _dp(dd), C.byref(t0), C.byref(t1))
    return (t0.value, t1.value) if hit else None


def trilinear(cube, p):
    V = _cube64(cube)
    nz, ny, nx = V.shape
    pp = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_trilinear(_dp(V), nx, ny, nz, _dp(pp))
