"""svr: MI355X-native ray-cast colouring and filtering of spectral cubes.

Thin Python binding over the libsvr C ABI (include/svr.h): argument marshalling only.
Every step of the rendering, smoothing, line-ratio, adjoint and batched paths runs in the
hand-written HIP kernels of libsvr.so; PyTorch supplies device memory and streams.  There
is no CPU fallback: if the library is missing, importing the functions raises.

Functions keep the C names (svr_render, svr_smooth, svr_line_ratio, svr_moments, ...).  Tensors are
CUDA (HIP) tensors, cubes are [z][y][x] (x = RA fastest, y = Dec, z = velocity).
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _capi
from ._capi import (  # noqa: F401
    SVR_F32, SVR_F16, SVR_BF16, SVR_MIP0, SVR_MIP1, SVR_MIPRGB, SVR_AVIP0, SVR_AVIP1,
    SVR_AVIPRGB, SVR_FILTER_NONE, SVR_FILTER_CLIP, SVR_FILTER_SCALE, EXPORTS,
)

MODES = {"mip0": SVR_MIP0, "mip1": SVR_MIP1, "miprgb": SVR_MIPRGB, "avip0": SVR_AVIP0,
         "avip1": SVR_AVIP1, "aviprgb": SVR_AVIPRGB}
FILTERS = {"none": SVR_FILTER_NONE, "clip": SVR_FILTER_CLIP, "scale": SVR_FILTER_SCALE}
STORAGE = {"f32": SVR_F32, "f16": SVR_F16, "bf16": SVR_BF16}
_TORCH_DT = {torch.float32: SVR_F32, torch.float16: SVR_F16, torch.bfloat16: SVR_BF16}
_DT_TORCH = {v: k for k, v in _TORCH_DT.items()}


class SvrError(RuntimeError):
    def __init__(self, status, where):
        L = _capi.load()
        self.status = status
        msg = L.svr_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.svr_status_string(status).decode()} ({msg})")


def lib():
    return _capi.load()


def _check(status, where):
    if status != 0:
        raise SvrError(status, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _cuda(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    return t


def cube_view(cube):
    """svr_cube_view of a 3-D [z][y][x] tensor (strided views allowed)."""
    _cuda(cube, "cube")
    if cube.dim() != 3 or cube.dtype not in _TORCH_DT:
        raise TypeError("cube must be a 3-D float32/float16/bfloat16 tensor [z][y][x]")
    v = _capi.CubeView()
    v.data = cube.data_ptr()
    v.dtype = _TORCH_DT[cube.dtype]
    v.nz, v.ny, v.nx = cube.shape
    if cube.is_contiguous():
        v.sx = v.sy = v.sz = 0
    else:
        v.sz, v.sy, v.sx = cube.stride()
    return v


def camera_struct(cam):
    """svr_camera from any object with type/eye/U/V/W/width/height attributes."""
    c = _capi.Camera()
    c.type = int(cam.type)
    for name in ("eye", "U", "V", "W"):
        getattr(c, name)[:] = [float(x) for x in getattr(cam, name)]
    c.width, c.height = int(cam.width), int(cam.height)
    return c


PARAM_DEFAULTS = dict(mode="mip0", filter="none", box_arm=0, mip_alpha=0, ratio=0,
                      opacity_from_lut=0, k=0.22, min_val=1e-6, ert=0.99, clim_lo=0.0,
                      clim_hi=0.0, dt=0.5, min_t=-math.inf, max_t=math.inf,
                      min_t2=-math.inf, max_t2=math.inf, ratio_lo=0.0, ratio_hi=1.0,
                      star=None)


def params_struct(params=None, **kw):
    """svr_params from a dict / keywords (names as in include/svr.h; clim_hi <= clim_lo
    selects the volume's own finite min/max)."""
    if isinstance(params, _capi.Params):
        return params
    q = dict(PARAM_DEFAULTS)
    q.update(params or {})
    q.update(kw)
    p = _capi.Params()
    p.mode = MODES[q["mode"]] if isinstance(q["mode"], str) else int(q["mode"])
    p.filter = FILTERS[q["filter"]] if isinstance(q["filter"], str) else int(q["filter"])
    for name in ("box_arm", "mip_alpha", "ratio", "opacity_from_lut"):
        setattr(p, name, int(q[name]))
    for name in ("k", "min_val", "ert", "clim_lo", "clim_hi", "dt", "min_t", "max_t",
                 "min_t2", "max_t2", "ratio_lo", "ratio_hi"):
        setattr(p, name, float(q[name]))
    # in-ray Gaussian (Section 4.2): star = (c0, [(off_1, w_1), ...]) or None
    if q["star"]:
        c0, pairs = q["star"]
        if len(pairs) > 4:
            raise ValueError("at most 4 (offset, weight) pairs")
        p.star_n = len(pairs)
        p.star_c0 = float(c0)
        for i, (o, w) in enumerate(pairs):
            p.star_off[i] = float(o)
            p.star_w[i] = float(w)
    return p


def lut_struct(lut):
    _cuda(lut, "colour table")
    if lut.dtype != torch.float32 or lut.dim() != 2 or lut.shape[1] != 4 or not lut.is_contiguous():
        raise TypeError("colour table must be a contiguous float32 [n, 4] tensor")
    t = _capi.Lut()
    t.rgba = lut.data_ptr()
    t.n = lut.shape[0]
    return t


# ------------------------------------------------------------------------------- volumes
class Volume:
    """Owner of an svr_volume handle (library-owned bricked copy of a cube)."""

    def __init__(self, handle, shape, storage, brick):
        self.handle = handle
        self.shape = shape            # (nz, ny, nx)
        self.storage = storage        # SVR_F32 / SVR_F16 / SVR_BF16
        self.brick = brick

    def close(self):
        if self.handle:
            # the library frees device memory; make sure no queued work still reads it
            torch.cuda.synchronize()
            _check(lib().svr_volume_destroy(self.handle), "svr_volume_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return C.c_void_p(self.handle)

    @property
    def nbytes(self):
        """Device bytes the volume holds (bricked storage with apron and padding)."""
        return svr_volume_info(self)["bytes"]


def svr_volume_create(cube, storage="f32", brick=8, nan_fill=float("nan"), stream=None):
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    v = cube_view(cube)
    h = C.c_void_p()
    _check(lib().svr_volume_create(C.byref(v), st, int(brick), float(nan_fill), _stream(stream),
                                   C.byref(h)), "svr_volume_create")
    return Volume(h.value, tuple(cube.shape), st, int(brick) or 8)


def svr_volume_destroy(vol):
    vol.close()


def svr_volume_upload(vol, cube, nan_fill=float("nan"), stream=None):
    v = cube_view(cube)
    _check(lib().svr_volume_upload(vol, C.byref(v), float(nan_fill), _stream(stream)),
           "svr_volume_upload")


def svr_volume_info(vol):
    dims = (C.c_int32 * 3)()
    st, br = C.c_int32(), C.c_int32()
    nb = C.c_int64()
    _check(lib().svr_volume_info(vol, dims, C.byref(st), C.byref(br), C.byref(nb)),
           "svr_volume_info")
    return dict(dims_zyx=tuple(dims), storage=st.value, brick=br.value, bytes=nb.value)


def svr_volume_clim(vol, stream=None):
    out = (C.c_float * 2)()
    _check(lib().svr_volume_clim(vol, out, _stream(stream)), "svr_volume_clim")
    return float(out[0]), float(out[1])


def svr_volume_export(vol, stream=None):
    out = torch.empty(vol.shape, dtype=_DT_TORCH[vol.storage], device="cuda")
    _check(lib().svr_volume_export(vol, C.c_void_p(out.data_ptr()), _stream(stream)),
           "svr_volume_export")
    return out


def svr_minmax(cube, stream=None):
    v = cube_view(cube)
    out = (C.c_float * 2)()
    _check(lib().svr_minmax(C.byref(v), out, _stream(stream)), "svr_minmax")
    return float(out[0]), float(out[1])


def svr_minmax_noalloc(cube, out, stream=None):
    """Allocation-free finite min/max into `out` (a float32 CUDA tensor of 2 elements),
    asynchronous on the stream."""
    v = cube_view(cube)
    _cuda(out, "out")
    if out.dtype != torch.float32 or out.numel() < 2 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float32 tensor of at least 2 elements")
    _check(lib().svr_minmax_noalloc(C.byref(v), C.c_void_p(out.data_ptr()), _stream(stream)),
           "svr_minmax_noalloc")
    return out


# ------------------------------------------------------------------------------- render
def svr_params_validate(params=None, **kw):
    p = params_struct(params, **kw)
    _check(lib().svr_params_validate(C.byref(p)), "svr_params_validate")


def svr_render(vol, camera, lut, params=None, vol2=None, out=None, samples=False,
               stream=None, **kw):
    """Render one image -> float32 tensor [height][width][4] (and per-pixel sample counts
    when samples=True)."""
    cam = camera_struct(camera)
    p = params_struct(params, **kw)
    t = lut_struct(lut)
    if out is None:
        out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
    ns = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda") if samples else None
    _check(lib().svr_render(vol, vol2 if vol2 is not None else None, C.byref(cam), C.byref(t),
                            C.byref(p), C.c_void_p(out.data_ptr()),
                            C.c_void_p(ns.data_ptr()) if ns is not None else None,
                            _stream(stream)), "svr_render")
    return (out, ns) if samples else out


def svr_render_segments(vol, camera, params=None, **kw):
    """Segments svr_render splits each ray of this view into (1: one pass per ray)."""
    cam = camera_struct(camera)
    p = params_struct(params, **kw)
    n = C.c_int32(0)
    _check(lib().svr_render_segments(vol, C.byref(cam), C.byref(p), C.byref(n)),
           "svr_render_segments")
    return int(n.value)


# ------------------------------------------------------------------------------- smoothing
def svr_smooth_workspace(cube, ntaps):
    """Device bytes of workspace svr_smooth needs for `ntaps` taps (0 for the fused kernels)."""
    v = cube_view(cube)
    n = C.c_size_t()
    _check(lib().svr_smooth_workspace(C.byref(v), int(ntaps), C.byref(n)),
           "svr_smooth_workspace")
    return n.value


def svr_smooth(cube, taps, out=None, workspace=None, stream=None):
    v = cube_view(cube)
    g = (C.c_float * len(taps))(*[float(x) for x in taps])
    if out is None:
        out = torch.empty_like(cube, memory_format=torch.contiguous_format)
    need = svr_smooth_workspace(cube, len(taps))
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    ws_ptr = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().svr_smooth(C.byref(v), g, len(taps), C.c_void_p(out.data_ptr()), ws_ptr,
                            ws_bytes, _stream(stream)), "svr_smooth")
    return out


def svr_line_ratio(cube, z0_a, z0_b, nz_w, min_t_a=-math.inf, min_t_b=-math.inf, datamin=0.0,
                   out=None, stream=None):
    v = cube_view(cube)
    nz, ny, nx = cube.shape
    if out is None:
        out = torch.empty((nz_w, ny, nx), dtype=torch.float32, device="cuda")
    _check(lib().svr_line_ratio(C.byref(v), int(z0_a), int(z0_b), int(nz_w), float(min_t_a),
                                float(min_t_b), float(datamin), C.c_void_p(out.data_ptr()),
                                _stream(stream)), "svr_line_ratio")
    return out


def svr_moments(cube, z0=0, nz_w=None, dv=1.0, min_t=-math.inf, max_t=math.inf, out=None,
                stream=None):
    """Moment maps of every spectrum over channels [z0, z0 + nz_w): (m0, m1, argmax), float32,
    float32 and int32 tensors of shape [ny, nx] (out: an optional triple of such tensors)."""
    v = cube_view(cube)
    nz, ny, nx = cube.shape
    nz_w = nz - z0 if nz_w is None else nz_w
    if out is None:
        out = (torch.empty((ny, nx), dtype=torch.float32, device="cuda"),
               torch.empty((ny, nx), dtype=torch.float32, device="cuda"),
               torch.empty((ny, nx), dtype=torch.int32, device="cuda"))
    ptr = [C.c_void_p(t.data_ptr()) if t is not None else None for t in out]
    _check(lib().svr_moments(C.byref(v), int(z0), int(nz_w), float(dv), float(min_t),
                             float(max_t), ptr[0], ptr[1], ptr[2], _stream(stream)),
           "svr_moments")
    return out


def svr_sync(stream=None):
    _check(lib().svr_sync(_stream(stream)), "svr_sync")


from ._train import (  # noqa: E402,F401
    svr_render_train_workspace, svr_render_train, svr_render_backward, RenderFn,
)
from ._batch import (  # noqa: E402,F401
    Batch, svr_batch_create, svr_batch_launch, svr_batch_info, svr_batch_destroy,
    svr_set_tune_cache,
)
