"""ctypes declarations of the libsvr C ABI (include/svr.h).  No computation lives here."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SVR_LIBRARY may name another build of the same library (the tests load a build whose
# host code carries AddressSanitizer); by default the in-tree libsvr.so
LIB_PATH = os.environ.get("SVR_LIBRARY") or os.path.join(HERE, "libsvr.so")

SVR_OK, SVR_EINVAL, SVR_ENOMEM, SVR_EHIP, SVR_EUNSUPPORTED = range(5)
SVR_F32, SVR_F16, SVR_BF16 = range(3)
SVR_MIP0, SVR_MIP1, SVR_MIPRGB, SVR_AVIP0, SVR_AVIP1, SVR_AVIPRGB = range(6)
SVR_FILTER_NONE, SVR_FILTER_CLIP, SVR_FILTER_SCALE = range(3)
SVR_MAX_LUT = 1024
SVR_MAX_BOX_ARM = 15
SVR_MAX_TAPS = 63

# every symbol include/svr.h declares
EXPORTS = (
    "svr_status_string", "svr_last_error", "svr_version", "svr_minmax", "svr_minmax_noalloc",
    "svr_volume_create", "svr_volume_destroy", "svr_volume_upload", "svr_volume_info",
    "svr_volume_clim",
    "svr_volume_export", "svr_params_validate", "svr_render", "svr_render_segments", "svr_smooth_workspace",
    "svr_smooth",
    "svr_line_ratio", "svr_moments", "svr_render_train_workspace", "svr_render_train",
    "svr_render_backward", "svr_batch_create", "svr_batch_launch", "svr_batch_info",
    "svr_batch_destroy", "svr_set_tune_cache", "svr_sync",
)


class CubeView(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("nx", C.c_int32),
                ("ny", C.c_int32), ("nz", C.c_int32), ("sx", C.c_int64), ("sy", C.c_int64),
                ("sz", C.c_int64)]


class Camera(C.Structure):
    _fields_ = [("type", C.c_int32), ("eye", C.c_float * 3), ("U", C.c_float * 3),
                ("V", C.c_float * 3), ("W", C.c_float * 3), ("width", C.c_int32),
                ("height", C.c_int32)]


class Lut(C.Structure):
    _fields_ = [("rgba", C.c_void_p), ("n", C.c_int32)]


class BatchStats(C.Structure):
    _fields_ = [("items", C.c_int64), ("grid", C.c_int32), ("tile_waves_x", C.c_int32),
                ("brick", C.c_int32), ("from_cache", C.c_int32), ("default_ms", C.c_float),
                ("tuned_ms", C.c_float)]


class Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("filter", C.c_int32), ("box_arm", C.c_int32),
                ("mip_alpha", C.c_int32), ("ratio", C.c_int32), ("opacity_from_lut", C.c_int32),
                ("k", C.c_float), ("min_val", C.c_float), ("ert", C.c_float),
                ("clim_lo", C.c_float), ("clim_hi", C.c_float), ("dt", C.c_float),
                ("min_t", C.c_float), ("max_t", C.c_float), ("min_t2", C.c_float),
                ("max_t2", C.c_float), ("ratio_lo", C.c_float), ("ratio_hi", C.c_float),
                ("star_n", C.c_int32), ("star_c0", C.c_float), ("star_off", C.c_float * 4),
                ("star_w", C.c_float * 4)]


_lib = None


def load():
    """Load libsvr.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_1707_00442_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    P, vp, i32, i64, f32 = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_float
    sig = {
        "svr_status_string": (C.c_char_p, [C.c_int]),
        "svr_last_error": (C.c_char_p, []),
        "svr_version": (C.c_char_p, []),
        "svr_minmax": (C.c_int, [P(CubeView), P(f32), vp]),
        "svr_minmax_noalloc": (C.c_int, [P(CubeView), vp, vp]),
        "svr_volume_create": (C.c_int, [P(CubeView), i32, i32, f32, vp, P(vp)]),
        "svr_volume_destroy": (C.c_int, [vp]),
        "svr_volume_upload": (C.c_int, [vp, P(CubeView), f32, vp]),
        "svr_volume_info": (C.c_int, [vp, P(i32), P(i32), P(i32), P(i64)]),
        "svr_volume_clim": (C.c_int, [vp, P(f32), vp]),
        "svr_volume_export": (C.c_int, [vp, vp, vp]),
        "svr_params_validate": (C.c_int, [P(Params)]),
        "svr_render": (C.c_int, [vp, vp, P(Camera), P(Lut), P(Params), vp, vp, vp]),
        "svr_render_segments": (C.c_int, [vp, P(Camera), P(Params), P(C.c_int32)]),
        "svr_smooth_workspace": (C.c_int, [P(CubeView), i32, P(C.c_size_t)]),
        "svr_smooth": (C.c_int, [P(CubeView), P(f32), i32, vp, vp, C.c_size_t, vp]),
        "svr_line_ratio": (C.c_int, [P(CubeView), i32, i32, i32, f32, f32, f32, vp, vp]),
        "svr_moments": (C.c_int, [P(CubeView), i32, i32, f32, f32, f32, vp, vp, vp, vp]),
        "svr_render_train_workspace": (C.c_int, [vp, P(Camera), P(Params), P(C.c_size_t)]),
        "svr_render_train": (C.c_int, [vp, P(Camera), P(Lut), P(Params), vp, vp, C.c_size_t,
                                       vp]),
        "svr_render_backward": (C.c_int, [vp, P(Camera), P(Lut), P(Params), vp, C.c_size_t,
                                          vp, vp, vp, vp]),
        "svr_batch_create": (C.c_int, [P(vp), P(Camera), i32, P(Lut), P(Params), P(vp), i32,
                                       vp, P(vp)]),
        "svr_batch_launch": (C.c_int, [vp, vp]),
        "svr_batch_info": (C.c_int, [vp, P(BatchStats)]),
        "svr_batch_destroy": (C.c_int, [vp]),
        "svr_set_tune_cache": (C.c_int, [C.c_char_p]),
        "svr_sync": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
