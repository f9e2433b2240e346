"""Batched persistent rendering: marshalling for svr_batch_*."""
from __future__ import annotations

import ctypes as C

import torch


class Batch:
    """Owner of an svr_batch handle; keeps the volumes, table and outputs alive."""

    def __init__(self, handle, vols, lut, outs):
        self.handle, self.vols, self.lut, self.outs = handle, vols, lut, outs
        self.stats = {}

    def __getattr__(self, name):
        # items, grid, tile_waves_x, brick, from_cache, default_ms, tuned_ms
        stats = self.__dict__.get("stats", {})
        if name in stats:
            return stats[name]
        raise AttributeError(name)

    @property
    def _as_parameter_(self):
        return C.c_void_p(self.handle)

    def launch(self, stream=None):
        svr_batch_launch(self, stream)
        return self.outs

    def close(self):
        if self.handle:
            from . import lib, _check
            torch.cuda.synchronize()
            _check(lib().svr_batch_destroy(self.handle), "svr_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def svr_batch_create(vols, cameras, lut, params=None, outs=None, tune=0, stream=None, **kw):
    """tune: 0 default shape, 1 (or True) tuned with the cache, 2 always search."""
    from . import _capi, lib, _check, _stream, camera_struct, params_struct, lut_struct
    n = len(vols)
    cams = (_capi.Camera * n)(*[camera_struct(c) for c in cameras])
    if outs is None:
        outs = [torch.empty((c.height, c.width, 4), dtype=torch.float32, device="cuda")
                for c in cameras]
    hv = (C.c_void_p * n)(*[v.handle for v in vols])
    ho = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    p = params_struct(params, **kw)
    t = lut_struct(lut)
    h = C.c_void_p()
    _check(lib().svr_batch_create(hv, cams, n, C.byref(t), C.byref(p), ho, int(tune),
                                  _stream(stream), C.byref(h)), "svr_batch_create")
    b = Batch(h.value, list(vols), lut, outs)
    b.stats = svr_batch_info(b)
    return b


def svr_batch_launch(batch, stream=None):
    from . import lib, _check, _stream
    _check(lib().svr_batch_launch(batch, _stream(stream)), "svr_batch_launch")


def svr_batch_info(batch):
    """The launch the batch replays, as a dict (fields of svr_batch_stats)."""
    from . import lib, _check, _capi
    st = _capi.BatchStats()
    _check(lib().svr_batch_info(batch, C.byref(st)), "svr_batch_info")
    return {name: getattr(st, name) for name, _ in _capi.BatchStats._fields_}


def svr_set_tune_cache(path):
    """Tuning cache file of the batched autotuner (None: no cache)."""
    from . import lib, _check
    _check(lib().svr_set_tune_cache(path.encode() if path else None), "svr_set_tune_cache")


def svr_batch_destroy(batch):
    batch.close()
