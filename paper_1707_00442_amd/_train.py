"""Differentiable AVIP0 render: marshalling for svr_render_train / svr_render_backward."""
from __future__ import annotations

import ctypes as C

import torch

from . import _capi


def _p():
    from . import (lib, _check, _stream, camera_struct, params_struct, lut_struct)
    return lib, _check, _stream, camera_struct, params_struct, lut_struct


def svr_render_train_workspace(vol, camera, params=None, **kw):
    lib, _check, _stream, camera_struct, params_struct, _ = _p()
    cam = camera_struct(camera)
    p = params_struct(params, **kw)
    n = C.c_size_t()
    _check(lib().svr_render_train_workspace(vol, C.byref(cam), C.byref(p), C.byref(n)),
           "svr_render_train_workspace")
    return n.value


def svr_render_train(vol, camera, tf, params=None, out=None, workspace=None, stream=None, **kw):
    lib, _check, _stream, camera_struct, params_struct, lut_struct = _p()
    cam = camera_struct(camera)
    p = params_struct(params, **kw)
    t = lut_struct(tf)
    if out is None:
        out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
    need = svr_render_train_workspace(vol, camera, p)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    _check(lib().svr_render_train(vol, C.byref(cam), C.byref(t), C.byref(p),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), _stream(stream)), "svr_render_train")
    return out, workspace


def svr_render_backward(vol, camera, tf, params, workspace, grad_rgba, grad_tf=None,
                        grad_vox=None, stream=None, want_vox=True):
    lib, _check, _stream, camera_struct, params_struct, lut_struct = _p()
    cam = camera_struct(camera)
    p = params_struct(params)
    t = lut_struct(tf)
    g = grad_rgba.contiguous().float()
    if grad_tf is None:
        grad_tf = torch.zeros_like(tf)
    if grad_vox is None and want_vox:
        grad_vox = torch.zeros(vol.shape, dtype=torch.float32, device="cuda")
    _check(lib().svr_render_backward(vol, C.byref(cam), C.byref(t), C.byref(p),
                                     C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     C.c_void_p(g.data_ptr()), C.c_void_p(grad_tf.data_ptr()),
                                     C.c_void_p(grad_vox.data_ptr()) if grad_vox is not None
                                     else None, _stream(stream)), "svr_render_backward")
    return grad_tf, grad_vox


class RenderFn(torch.autograd.Function):
    """image = RenderFn.apply(cube, tf, camera, params, storage, brick).

    Forward: uploads `cube` into a volume and runs svr_render_train (AVIP0 with the
    piecewise-linear RGBA transfer function `tf` [n, 4]).  Backward: svr_render_backward,
    giving dL/dtf and dL/dcube (float32, [z][y][x])."""

    @staticmethod
    def forward(ctx, cube, tf, camera, params, storage="f32", brick=8):
        from . import svr_volume_create
        vol = svr_volume_create(cube.detach(), storage=storage, brick=brick)
        tfc = tf.detach().contiguous().float()
        img, ws = svr_render_train(vol, camera, tfc, params)
        ctx.vol, ctx.ws, ctx.camera, ctx.params, ctx.tf = vol, ws, camera, params, tfc
        ctx.cube_dtype = cube.dtype
        ctx.needs = (ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return img

    @staticmethod
    def backward(ctx, grad_img):
        gtf, gvox = svr_render_backward(ctx.vol, ctx.camera, ctx.tf, ctx.params, ctx.ws,
                                        grad_img, want_vox=ctx.needs[0])
        return (gvox.to(ctx.cube_dtype) if ctx.needs[0] else None,
                gtf if ctx.needs[1] else None, None, None, None, None)


__all__ = ["svr_render_train_workspace", "svr_render_train", "svr_render_backward", "RenderFn",
           "_capi"]
