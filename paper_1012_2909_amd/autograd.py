"""Differentiable rendering: a torch.autograd.Function around the HIP
forward and adjoint kernels.

The forward pass renders the composite image and keeps, per pixel, only the
number of samples taken and the transmittance at every 8th sample
(vr.CHECKPOINT_INTERVAL); the backward pass replays each segment from its
checkpoint and accumulates gradients with respect to the transfer-function table and the
voxels.  Both run in the library's kernels; this module only marshals
tensors.
"""
from __future__ import annotations

import torch

from . import vr


class VolumeRenderFn(torch.autograd.Function):
    """image = VolumeRenderFn.apply(volume, table, renderer, camera, vmin, vmax, step, ert)

    volume: float32 (nz, ny, nx) cuda tensor; table: float32 (n, 4) cuda tensor
    (straight RGBA over [vmin, vmax]).  Returns premultiplied RGBA (h, w, 4).
    """

    @staticmethod
    def forward(ctx, volume, table, renderer: "vr.Renderer", camera, vmin: float, vmax: float,
                step: float = 0.5, ert: float = 0.99):
        vol, tab = volume.detach(), table.detach()
        renderer.load_volume(vol, storage="f32", brick=0, orientations=1)
        renderer.set_transfer_function(tab, vmin, vmax)
        renderer.set_camera(camera)
        img, ws = renderer.render("composite", "trilinear", step, ert, save=True)
        ctx.renderer = renderer
        ctx.ws = ws
        ctx.cfg = (step, ert)
        # what the forward rendered from, so that the backward replays the
        # same rays even if the renderer was used in between
        ctx.scene = (vol, tab, camera, vmin, vmax)
        ctx.generation = renderer.generation
        ctx.shapes = (volume.shape, table.shape)
        ctx.needs = (volume.requires_grad, table.requires_grad)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        step, ert = ctx.cfg
        vshape, tshape = ctx.shapes
        R = ctx.renderer
        if R.generation != ctx.generation:
            vol, tab, camera, vmin, vmax = ctx.scene
            R.load_volume(vol, storage="f32", brick=0, orientations=1)
            R.set_transfer_function(tab, vmin, vmax)
            R.set_camera(camera)
        dev = grad_img.device
        gv = torch.zeros(vshape, dtype=torch.float32, device=dev) if ctx.needs[0] else None
        gl = torch.zeros(tshape, dtype=torch.float32, device=dev) if ctx.needs[1] else None
        R.render_backward(grad_img.contiguous(), ctx.ws, gl, gv, step=step, ert=ert)
        return gv, gl, None, None, None, None, None, None


def render(volume, table, renderer, camera, vmin, vmax, step=0.5, ert=0.99):
    return VolumeRenderFn.apply(volume, table, renderer, camera, vmin, vmax, step, ert)
