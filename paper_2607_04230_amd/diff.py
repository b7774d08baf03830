"""Differentiable soft-coverage rendering of a strand stream.

SoftRender.apply(pos_w, rgb, ctx) renders the stream with the SOFT resolve
(coverage of the visible segment under a Gaussian pixel filter, shaded once
per pixel).  Visibility is held fixed: the forward pass rasterizes the
visibility buffer and does not keep it; the backward pass rasterizes it again
(bit-identical, the raster is deterministic) and runs the hand-written
gradient kernel hm_resolve_shade_bwd, which accumulates dLoss/d(position,
width) and dLoss/d(colour) with fp32 atomics.
"""
from __future__ import annotations

import torch

from . import hm
from .scenes import MODE_SOFT, ResolveParams


class SoftContext:
    """Fixed (non-differentiated) parts of a soft render: flags, scene offsets,
    cameras, frame, workspaces and the visibility scratch buffer."""

    def __init__(self, flags, scene_off, cams, width, height, r_min=1.0, resolve=None,
                 bg=(0.0, 0.0, 0.0), rparams=None):
        S = scene_off.shape[0] - 1
        self.flags, self.scene_off, self.cams = flags, scene_off, cams
        self.cap = flags.shape[0]
        self.fr = hm.frame(S, width, height)
        self.rparams = rparams or hm.raster_defaults(self.fr)
        self.rparams.r_min = r_min
        self.sp = hm.shade_params(resolve or ResolveParams(), MODE_SOFT, bg)
        dev = flags.device
        self.vis = torch.empty((S, 2, height, width), dtype=torch.int64, device=dev)
        self.ws = torch.empty(hm.workspace_size(hm.CALL_RASTER, self.fr, cap=self.cap,
                                                rparams=self.rparams), dtype=torch.uint8,
                              device=dev)
        self.ws_res = torch.empty(max(hm.workspace_size(hm.CALL_RESOLVE, self.fr), 1),
                                  dtype=torch.uint8, device=dev)
        self.shape = (S, height, width, 4)

    def strands(self, pos_w, rgb):
        return hm.strands(pos_w, rgb, self.flags, self.scene_off, self.cap)

    def raster(self, pos_w, rgb):
        hm.raster_vis(self.strands(pos_w, rgb), self.cams, self.fr, self.rparams, None, self.vis,
                      self.ws)

    def forward(self, pos_w, rgb, out=None):
        out = torch.empty(self.shape, dtype=torch.float32, device=pos_w.device) if out is None else out
        self.raster(pos_w, rgb)
        hm.resolve_shade(self.strands(pos_w, rgb), self.vis, self.cams, self.fr, self.sp, out,
                         self.ws_res)
        return out

    def backward(self, pos_w, rgb, d_out, gpos, grgb):
        self.raster(pos_w, rgb)                      # recompute visibility
        hm.resolve_shade_bwd(self.strands(pos_w, rgb), self.vis, self.cams, self.fr, self.sp,
                             d_out, gpos, grgb)


class SoftRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos_w, rgb, sctx: SoftContext):
        pos_w = pos_w.contiguous()
        rgb = rgb.contiguous()
        out = sctx.forward(pos_w, rgb)
        ctx.save_for_backward(pos_w, rgb)
        ctx.sctx = sctx
        return out

    @staticmethod
    def backward(ctx, d_out):
        pos_w, rgb = ctx.saved_tensors
        gpos = torch.zeros_like(pos_w)
        grgb = torch.zeros_like(rgb)
        ctx.sctx.backward(pos_w, rgb, d_out.contiguous(), gpos, grgb)
        return gpos, grgb, None


def soft_render(pos_w, rgb, sctx: SoftContext):
    return SoftRender.apply(pos_w, rgb, sctx)
