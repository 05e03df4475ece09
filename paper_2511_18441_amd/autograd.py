"""torch.autograd.Function over the hand-written HIP backward (recogs_render_backward).

Differentiable inputs: the activated opacities, the SH DC coefficients (the first
three planes of the scene's SH array) and the fused recolour matrix M; gradients of
eq. (8) restricted to those, as the refit of the paper updates colour only (Sec. 3.3).

The backward replays the per-tile state the forward left in its workspace, so the
workspace must not render anything else in between: a loss over several views uses
one workspace per view. The forward records the workspace's render generation and the
backward raises if another render has run on it since.
"""
from __future__ import annotations

import torch

from .binding import camera_struct, opts_struct, recogs_render_backward, render


class RecogsRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, opacity, sh_dc, M, dscene, cam, ws, mask, b, tile=(16, 16), ppt=1, bg=(0.0, 0.0, 0.0)):
        if opacity.data_ptr() != dscene.opacity.data_ptr() or sh_dc.data_ptr() != dscene.sh.data_ptr():
            raise ValueError("opacity and sh_dc must be the scene's own opacity and leading SH planes")
        Mc = M.detach().contiguous().reshape(9) if M is not None else None
        image = render(dscene, cam, ws, tile, ppt, bg, mask, Mc, b, keep_backward=True)
        ctx.save_for_backward(image)
        ctx.stamp = (ws.ws, int(ws.ws.generation))
        ctx.args = (dscene, cam, ws, mask, Mc, b, tile, ppt, bg, opacity.dtype, sh_dc.dtype, M is not None)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        (image,) = ctx.saved_tensors
        dscene, cam, ws, mask, Mc, b, tile, ppt, bg, op_dt, sh_dt, has_M = ctx.args
        if ws.ws is not ctx.stamp[0] or int(ws.ws.generation) != ctx.stamp[1]:
            raise RuntimeError("the workspace rendered again after this forward: its state now belongs to another "
                               "render (use one workspace per view)")
        n = dscene.n
        dev = image.device
        g = grad_image.detach().to(torch.float32).contiguous()
        dop = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        ddc = torch.empty((3, max(n, 1)), dtype=torch.float32, device=dev)
        dM = torch.empty(9, dtype=torch.float32, device=dev)
        o = opts_struct(tile, ppt, bg, mask, Mc, b, keep_backward=True)
        recogs_render_backward(dscene.c_struct(), camera_struct(cam), o, ws.ws, image.data_ptr(), g.data_ptr(),
                               dop.data_ptr(), ddc.data_ptr(), dM.data_ptr())
        gop = torch.zeros(dscene.stride, dtype=op_dt, device=dev)
        gop[:n] = dop[:n].to(op_dt)
        gdc = torch.zeros((3, dscene.stride), dtype=sh_dt, device=dev)
        gdc[:, :n] = ddc[:, :n].to(sh_dt)
        return (gop, gdc, dM.view(3, 3) if has_M else None) + (None,) * 8
