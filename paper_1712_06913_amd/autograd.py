"""torch.autograd wrappers of the imaging operator and its adjoint.

ImagingOp:  vis (complex64, all instances packed)  ->  dirty images (float32, packed)
            forward = mi_dirty_image, backward = mi_degrid(adjoint=1), i.e.
            A^T y = (2 w_k / B0) P(y)_k  (the transpose under <a,b> = sum a b and
            <v,u> = Re sum conj(v) u; for torch's complex gradient convention the
            gradient of a real loss w.r.t. v is exactly that vector).
PredictOp:  model image (float32, packed) -> model visibilities P(model) (complex64)
            forward = mi_degrid(adjoint=0), backward = mi_predict_transpose: the imager
            with unit weights on the kept visibilities, scaled by 1/(2 corr) instead of
            1/(corr B0), P^T(v) = sum_k Re(v_k S_k(x)) / corr(x).

Both run entirely in the HIP library; these classes only wire the calls together.
"""
from __future__ import annotations

import torch

from . import api


class ImagingOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vis, batch, uv, w):
        dirty, _, _ = api.dirty_image(batch, vis.contiguous(), uv, w, beam=False)
        ctx.batch, ctx.uv, ctx.w = batch, uv, w
        return dirty

    @staticmethod
    def backward(ctx, grad_out):
        g = api.degrid(ctx.batch, grad_out.contiguous().float(), ctx.uv, ctx.w, adjoint=True)
        return g, None, None, None


class PredictOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, batch, uv, w):
        vis = api.degrid(batch, model.contiguous(), uv, w, adjoint=False)
        ctx.batch, ctx.uv, ctx.w = batch, uv, w
        return vis

    @staticmethod
    def backward(ctx, grad_vis):
        img = api.predict_transpose(ctx.batch, grad_vis.contiguous().to(torch.complex64), ctx.uv, ctx.w)
        return img, None, None, None


def dirty(vis, batch, uv, w):
    """Differentiable dirty image of packed visibilities."""
    return ImagingOp.apply(vis, batch, uv, w)


def predict(model, batch, uv, w):
    """Differentiable model visibilities of packed model images."""
    return PredictOp.apply(model, batch, uv, w)
