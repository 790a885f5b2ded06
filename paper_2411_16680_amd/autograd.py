"""torch.autograd wrapper of one float32 Update & Fuse step (+ composite).

The forward calls qk_update_fuse (QK_PREC_FP32) into fresh output tensors,
the backward calls qk_update_fuse_backward; both run in libquark's HIP
kernels.  Steps chain through torch's autograd like any other op, so a
multi-step solve is differentiated by calling ``update_fuse_step`` in a loop.
"""

from __future__ import annotations

from typing import Dict, Sequence

import torch

from . import lib

_WEIGHTS = lib.WEIGHT_NAMES


class _Meta:
    """Non-tensor arguments of a step (cameras, planes, mode, context)."""

    def __init__(self, qctx, in_cams, novel, near, far, mode, composite, attn_form, n_feats):
        self.qctx = qctx
        self.in_cams = list(in_cams)
        self.novel = novel
        self.near = float(near)
        self.far = float(far)
        self.mode = mode
        self.composite = composite
        self.attn_form = attn_form
        self.n_feats = n_feats


def _need(t: torch.Tensor, what: str) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_cuda:
        raise lib.QuarkError(lib.QK_EDTYPE, f"{what} must be a float32 device tensor")
    return t.contiguous()


class UpdateFuseFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, meta: _Meta, F, depth, alpha, *rest):
        weights = dict(zip(_WEIGHTS, rest[:len(_WEIGHTS)]))
        feats = list(rest[len(_WEIGHTS):])
        L, H, W = (int(s) for s in depth.shape)
        F_out = torch.empty_like(F)
        d_out = torch.empty_like(depth)
        a_out = torch.empty_like(alpha)
        rgb = torch.empty((H, W, 3), device=F.device, dtype=torch.float32) if meta.composite else None
        lib.update_fuse(meta.qctx, meta.in_cams, feats, meta.novel, meta.near, meta.far, weights,
                        (F, depth, alpha), (F_out, d_out, a_out), precision="fp32",
                        attn_form=meta.attn_form, mode=meta.mode, rgb_out=rgb)
        ctx.meta = meta
        ctx.save_for_backward(F, depth, alpha, F_out, a_out, *rest)
        ctx.set_materialize_grads(False)
        if meta.composite:
            return F_out, d_out, a_out, rgb
        return F_out, d_out, a_out

    @staticmethod
    def backward(ctx, dF_out, dd_out, da_out, d_rgb=None):
        meta: _Meta = ctx.meta
        saved = ctx.saved_tensors
        F, depth, alpha, F_out, a_out = saved[:5]
        rest = saved[5:]
        weights = dict(zip(_WEIGHTS, rest[:len(_WEIGHTS)]))
        feats = list(rest[len(_WEIGHTS):])
        dF = torch.empty_like(F)
        dd = torch.empty_like(depth)
        da = torch.empty_like(alpha)
        dfeats = [torch.empty_like(f) for f in feats]
        dW = {k: torch.empty_like(v) for k, v in weights.items()}
        cont = lambda t: None if t is None else t.contiguous()
        d_out = None
        if dF_out is not None or dd_out is not None or da_out is not None:
            d_out = (cont(dF_out), cont(dd_out), cont(da_out))
        lib.update_fuse_backward(meta.qctx, meta.in_cams, feats, meta.novel, meta.near, meta.far,
                                 weights, (F, depth, alpha), (F_out, None, a_out),
                                 (dF, dd, da), dfeats, dW, d_rgb=cont(d_rgb), d_out=d_out,
                                 mode=meta.mode)
        return (None, dF, dd, da, *[dW[k] for k in _WEIGHTS], *dfeats)


def update_fuse_step(qctx: lib.Context, in_cams: Sequence, feats: Sequence[torch.Tensor], novel,
                     near: float, far: float, weights: Dict[str, torch.Tensor], F: torch.Tensor,
                     depth: torch.Tensor, alpha: torch.Tensor, *, mode: str = "residual",
                     composite: bool = True, attn_form: str = "standard"):
    """One differentiable float32 Update & Fuse step.  Returns (F', depth',
    alpha', rgb) when ``composite`` else (F', depth', alpha').  Every tensor
    must be a contiguous float32 device tensor; gradients flow to F, depth,
    alpha, every feature map and every weight."""
    F = _need(F, "F")
    depth = _need(depth, "depth")
    alpha = _need(alpha, "alpha")
    feats = [_need(f, "feature map") for f in feats]
    w = [_need(weights[k], k) for k in _WEIGHTS]
    meta = _Meta(qctx, in_cams, novel, near, far, mode, composite, attn_form, len(feats))
    return UpdateFuseFunction.apply(meta, F, depth, alpha, *w, *feats)
