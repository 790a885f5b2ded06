"""Scene-level driver on the GPU: moves a ``synth.Scene`` into device
tensors and runs its levels through libquark.  Marshalling only -- every
step of the method runs in the library's kernels."""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import lib


def _to_dev(a: np.ndarray, device):
    import torch
    if a.dtype == np.uint16:          # bfloat16 bit patterns
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).to(device).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


@dataclass
class DeviceLevel:
    L: int
    H: int
    W: int
    C: int
    feats: List
    F: object
    depth: object
    alpha: object
    weights: Dict
    F_out: object
    depth_out: object
    alpha_out: object
    rgb: Optional[object] = None
    acc: Optional[object] = None
    composite: bool = True
    heads: int = 1                     # attention heads (head width C / heads)
    extra: dict = field(default_factory=dict)


def level_to_device(level, device="cuda", composite: Optional[bool] = None) -> DeviceLevel:
    import torch
    comp = level.composite if composite is None else composite
    feats = [_to_dev(f, device) for f in level.feats]
    F = _to_dev(level.F, device)
    depth = _to_dev(level.depth, device)
    alpha = _to_dev(level.alpha, device)
    w = {k: _to_dev(np.ascontiguousarray(v, dtype=np.float32), device)
         for k, v in level.weights.items()}
    dl = DeviceLevel(level.L, level.H, level.W, level.C, feats, F, depth, alpha, w,
                     torch.empty_like(F), torch.empty_like(depth), torch.empty_like(alpha),
                     composite=comp, heads=int(getattr(level, "heads", 1)))
    if comp:
        dl.rgb = torch.empty((level.H, level.W, 3), dtype=torch.float32, device=device)
        dl.acc = torch.empty((level.H, level.W), dtype=torch.float32, device=device)
    return dl


def scene_to_device(scene, device="cuda") -> List[DeviceLevel]:
    return [level_to_device(l, device) for l in scene.levels]


def run_level(ctx: lib.Context, scene, dl: DeviceLevel, *, steps: Optional[int] = None,
              precision: Optional[str] = None, attn_form: str = "standard",
              mode: str = "residual", stream=None):
    """``steps`` Update & Fuse steps (the first reads the input state, later
    ones update the output state in place), compositing on the last step
    when the level composites."""
    steps = scene.steps if steps is None else steps
    precision = precision or ("bf16" if scene.dtype == "bf16" else "fp32")
    wts = dl.extra.get("qk_weights")
    if wts is None:                    # built once (the tensors stay in dl.weights)
        wts = dl.extra["qk_weights"] = lib.make_weights(dl.weights, heads=dl.heads)
    for s in range(steps):
        src = (dl.F, dl.depth, dl.alpha) if s == 0 else (dl.F_out, dl.depth_out, dl.alpha_out)
        last = s == steps - 1
        lib.update_fuse(ctx, scene.in_cams, dl.feats, scene.novel, scene.near, scene.far,
                        wts, src, (dl.F_out, dl.depth_out, dl.alpha_out),
                        precision=precision, attn_form=attn_form, mode=mode,
                        rgb_out=dl.rgb if (last and dl.composite) else None,
                        acc_out=dl.acc if (last and dl.composite) else None, stream=stream)


def run_scene(ctx: lib.Context, scene, dls: List[DeviceLevel], **kw):
    for dl in dls:
        run_level(ctx, scene, dl, **kw)


def level_outputs_numpy(dl: DeviceLevel) -> Dict[str, np.ndarray]:
    import torch
    torch.cuda.synchronize()
    out = {"F": dl.F_out.float().cpu().numpy().astype(np.float64),
           "depth": dl.depth_out.cpu().numpy().astype(np.float64),
           "alpha": dl.alpha_out.cpu().numpy().astype(np.float64)}
    if dl.rgb is not None:
        out["rgb"] = dl.rgb.cpu().numpy().astype(np.float64)
        out["acc"] = dl.acc.cpu().numpy().astype(np.float64)
    return out
