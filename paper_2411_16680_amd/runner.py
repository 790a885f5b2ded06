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
              mode: str = "residual", stream=None, composite: Optional[bool] = None,
              from_output: bool = False):
    """``steps`` Update & Fuse steps (the first reads the input state, or the
    output state when ``from_output``; later ones update the output state in
    place), compositing on the last step when ``composite`` (default: when
    the level composites)."""
    steps = scene.steps if steps is None else steps
    composite = dl.composite if composite is None else composite
    precision = precision or ("bf16" if scene.dtype == "bf16" else "fp32")
    attn_form = step_form(attn_form, dl)
    wts = dl.extra.get("qk_weights")
    if wts is None:                    # built once (the tensors stay in dl.weights)
        wts = dl.extra["qk_weights"] = lib.make_weights(dl.weights, heads=dl.heads)
    for s in range(steps):
        first_in = s == 0 and not from_output
        src = (dl.F, dl.depth, dl.alpha) if first_in else (dl.F_out, dl.depth_out, dl.alpha_out)
        last = s == steps - 1
        lib.update_fuse(ctx, scene.in_cams, dl.feats, scene.novel, scene.near, scene.far,
                        wts, src, (dl.F_out, dl.depth_out, dl.alpha_out),
                        precision=precision, attn_form=attn_form, mode=mode,
                        rgb_out=dl.rgb if (last and composite) else None,
                        acc_out=dl.acc if (last and composite) else None, stream=stream)


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


# ---------------------------------------------------------------------------
# Chained multi-scale updates (the paper's iterative Update & Fuse schedule)
# ---------------------------------------------------------------------------

@dataclass
class DeviceChain:
    feats: List[List]                  # per pyramid level, V device maps
    F0: object
    weights: List[Dict]                # per step, device tensors
    qkw: List[object]                  # per step, qk_weights
    collapse_w: List[Optional[tuple]]
    conv_w: List[Optional[tuple]]
    F_in: List[Optional[object]]       # per step: upsampled / collapsed input (or None)
    F_conv: List[Optional[object]]     # per step: after the residual CNN block (or None)
    tmp: List[Optional[object]]        # per step: collapsed, before upsampling
    depth: List[object]
    alpha: List[object]
    F_out: List[object]
    depth_out: List[object]
    alpha_out: List[object]
    rgb: object
    color: Optional[object] = None     # last step with a CNN block: decoded colour
    acc: Optional[object] = None


def chain_tensors(ch, device="cuda"):
    """A chain scene's data on the device: the pyramid [level][view], the
    per-step weight dicts, and the collapse and conv weight pairs."""
    feats = [[_to_dev(f, device) for f in lvl] for lvl in ch.feats]
    ws = [{k: _to_dev(np.ascontiguousarray(v, dtype=np.float32), device) for k, v in w.items()}
          for w in ch.weights]
    cw = [None if c is None else tuple(_to_dev(np.ascontiguousarray(a, dtype=np.float32), device)
                                       for a in c) for c in ch.collapse_w]
    kw = [None if c is None else tuple(_to_dev(np.ascontiguousarray(a, dtype=np.float32), device)
                                       for a in c) for c in ch.conv_w]
    return feats, ws, cw, kw


def chain_to_device(ch, device="cuda") -> DeviceChain:
    import torch
    feats, ws, cw, kw = chain_tensors(ch, device)
    qkw = [lib.make_weights(w, heads=st.heads) for w, st in zip(ws, ch.steps)]
    last = ch.steps[-1]
    chain_kw, _ = frame_buffers(ch.steps, ch.C, ch.V, (last.H, last.W), ch.dtype, device)
    chain_kw["F0"].copy_(_to_dev(ch.F0, device))
    color = (torch.empty((last.L, last.H, last.W, 3), dtype=torch.float32, device=device)
             if last.conv else None)
    return DeviceChain(feats=feats, weights=ws, qkw=qkw, collapse_w=cw, conv_w=kw, color=color,
                       **chain_kw)


def step_form(attn_form: str, step) -> str:
    """The attention form a step runs in: ``attn_form`` itself, or for
    "auto" the one-to-many form on a step with one head and the standard
    form on a step with several (the faster of the two on MI355X at the
    paper's head counts; both compute the same attention)."""
    if attn_form != "auto":
        return attn_form
    return "folded" if int(step.heads) == 1 else "standard"


def run_chain(ctx: lib.Context, ch, dc: DeviceChain, attn_form: str = "standard", stream=None):
    """The steps in order.  Step i > 0 takes step i - 1's output features,
    collapses their layers (qk_layer_collapse) and / or doubles their grid
    (qk_upsample2x) as its transition asks; every step decodes its input
    features into depth and alpha (qk_ldm_decode), runs Update & Fuse with
    the absolute decode (qk_update_fuse) and, if it has one, its residual CNN
    block (qk_residual_conv).  The last step composites its output: inside
    Update & Fuse, or after its CNN block by decoding the block's output
    (qk_ldm_decode) and compositing it (qk_composite)."""
    prec = "bf16" if ch.dtype == "bf16" else "fp32"
    F = dc.F0
    n = len(ch.steps)
    for i, st in enumerate(ch.steps):
        if i > 0:
            prev = ch.steps[i - 1]
            F = dc.F_conv[i - 1] if prev.conv else dc.F_out[i - 1]
            if st.collapse:
                W1, W2 = dc.collapse_w[i]
                lib.layer_collapse(ctx, F, W1, W2, dc.tmp[i], stream=stream)
                F = dc.tmp[i]
            if st.upsample:
                lib.upsample2x(ctx, F, dc.F_in[i], stream=stream)
                F = dc.F_in[i]
        w = dc.weights[i]
        lib.ldm_decode(ctx, F, dc.depth[i], dc.alpha[i], w["w_sigma"], w["w_depth"], w["W_color"],
                       ch.near, ch.far, stream=stream)
        comp = i == n - 1 and not st.conv
        lib.update_fuse(ctx, ch.in_cams, dc.feats[st.level], ch.novel, ch.near, ch.far, dc.qkw[i],
                        (F, dc.depth[i], dc.alpha[i]),
                        (dc.F_out[i], dc.depth_out[i], dc.alpha_out[i]),
                        precision=prec, attn_form=step_form(attn_form, st), mode="paper",
                        rgb_out=dc.rgb if comp else None, acc_out=dc.acc if comp else None,
                        stream=stream)
        if st.conv:
            K1, K2 = dc.conv_w[i]
            lib.residual_conv(ctx, dc.F_out[i], K1, K2, dc.F_conv[i], stream=stream)
            if i == n - 1:
                # the output LDM: decode of the block's output, then composite
                lib.ldm_decode(ctx, dc.F_conv[i], dc.depth_out[i], dc.alpha_out[i], w["w_sigma"],
                               w["w_depth"], w["W_color"], ch.near, ch.far, color_out=dc.color,
                               stream=stream)
                lib.composite(ctx, dc.color, dc.alpha_out[i], dc.rgb, dc.acc, stream=stream)


# ---------------------------------------------------------------------------
# The whole frame: ray-encoded pyramid, learned initialisation, the chained
# steps, and the final render of the last step's LDM (Eq. 1)
# ---------------------------------------------------------------------------

@dataclass
class DevicePipeline:
    chain: DeviceChain
    feats_raw: List[List]              # per level, the V maps as the encoder gave them
    feats: List[List]                  # per level, work copies that receive the encoding
    Wr: List[object]                   # per level [32][C] float32
    f0: object                         # [C] float32
    blend_logit: object                # [L][H][W][V] float32, the last step's
    depth_logit: object                # [L][H][W] float32, the final volume's
    sigma_logit: object
    images: List[object]               # V RGBA8 [H][W][4]
    rgb: object                        # [H][W][3] float32
    acc: object                        # [H][W]
    depth: object                      # [H][W]


def frame_buffers(steps, C: int, V: int, out_hw, dtype: str, device="cuda"):
    """One frame's own device buffers for the chained steps ``steps``: per
    step the transition outputs, the decoded input state, the update's
    output and the residual block's output (as in ``chain_to_device``), the
    first step's initial volume, the last step's blend-weight logits, the
    final volume's logits and the render's outputs on ``out_hw``.  Returns
    the keyword arguments of ``DeviceChain`` (without data or weights) and of
    ``DevicePipeline``'s per-frame fields."""
    import torch
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    f32 = dict(dtype=torch.float32, device=device)
    F_in, tmp, depth, alpha, F_out, d_out, a_out, F_conv = [], [], [], [], [], [], [], []
    prev = None
    for i, st in enumerate(steps):
        shp = (st.L, st.H, st.W)
        if i > 0:                      # the transition must produce this step's grid
            want = (prev[0] // 2 if st.collapse else prev[0],
                    2 * prev[1] if st.upsample else prev[1], 2 * prev[2] if st.upsample else prev[2])
            if shp != want or (st.collapse and prev[0] % 2):
                raise ValueError(f"step {i}: grid {shp} does not follow {prev} by its transition")
        tmp.append(torch.empty((st.L,) + prev[1:] + (C,), dtype=tdt, device=device)
                   if i > 0 and st.collapse else None)
        F_in.append(torch.empty(shp + (C,), dtype=tdt, device=device)
                    if i > 0 and st.upsample else None)
        depth.append(torch.empty(shp, **f32))
        alpha.append(torch.empty(shp, **f32))
        F_out.append(torch.empty(shp + (C,), dtype=tdt, device=device))
        F_conv.append(torch.empty(shp + (C,), dtype=tdt, device=device) if st.conv else None)
        d_out.append(torch.empty(shp, **f32))
        a_out.append(torch.empty(shp, **f32))
        prev = shp
    s0, last = steps[0], steps[-1]
    lshp = (last.L, last.H, last.W)
    H, W = out_hw
    chain = dict(F0=torch.empty((s0.L, s0.H, s0.W, C), dtype=tdt, device=device), F_in=F_in,
                 F_conv=F_conv, tmp=tmp, depth=depth, alpha=alpha, F_out=F_out, depth_out=d_out,
                 alpha_out=a_out, rgb=torch.empty((H, W, 3), **f32))
    frame = dict(blend_logit=torch.empty(lshp + (V,), **f32), depth_logit=torch.empty(lshp, **f32),
                 sigma_logit=torch.empty(lshp, **f32), rgb=chain["rgb"],
                 acc=torch.empty((H, W), **f32), depth=torch.empty((H, W), **f32))
    return chain, frame


def make_device_pipeline(steps, C: int, feats_raw, weights, collapse_w, conv_w, Wr, f0, images,
                         out_hw, dtype: str, device="cuda") -> DevicePipeline:
    """A frame's ``DevicePipeline``: its own buffers (``frame_buffers``) and
    work copies of the pyramid, around shared device tensors -- the scene's
    pyramid ``feats_raw`` [level][view] and ``images``, and the network's
    weights (per step dicts, collapse and conv pairs, per level Wr, f0)."""
    import torch
    V = len(feats_raw[0])
    chain_kw, frame_kw = frame_buffers(steps, C, V, out_hw, dtype, device)
    qkw = [lib.make_weights(w, heads=st.heads) for w, st in zip(weights, steps)]
    dc = DeviceChain(feats=feats_raw, weights=weights, qkw=qkw, collapse_w=collapse_w,
                     conv_w=conv_w, **chain_kw)
    feats = [[torch.empty_like(f) for f in lvl] for lvl in feats_raw]
    return DevicePipeline(dc, feats_raw, feats, Wr, f0, images=images, **frame_kw)


def pipeline_to_device(pl, device="cuda") -> DevicePipeline:
    ch = pl.chain
    feats, ws, cw, kw = chain_tensors(ch, device)
    Wr = [_to_dev(np.ascontiguousarray(w, dtype=np.float32), device) for w in pl.Wr]
    f0 = _to_dev(np.ascontiguousarray(pl.f0, dtype=np.float32), device)
    images = [_to_dev(im, device) for im in pl.images]
    return make_device_pipeline(ch.steps, ch.C, feats, ws, cw, kw, Wr, f0, images, pl.out_hw,
                                ch.dtype, device)


def run_pipeline(ctx: lib.Context, pl, dp: DevicePipeline, attn_form: str = "standard",
                 stream=None):
    """One frame (``run_pipelines`` of one)."""
    run_pipelines(ctx, [(pl.chain, pl.low_hw, dp)], attn_form=attn_form, stream=stream)


def run_pipelines(ctx: lib.Context, frames, attn_form: str = "standard", stream=None):
    """Whole frames, ``frames`` a list of (scene, low_hw, DevicePipeline)
    where the scene gives in_cams, novel, near, far, steps and dtype (a
    ``synth.ChainScene`` or the like).  Per frame: (1) each level's
    ray-direction encoding (qk_ray_encoding, evaluated on the
    low-resolution grid) is added to the encoder's maps, written to the
    frame's own pyramid (out of place: the encoder's maps stay as they are
    for the next frame); (2) the first
    step starts from the learned initialisation (qk_ldm_init: f0 broadcast,
    flat layers at the anchors); (3) every step: its transition from the
    previous step's output (qk_layer_collapse, qk_upsample2x) and the
    absolute decode of its input (qk_ldm_decode) after the first, Update &
    Fuse with the absolute decode (the last step also writes the
    blend-weight logits of its attention) and its residual CNN block
    (qk_residual_conv); (4) the final volume's unactivated depth and density
    (qk_ldm_decode_logits) and the final render at the output grid
    (qk_render_ibr).  With several bfloat16 frames each step's Update & Fuse
    of every frame is one qk_batch_update_fuse launch (the frames share the
    network, so C and the heads); otherwise one qk_update_fuse per frame."""
    steps = frames[0][0].steps
    prec = "bf16" if frames[0][0].dtype == "bf16" else "fp32"
    batched = len(frames) > 1 and prec == "bf16"
    for sc, low_hw, dp in frames:
        for k, lvl in enumerate(dp.feats):
            lib.ray_encoding(ctx, sc.in_cams, sc.novel, sc.near, sc.far, dp.Wr[k], lvl,
                             low_hw=low_hw, stream=stream, src=dp.feats_raw[k])
        dc = dp.chain
        lib.ldm_init(ctx, dp.f0, sc.near, sc.far, (dc.F0, dc.depth[0], dc.alpha[0]),
                     stream=stream)
    n = len(steps)
    for i, st in enumerate(steps):
        ins = []
        for sc, _, dp in frames:
            dc = dp.chain
            w = dc.weights[i]
            F = dc.F0
            if i > 0:
                prev = steps[i - 1]
                F = dc.F_conv[i - 1] if prev.conv else dc.F_out[i - 1]
                if st.collapse:
                    W1, W2 = dc.collapse_w[i]
                    lib.layer_collapse(ctx, F, W1, W2, dc.tmp[i], stream=stream)
                    F = dc.tmp[i]
                if st.upsample:
                    lib.upsample2x(ctx, F, dc.F_in[i], stream=stream)
                    F = dc.F_in[i]
                lib.ldm_decode(ctx, F, dc.depth[i], dc.alpha[i], w["w_sigma"], w["w_depth"],
                               w["W_color"], sc.near, sc.far, stream=stream)
            ins.append(F)
        blend = i == n - 1
        if batched:
            reqs = [lib.Request(sc.in_cams, dp.feats[st.level], sc.novel, sc.near, sc.far,
                                dp.chain.qkw[i], (F, dp.chain.depth[i], dp.chain.alpha[i]),
                                (dp.chain.F_out[i], dp.chain.depth_out[i], dp.chain.alpha_out[i]),
                                mode="paper", blend_logit_out=dp.blend_logit if blend else None)
                    for (sc, _, dp), F in zip(frames, ins)]
            lib.batch_update_fuse(ctx, reqs, precision=prec, attn_form=step_form(attn_form, st),
                                  stream=stream)
        else:
            for (sc, _, dp), F in zip(frames, ins):
                dc = dp.chain
                lib.update_fuse(ctx, sc.in_cams, dp.feats[st.level], sc.novel, sc.near, sc.far,
                                dc.qkw[i], (F, dc.depth[i], dc.alpha[i]),
                                (dc.F_out[i], dc.depth_out[i], dc.alpha_out[i]),
                                precision=prec, attn_form=step_form(attn_form, st), mode="paper",
                                blend_logit_out=dp.blend_logit if blend else None, stream=stream)
        if st.conv:
            for _, _, dp in frames:
                dc = dp.chain
                K1, K2 = dc.conv_w[i]
                lib.residual_conv(ctx, dc.F_out[i], K1, K2, dc.F_conv[i], stream=stream)
    last = steps[-1]
    for sc, _, dp in frames:
        dc = dp.chain
        Ff = dc.F_conv[-1] if last.conv else dc.F_out[-1]
        w = dc.weights[-1]
        lib.ldm_logits(ctx, Ff, w["w_sigma"], w["w_depth"], dp.depth_logit, dp.sigma_logit,
                       stream=stream)
        lib.render_ibr(ctx, sc.in_cams, dp.images, sc.novel, sc.near, sc.far,
                       (dp.depth_logit, dp.sigma_logit, dp.blend_logit), dp.rgb,
                       acc_out=dp.acc, depth_out=dp.depth, stream=stream)
