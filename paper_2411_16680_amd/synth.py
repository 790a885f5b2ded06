"""Seeded synthetic inputs for the Update & Fuse step and the LDM composite.

This module only *draws* inputs: cameras, encoded feature pyramids, LDM state
(depth, alpha, features) and random-init weights, in the shapes and value
distributions of the paper's 1080p setting (Sec. 3.2, Tabs. of the network
appendix: 8 input views up to ~30 cm apart, C = 32 channels, d_k = 32).  It
holds none of the method's arithmetic: no projection, sampling, attention,
decode or composite.  Both the GPU path and the FP64 oracle receive exactly
the arrays produced here.

Conventions shared by every consumer of these arrays
-----------------------------------------------------
* Cameras: ``K`` is 3x3 row-major in pixel units of the camera's own
  ``(width, height)`` grid with half-pixel centres (pixel ``(x, y)`` has its
  centre at ``(x + 0.5, y + 0.5)``).  ``E`` is the 4x4 row-major
  world-to-camera transform with OpenCV axes (+x right, +y down, +z forward).
* Layouts are channel-last and layer-major: ``F[L][H][W][C]``,
  ``depth[L][H][W]``, ``alpha[L][H][W]``, feature map ``I[Hf][Wf][C]``.
  Layer 0 is the nearest layer.
* Values are drawn in float64 with NumPy's PCG64 and cast once, to float32,
  or to bfloat16 (round-to-nearest-even, stored as uint16 bit patterns) for
  the reduced-precision form.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "Camera", "Level", "Scene", "make_inputs", "make_custom", "f32_to_bf16_bits",
    "bf16_bits_to_f32", "CONFIG_NAMES",
]

CONFIG_NAMES = {
    1: "c1-tiny-64x48-V2",
    2: "c2-quarter1080p-480x270-V4-2step",
    3: "c3-multiscale-1080p-V8",
    4: "c4-backward-960x540-V4",
    5: "c5-serving-scene",
}


# ----------------------------------------------------------------------------
# bfloat16 storage helpers (a storage cast, not arithmetic of the method)
# ----------------------------------------------------------------------------

def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest-even); return uint16 bits."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    return ((u + rounding) >> 16).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


# ----------------------------------------------------------------------------
# Data containers
# ----------------------------------------------------------------------------

@dataclass
class Camera:
    K: np.ndarray          # (3, 3) float64
    E: np.ndarray          # (4, 4) float64, world -> camera
    width: int
    height: int


@dataclass
class Level:
    """One LDM level: its state, the matching feature maps and its weights."""
    L: int
    H: int
    W: int
    C: int                 # LDM feature channels
    Cf: int                # input feature channels
    heads: int
    head_dim: int
    feats: List[np.ndarray]            # V arrays [Hf][Wf][Cf] (float32 or bf16 bits)
    depth: np.ndarray                  # [L][H][W] float32
    alpha: np.ndarray                  # [L][H][W] float32
    F: np.ndarray                      # [L][H][W][C] float32 or bf16 bits
    weights: Dict[str, np.ndarray]     # float32 masters
    composite: bool = True             # render this level to RGB

    @property
    def N(self) -> int:
        return self.L * self.H * self.W


@dataclass
class Scene:
    config: int
    name: str
    seed: int
    dtype: str                         # "f32" or "bf16"
    in_cams: List[Camera]
    novel: Camera
    near: float
    far: float
    levels: List[Level]
    steps: int = 1
    target: Optional[np.ndarray] = None   # [H][W][3] float32 (loss target)
    depth_mode: str = "iid"
    extra: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return len(self.in_cams)


# ----------------------------------------------------------------------------
# Camera rigs
# ----------------------------------------------------------------------------

def _intrinsics(f: float, cx: float, cy: float) -> np.ndarray:
    return np.array([[f, 0.0, cx], [0.0, f, cy], [0.0, 0.0, 1.0]], dtype=np.float64)


def _fov_intrinsics(width: int, height: int, hfov_deg: float) -> np.ndarray:
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return _intrinsics(f, width / 2.0, height / 2.0)


def _extrinsic(R_wc: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """World-to-camera 4x4 from the camera's rotation (rows = camera axes in
    world coordinates) and its centre in world coordinates."""
    E = np.eye(4, dtype=np.float64)
    E[:3, :3] = R_wc
    E[:3, 3] = -R_wc @ centre
    return E


def _look_at_yaw(centre: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Rotation whose +z axis points from ``centre`` to ``target`` (in the
    x-z plane), +y pointing down (world +y)."""
    fwd = target - centre
    fwd = fwd / np.linalg.norm(fwd)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, fwd)
    right = right / np.linalg.norm(right)
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd], axis=0)


def _arc_rig(rng, V: int, arc_len: float, radius: float, width: int, height: int,
             hfov: float, novel_radius_jitter: float = 0.0):
    """V cameras evenly spaced on an arc of length ``arc_len`` of a circle of
    ``radius`` around a scene centre ``radius`` ahead of the origin, all
    looking at the centre.  The novel camera sits at a uniform angle inside
    the arc's span (radius optionally jittered)."""
    K = _fov_intrinsics(width, height, hfov)
    scene_c = np.array([0.0, 0.0, radius])
    span = arc_len / radius
    # draw order: novel angle, then novel radius
    theta_n = rng.uniform(-span / 2, span / 2)
    r_n = radius + (rng.uniform(-novel_radius_jitter, novel_radius_jitter)
                    if novel_radius_jitter > 0 else 0.0)

    def cam_at(theta, r):
        c = scene_c + r * np.array([math.sin(theta), 0.0, -math.cos(theta)])
        return Camera(K.copy(), _extrinsic(_look_at_yaw(c, scene_c), c), width, height)

    cams = []
    for i in range(V):
        th = -span / 2 + span * (i / (V - 1) if V > 1 else 0.5)
        cams.append(cam_at(th, radius))
    return cams, cam_at(theta_n, r_n)


# ----------------------------------------------------------------------------
# Draw helpers
# ----------------------------------------------------------------------------

def _normal(rng, shape, std=1.0):
    return (rng.standard_normal(size=shape, dtype=np.float64) * std).astype(np.float32)


def _cast(a32: np.ndarray, dtype: str) -> np.ndarray:
    return f32_to_bf16_bits(a32) if dtype == "bf16" else a32


def _sorted_depths(rng, L, H, W, lo, hi, dist: str, mode: str) -> np.ndarray:
    if mode == "smooth":
        # log-uniform marginal pushed through a 16-px-block bilinear field
        gh, gw = H // 16 + 2, W // 16 + 2
        g = rng.uniform(0.0, 1.0, size=(L, gh, gw))
        ys = (np.arange(H) + 0.5) / 16.0
        xs = (np.arange(W) + 0.5) / 16.0
        y0 = np.floor(ys).astype(int); x0 = np.floor(xs).astype(int)
        fy = (ys - y0)[None, :, None]; fx = (xs - x0)[None, None, :]
        u = (g[:, y0][:, :, x0] * (1 - fy) * (1 - fx) + g[:, y0 + 1][:, :, x0] * fy * (1 - fx)
             + g[:, y0][:, :, x0 + 1] * (1 - fy) * fx + g[:, y0 + 1][:, :, x0 + 1] * fy * fx)
    else:
        u = rng.uniform(0.0, 1.0, size=(L, H, W))
    if dist == "uniform":
        d = lo + (hi - lo) * u
    else:  # log-uniform
        d = np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * u)
    d.sort(axis=0)                     # layer 0 nearest
    return d.astype(np.float32)


def _smooth_image(rng, H: int, W: int, block: int) -> np.ndarray:
    """An RGBA8 image whose colours are a bilinear field over uniform
    random bytes on a ``block``-pixel grid (alpha 255): piecewise smooth, as
    photographs are, rather than i.i.d. per pixel."""
    gh, gw = H // block + 2, W // block + 2
    g = rng.uniform(0.0, 255.0, size=(gh, gw, 3))
    ys = (np.arange(H) + 0.5) / block
    xs = (np.arange(W) + 0.5) / block
    y0 = np.floor(ys).astype(int); x0 = np.floor(xs).astype(int)
    fy = (ys - y0)[:, None, None]; fx = (xs - x0)[None, :, None]
    v = (g[y0][:, x0] * (1 - fy) * (1 - fx) + g[y0 + 1][:, x0] * fy * (1 - fx)
         + g[y0][:, x0 + 1] * (1 - fy) * fx + g[y0 + 1][:, x0 + 1] * fy * fx)
    im = np.empty((H, W, 4), dtype=np.uint8)
    im[..., :3] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    im[..., 3] = 255
    return im


def _alpha(rng, shape, dist: str) -> np.ndarray:
    if dist == "uniform":
        a = rng.uniform(0.0, 1.0, size=shape)
    else:
        a = rng.beta(0.5, 0.5, size=shape)
    return a.astype(np.float32)


def _weights(rng, C: int, Cf: int, heads: int, head_dim: int) -> Dict[str, np.ndarray]:
    hd = heads * head_dim
    w = {}
    w["Wq"] = _normal(rng, (C, hd), 1.0 / math.sqrt(C))
    w["Wk"] = _normal(rng, (Cf, hd), 1.0 / math.sqrt(Cf))
    w["Wv"] = _normal(rng, (Cf, hd), 1.0 / math.sqrt(Cf))
    w["Wo"] = _normal(rng, (hd, C), 1.0 / math.sqrt(hd))
    w["w_sigma"] = _normal(rng, (C,), 1.0 / math.sqrt(C))
    w["w_depth"] = _normal(rng, (C,), 1.0 / math.sqrt(C))
    w["W_color"] = _normal(rng, (C, 3), 1.0 / math.sqrt(C))
    return w


# ----------------------------------------------------------------------------
# Configurations
# ----------------------------------------------------------------------------

def make_inputs(config: int, dtype: str = "f32", seed: Optional[int] = None,
                depth_mode: str = "iid", c3_levels: Optional[List[int]] = None) -> Scene:
    """Draw the inputs of workload ``config`` (1..4).

    1: V=2, 64x48, C=16, L=4, d=16, one step + composite.
    2: V=4, 480x270, C=32, L=16, d=32, two steps + composite.
    3: V=8, four levels (k=8,4,2,1) of a 1920x1080 frame, C=64/32/16/8,
       L=32/16/8/4, one step per level, composite of the finest level.
    4: V=4, 960x540, C=16, L=8, d=16, one step + composite, with a target.
    ``c3_levels`` optionally restricts config 3 to a subset of its levels
    (indices 0..3); the draws of the omitted levels are still consumed so the
    remaining arrays are identical to the full draw.
    """
    if dtype not in ("f32", "bf16"):
        raise ValueError("dtype must be 'f32' or 'bf16'")
    seed = 1000 + config if seed is None else seed
    rng = np.random.default_rng(seed)

    if config == 1:
        W, H, C, L, V = 64, 48, 16, 4, 2
        K = _intrinsics(60.0, 32.0, 24.0)
        eye = np.eye(3)
        in_cams = [Camera(K.copy(), _extrinsic(eye, np.array([0.0, 0, 0])), W, H),
                   Camera(K.copy(), _extrinsic(eye, np.array([0.1, 0, 0])), W, H)]
        novel = Camera(K.copy(), _extrinsic(eye, np.array([0.05, 0, 0])), W, H)
        feats = [_cast(_normal(rng, (H, W, C)), dtype) for _ in range(V)]
        depth = _sorted_depths(rng, L, H, W, 1.0, 10.0, "uniform", depth_mode)
        alpha = _alpha(rng, (L, H, W), "uniform")
        F = _cast(_normal(rng, (L, H, W, C)), dtype)
        wts = _weights(rng, C, C, 1, 16)
        lvl = Level(L, H, W, C, C, 1, 16, feats, depth, alpha, F, wts, True)
        return Scene(1, CONFIG_NAMES[1], seed, dtype, in_cams, novel, 1.0, 10.0, [lvl],
                     steps=1, depth_mode=depth_mode)

    if config in (2, 4):
        if config == 2:
            W, H, C, L, V, steps = 480, 270, 32, 16, 4, 2
        else:
            W, H, C, L, V, steps = 960, 540, 16, 8, 4, 1
        in_cams, novel = _arc_rig(rng, V, 0.3, 2.0, W, H, 60.0)
        feats = [_cast(_normal(rng, (H, W, C)), dtype) for _ in range(V)]
        depth = _sorted_depths(rng, L, H, W, 0.5, 20.0, "log", depth_mode)
        alpha = _alpha(rng, (L, H, W), "beta")
        F = _cast(_normal(rng, (L, H, W, C)), dtype)
        wts = _weights(rng, C, C, 1, C)
        lvl = Level(L, H, W, C, C, 1, C, feats, depth, alpha, F, wts, True)
        target = None
        if config == 4:
            target = rng.uniform(0.0, 1.0, size=(H, W, 3)).astype(np.float32)
        return Scene(config, CONFIG_NAMES[config], seed, dtype, in_cams, novel, 0.5, 20.0,
                     [lvl], steps=steps, target=target, depth_mode=depth_mode)

    if config == 3:
        FW, FH, V = 1920, 1080, 8
        ks = [8, 4, 2, 1]
        Cs = [64, 32, 16, 8]
        Ls = [32, 16, 8, 4]
        keep = set(range(4)) if c3_levels is None else set(c3_levels)
        in_cams, novel = _arc_rig(rng, V, 0.5, 1.5, FW, FH, 60.0, novel_radius_jitter=0.05)
        feats = [[None] * 4 for _ in range(V)]
        for m in range(V):                      # view-major, then level
            for li, (k, C) in enumerate(zip(ks, Cs)):
                shape = (FH // k, FW // k, C)
                if li in keep:
                    feats[m][li] = _cast(_normal(rng, shape), dtype)
                else:
                    rng.standard_normal(size=shape, dtype=np.float64)
        depths, alphas, Fs = [], [], []
        for li, (k, L) in enumerate(zip(ks, Ls)):
            depths.append(_sorted_depths(rng, L, FH // k, FW // k, 0.5, 20.0, "log", depth_mode))
        for li, (k, L) in enumerate(zip(ks, Ls)):
            alphas.append(_alpha(rng, (L, FH // k, FW // k), "beta"))
        for li, (k, L, C) in enumerate(zip(ks, Ls, Cs)):
            shape = (L, FH // k, FW // k, C)
            if li in keep:
                Fs.append(_cast(_normal(rng, shape), dtype))
            else:
                rng.standard_normal(size=shape, dtype=np.float64)
                Fs.append(None)
        levels = []
        for li, (k, L, C) in enumerate(zip(ks, Ls, Cs)):
            wts = _weights(rng, C, C, 1, C)
            if li in keep:
                levels.append(Level(L, FH // k, FW // k, C, C, 1, C,
                                    [feats[m][li] for m in range(V)], depths[li], alphas[li],
                                    Fs[li], wts, composite=(li == 3)))
        sc = Scene(3, CONFIG_NAMES[3], seed, dtype, in_cams, novel, 0.5, 20.0, levels,
                   steps=1, depth_mode=depth_mode)
        sc.extra["level_ids"] = sorted(keep)
        return sc

    raise ValueError(f"unknown config {config}")


def make_custom(*, V: int, H: int, W: int, C: int, L: int, heads: int = 1,
                head_dim: Optional[int] = None, Cf: Optional[int] = None,
                feat_hw: Optional[tuple] = None, dtype: str = "f32", seed: int = 7,
                steps: int = 1, near: float = 0.5, far: float = 20.0,
                arc: float = 0.3, radius: float = 2.0, hfov: float = 60.0,
                alpha_dist: str = "beta", composite: bool = True,
                with_target: bool = False) -> Scene:
    """A small arc-rig scene of arbitrary shape, for edge-case and ragged-tile
    tests.  Feature maps may have their own grid (``feat_hw``); the input
    cameras are given on the LDM's grid and rescaled by consumers."""
    head_dim = C if head_dim is None else head_dim
    Cf = C if Cf is None else Cf
    Hf, Wf = (H, W) if feat_hw is None else feat_hw
    rng = np.random.default_rng(seed)
    in_cams, novel = _arc_rig(rng, V, arc, radius, W, H, hfov)
    feats = [_cast(_normal(rng, (Hf, Wf, Cf)), dtype) for _ in range(V)]
    depth = _sorted_depths(rng, L, H, W, near, far, "log", "iid")
    alpha = _alpha(rng, (L, H, W), alpha_dist)
    F = _cast(_normal(rng, (L, H, W, C)), dtype)
    wts = _weights(rng, C, Cf, heads, head_dim)
    lvl = Level(L, H, W, C, Cf, heads, head_dim, feats, depth, alpha, F, wts, composite)
    target = rng.uniform(0.0, 1.0, size=(H, W, 3)).astype(np.float32) if with_target else None
    return Scene(0, f"custom-V{V}-{W}x{H}-L{L}-C{C}", seed, dtype, in_cams, novel, near, far,
                 [lvl], steps=steps, target=target)


# ----------------------------------------------------------------------------
# Final render workload: unactivated LDM attributes at a reduced grid plus
# the full-resolution input images
# ----------------------------------------------------------------------------

@dataclass
class RenderScene:
    in_cams: List[Camera]
    images: List[np.ndarray]           # V arrays [Hi][Wi][4] uint8 (RGBA8, alpha 255)
    novel: Camera
    near: float
    far: float
    depth_logit: np.ndarray            # [L][h][w] float32
    sigma_logit: np.ndarray            # [L][h][w] float32
    blend_logit: np.ndarray            # [L][h][w][V] float32
    H: int                             # output grid
    W: int

    @property
    def V(self) -> int:
        return len(self.in_cams)

    @property
    def logits(self):
        return self.depth_logit, self.sigma_logit, self.blend_logit


def make_render(*, V: int = 8, W: int = 1920, H: int = 1080, s: int = 2, L: int = 4,
                lowres_hw: Optional[tuple] = None, img_hw: Optional[tuple] = None,
                seed: int = 1006, arc: float = 0.5, radius: float = 1.5, hfov: float = 60.0,
                near: float = 0.5, far: float = 20.0, sigma_std: float = 1.5) -> RenderScene:
    """The final render's inputs: V RGBA8 input images (uniform random
    bytes, alpha 255) of ``img_hw`` (default the output grid) on an arc rig
    (the multi-scale workload's rig by default: 0.5 m arc of a 1.5 m ring, 60
    degree field of view, novel camera jittered 5 cm in radius), and the
    final LDM's logits on a grid ``s`` times coarser than the output (or
    ``lowres_hw``): depth and blend logits N(0, 1), density logits
    N(0, sigma_std).  Draw order: cameras, images (view-major), depth,
    density, blend logits."""
    rng = np.random.default_rng(seed)
    Hi, Wi = (H, W) if img_hw is None else img_hw
    h, w = (H // s, W // s) if lowres_hw is None else lowres_hw
    in_cams, novel = _arc_rig(rng, V, arc, radius, Wi, Hi, hfov, novel_radius_jitter=0.05)
    images = []
    for _ in range(V):
        im = rng.integers(0, 256, size=(Hi, Wi, 4), dtype=np.uint8)
        im[..., 3] = 255
        images.append(im)
    dlog = _normal(rng, (L, h, w))
    slog = _normal(rng, (L, h, w), std=sigma_std)
    blog = _normal(rng, (L, h, w, V))
    return RenderScene(in_cams, images, novel, near, far, dlog, slog, blog, H, W)


# ----------------------------------------------------------------------------
# Render-to-input-views workload: a decoded intermediate LDM and the views
# it is projected into
# ----------------------------------------------------------------------------

@dataclass
class ViewsScene:
    in_cams: List[Camera]
    novel: Camera
    near: float
    far: float
    depth: np.ndarray                  # [L][H][W] float32, sorted near to far per pixel
    alpha: np.ndarray                  # [L][H][W] float32
    color: np.ndarray                  # [L][H][W][3] float32 in [0, 1]
    view_hw: List[tuple]               # per view (Hm, Wm): the grid it is rendered on

    @property
    def V(self) -> int:
        return len(self.in_cams)


def make_views(*, V: int = 8, W: int = 1920, H: int = 1080, L: int = 4,
               view_hw: Optional[tuple] = None, seed: int = 1007, arc: float = 0.5,
               radius: float = 1.5, hfov: float = 60.0, near: float = 0.5, far: float = 20.0,
               depth_mode: str = "iid") -> ViewsScene:
    """An intermediate LDM to render into the input views: the multi-scale
    workload's rig by default (V = 8, 60 degree field of view, 0.5 m arc of a
    1.5 m ring, novel radius jittered 5 cm), depths log-uniform in
    [near, far] sorted per pixel (i.i.d. or smooth), alpha Beta(1/2, 1/2),
    colours uniform in [0, 1]; every view rendered on ``view_hw`` (default
    the LDM grid).  Draw order: cameras, depth, alpha, colour."""
    rng = np.random.default_rng(seed)
    in_cams, novel = _arc_rig(rng, V, arc, radius, W, H, hfov, novel_radius_jitter=0.05)
    depth = _sorted_depths(rng, L, H, W, near, far, "log", depth_mode)
    alpha = _alpha(rng, (L, H, W), "beta")
    color = rng.uniform(0.0, 1.0, size=(L, H, W, 3)).astype(np.float32)
    vhw = [(H, W) if view_hw is None else tuple(view_hw)] * V
    return ViewsScene(in_cams, novel, near, far, depth, alpha, color, vhw)


# ----------------------------------------------------------------------------
# Residual CNN block workload: a feature volume and two 3x3 kernels
# ----------------------------------------------------------------------------

def make_conv_block(*, L: int = 16, H: int = 270, W: int = 480, C: int = 32, seed: int = 1008,
                    dtype: str = "bf16"):
    """A feature volume [L][H][W][C] N(0, 1) (bfloat16 bits or float32) and
    two kernels [3][3][C][C] N(0, 1/sqrt(9 C)) (std = 1/sqrt(fan_in)).
    Returns (F, W1, W2).  Draw order: F, W1, W2."""
    rng = np.random.default_rng(seed)
    F = _cast(_normal(rng, (L, H, W, C)), dtype)
    std = 1.0 / math.sqrt(9.0 * C)
    W1 = _normal(rng, (3, 3, C, C), std)
    W2 = _normal(rng, (3, 3, C, C), std)
    return F, W1, W2


def make_collapse(*, L: int = 16, H: int = 270, W: int = 480, C: int = 32, seed: int = 1009,
                  dtype: str = "bf16"):
    """A feature volume [L][H][W][C] N(0, 1) and the layer collapse's MLP
    weights W1 [2C][C] N(0, 1/sqrt(2C)), W2 [C][C] N(0, 1/sqrt(C)).  Returns
    (F, W1, W2).  Draw order: F, W1, W2."""
    rng = np.random.default_rng(seed)
    F = _cast(_normal(rng, (L, H, W, C)), dtype)
    W1 = _normal(rng, (2 * C, C), 1.0 / math.sqrt(2 * C))
    W2 = _normal(rng, (C, C), 1.0 / math.sqrt(C))
    return F, W1, W2


# ----------------------------------------------------------------------------
# Ray-direction encoding workload: an input rig, a novel camera and the
# projection weights of every pyramid level (the feature maps themselves are
# drawn by the caller, on the host or the device)
# ----------------------------------------------------------------------------

RAY_LEVELS = ((8, 64), (4, 32), (2, 16), (1, 8))   # (k, C): grid (H/k, W/k)


@dataclass
class RayScene:
    in_cams: List[Camera]          # on the (W, H) input grid
    novel: Camera
    near: float
    far: float
    feat_hw: List[tuple]           # per level (Hf, Wf)
    Wr: List[np.ndarray]           # per level [32][C] float32


def make_ray(*, V: int = 8, W: int = 1920, H: int = 1080, levels=RAY_LEVELS, arc: float = 0.5,
             radius: float = 1.5, hfov: float = 60.0, near: float = 0.5, far: float = 20.0,
             seed: int = 1010) -> RayScene:
    """V cameras on an arc facing a centre (the 1080p, V = 8 rig by default),
    a novel camera inside the arc, and per level a projection Wr [32][C]
    N(0, 1/sqrt(32)).  Draw order: cameras, then Wr level by level."""
    rng = np.random.default_rng(seed)
    in_cams, novel = _arc_rig(rng, V, arc, radius, W, H, hfov, novel_radius_jitter=0.05)
    Wr = [_normal(rng, (32, C), 1.0 / math.sqrt(32.0)) for _, C in levels]
    return RayScene(in_cams, novel, near, far, [(H // k, W // k) for k, _ in levels], Wr)


# ----------------------------------------------------------------------------
# Chained multi-scale updates: the Update & Fuse steps of the paper's network
# table (LDM grid, layers, heads, transitions), random weights
# ----------------------------------------------------------------------------

@dataclass
class ChainStep:
    L: int
    H: int
    W: int
    level: int                     # pyramid level of its feature maps
    heads: int
    collapse: bool                 # halve the layers first (layer collapse)
    upsample: bool                 # then double the grid (2x upsampling)
    conv: bool = False             # a residual CNN block after the attention


# Quark's five Update & Fuse steps (appendix table, 1080p inputs): LDM grid
# and layers after each step's transition, image-feature level (36x60,
# 72x120, 144x240, 288x480), attention heads, one residual CNN block after
# the attention
QUARK_STEPS = (ChainStep(24, 36, 64, 0, 4, False, False, True),
               ChainStep(24, 72, 128, 1, 4, False, True, True),
               ChainStep(24, 72, 128, 1, 4, False, False, True),
               ChainStep(12, 144, 256, 2, 2, True, True, True),
               ChainStep(6, 288, 512, 3, 1, True, True, True))
QUARK_FEAT_HW = ((36, 60), (72, 120), (144, 240), (288, 480))


@dataclass
class ChainScene:
    in_cams: List[Camera]
    novel: Camera
    near: float
    far: float
    C: int
    steps: List[ChainStep]
    feats: List[List[np.ndarray]]  # per pyramid level, V maps [Hf][Wf][C]
    F0: np.ndarray                 # the first step's encoded LDM [L][H][W][C]
    weights: List[Dict[str, np.ndarray]]          # per step (heads of C / heads)
    collapse_w: List[Optional[tuple]]             # per step: (W1, W2) or None
    conv_w: List[Optional[tuple]]                 # per step: (W1, W2) 3x3 kernels or None
    dtype: str = "bf16"

    @property
    def V(self) -> int:
        return len(self.in_cams)

    def level(self, i: int) -> "Level":
        """Step i as a Level (its state arrays are produced by the chain)."""
        st = self.steps[i]
        return Level(st.L, st.H, st.W, self.C, self.C, st.heads, self.C // st.heads,
                     self.feats[st.level], None, None, None, self.weights[i],
                     composite=(i == len(self.steps) - 1))


def make_chain(*, V: int = 8, steps=QUARK_STEPS, feat_hw=QUARK_FEAT_HW, C: int = 32,
               input_hw=(1080, 1920), arc: float = 0.5, radius: float = 1.5, hfov: float = 60.0,
               dtype: str = "bf16", seed: int = 1011) -> ChainScene:
    """The rig of the multi-scale workload, one feature map per view and
    pyramid level N(0, 1), the first step's LDM features N(0, 1), and per step
    the attention / decode weights (std 1/sqrt(fan_in)), where it halves the
    layers the collapse MLP, and where it has one the residual CNN block's
    kernels.  Draw order: cameras, features (level-major, then view), F0,
    then per step its weights, collapse and conv weights."""
    rng = np.random.default_rng(seed)
    FH, FW = input_hw
    in_cams, novel = _arc_rig(rng, V, arc, radius, FW, FH, hfov, novel_radius_jitter=0.05)
    feats = [[_cast(_normal(rng, (h, w, C)), dtype) for _ in range(V)] for h, w in feat_hw]
    s0 = steps[0]
    F0 = _cast(_normal(rng, (s0.L, s0.H, s0.W, C)), dtype)
    weights, cw, kw = [], [], []
    for st in steps:
        weights.append(_weights(rng, C, C, st.heads, C // st.heads))
        cw.append((_normal(rng, (2 * C, C), 1.0 / math.sqrt(2 * C)),
                   _normal(rng, (C, C), 1.0 / math.sqrt(C))) if st.collapse else None)
        kw.append((_normal(rng, (3, 3, C, C), 1.0 / math.sqrt(9.0 * C)),
                   _normal(rng, (3, 3, C, C), 1.0 / math.sqrt(9.0 * C))) if st.conv else None)
    return ChainScene(in_cams, novel, 0.5, 20.0, C, list(steps), feats, F0, weights, cw, kw, dtype)


@dataclass
class PipelineScene:
    """The whole frame: a chain (its F0 unused: the first step starts from the
    learned initialisation), the initial feature f0, one ray-encoding
    projection per pyramid level on a low-resolution grid, and the full
    resolution RGBA8 input images the final render blends."""
    chain: ChainScene
    f0: np.ndarray                 # [C] float32, the learned initial feature
    Wr: List[np.ndarray]           # per pyramid level [32][C] float32
    low_hw: tuple                  # grid on which the ray encoding is evaluated
    images: List[np.ndarray]       # V arrays [H][W][4] uint8 (RGBA8, alpha 255)
    out_hw: tuple                  # output (H, W) of the final render


def make_pipeline(*, V: int = 8, steps=QUARK_STEPS, feat_hw=QUARK_FEAT_HW, C: int = 32,
                  input_hw=(1080, 1920), low_hw: Optional[tuple] = None, dtype: str = "bf16",
                  seed: int = 1011, image_block: int = 16) -> PipelineScene:
    """``make_chain``'s draws (same seed), then from a second generator
    (seed + 7919): f0 N(0, 1), per level Wr N(0, 1/32), the V images at the
    input / output grid: piecewise smooth colour fields (bilinear over
    uniform bytes on an ``image_block``-pixel grid; 0: uniform bytes per
    pixel), alpha 255.  The ray encoding is evaluated on the coarsest
    pyramid grid unless ``low_hw`` is given."""
    ch = make_chain(V=V, steps=steps, feat_hw=feat_hw, C=C, input_hw=input_hw, dtype=dtype,
                    seed=seed)
    rng = np.random.default_rng(seed + 7919)
    f0 = _normal(rng, (C,))
    Wr = [_normal(rng, (32, C), 1.0 / math.sqrt(32.0)) for _ in feat_hw]
    H, W = input_hw
    images = []
    for _ in range(V):
        if image_block > 0:
            images.append(_smooth_image(rng, H, W, image_block))
        else:
            im = rng.integers(0, 256, size=(H, W, 4), dtype=np.uint8)
            im[..., 3] = 255
            images.append(im)
    return PipelineScene(ch, f0, Wr, tuple(low_hw or feat_hw[0]), images, (H, W))


def to_bf16(scene: Scene) -> Scene:
    """The same draws stored in bfloat16 (features and LDM features are
    rounded to nearest-even; everything else is unchanged)."""
    import copy
    if scene.dtype == "bf16":
        return scene
    sc = copy.copy(scene)
    sc.dtype = "bf16"
    sc.levels = []
    for lvl in scene.levels:
        l2 = copy.copy(lvl)
        l2.feats = [f32_to_bf16_bits(f) for f in lvl.feats]
        l2.F = f32_to_bf16_bits(lvl.F)
        sc.levels.append(l2)
    return sc


# ----------------------------------------------------------------------------
# Serving workload (many scenes, Poisson requests)
# ----------------------------------------------------------------------------

SERVE_OUTPUTS = ((640, 360), (1280, 720), (1920, 1080))


@dataclass
class ServeScene:
    scene_id: int
    in_cams: List[Camera]          # on the input image grid
    centre: np.ndarray             # the point every input camera looks at
    centroid: np.ndarray           # mean of the input camera centres
    feat_hw: List[tuple]           # per pyramid level (Hf, Wf)
    img_hw: tuple                  # the input images' grid (H, W)
    seed: int                      # seed of its pyramid and images

    @property
    def V(self) -> int:
        return len(self.in_cams)


@dataclass
class ServeRequest:
    rid: int
    scene_id: int
    width: int
    height: int
    novel: Camera                  # on the request's output grid
    arrival: float                 # seconds after the start


@dataclass
class ServeModel:
    """The network every request runs (shared by scenes): the chained steps,
    their weights, the layer-collapse and residual-block weights, the learned
    initial feature and the per-level ray-encoding projections."""
    steps: List[ChainStep]
    C: int
    weights: List[Dict[str, np.ndarray]]
    collapse_w: List[Optional[tuple]]
    conv_w: List[Optional[tuple]]
    f0: np.ndarray
    Wr: List[np.ndarray]
    low_hw: tuple
    near: float = 0.5
    far: float = 20.0


def make_serving(n_scenes: int = 16, n_requests: int = 2000, rate: float = 60.0,
                 seed: int = 5000, views=(4, 6, 8), outputs=SERVE_OUTPUTS,
                 input_hw=(1080, 1920), steps=QUARK_STEPS, feat_hw=QUARK_FEAT_HW, C: int = 32):
    """Scenes, the network and a Poisson request stream.  Each scene has V in
    ``views`` cameras evenly on a 0.5 m arc of a radius-1.5 m ring facing
    its centre (60 degree field of view), a feature pyramid of ``feat_hw``
    levels with C channels and V input images on ``input_hw`` (both drawn on
    the device from the scene's seed).  The network: per step attention and
    decode weights, collapse MLPs and residual-block kernels (std
    1/sqrt(fan_in)), f0 N(0, 1), per level Wr N(0, 1/32).  A request picks a
    scene and an output size uniformly; its novel camera sits uniformly in
    a 0.3 m ball around the scene's camera centroid, looking at the centre,
    60 degree field of view.  Arrivals are a Poisson process of ``rate`` per
    second."""
    rng = np.random.default_rng(seed)
    FH, FW = input_hw
    scenes = []
    for s in range(n_scenes):
        V = int(views[rng.integers(0, len(views))])
        cams, _ = _arc_rig(rng, V, 0.5, 1.5, FW, FH, 60.0)
        centres = np.stack([-c.E[:3, :3].T @ c.E[:3, 3] for c in cams])
        scenes.append(ServeScene(s, cams, np.array([0.0, 0.0, 1.5]), centres.mean(axis=0),
                                 [tuple(hw) for hw in feat_hw], tuple(input_hw), seed + 1 + s))
    weights, cw, kw = [], [], []
    for st in steps:
        weights.append(_weights(rng, C, C, st.heads, C // st.heads))
        cw.append((_normal(rng, (2 * C, C), 1.0 / math.sqrt(2 * C)),
                   _normal(rng, (C, C), 1.0 / math.sqrt(C))) if st.collapse else None)
        kw.append((_normal(rng, (3, 3, C, C), 1.0 / math.sqrt(9.0 * C)),
                   _normal(rng, (3, 3, C, C), 1.0 / math.sqrt(9.0 * C))) if st.conv else None)
    f0 = _normal(rng, (C,))
    Wr = [_normal(rng, (32, C), 1.0 / math.sqrt(32.0)) for _ in feat_hw]
    model = ServeModel(list(steps), C, weights, cw, kw, f0, Wr, tuple(feat_hw[0]))
    reqs = []
    t = 0.0
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        sc = scenes[int(rng.integers(0, n_scenes))]
        W, H = outputs[int(rng.integers(0, len(outputs)))]
        while True:                                   # uniform in the ball
            off = rng.uniform(-0.3, 0.3, size=3)
            if np.dot(off, off) <= 0.09:
                break
        c = sc.centroid + off
        K = _fov_intrinsics(W, H, 60.0)
        novel = Camera(K, _extrinsic(_look_at_yaw(c, sc.centre), c), W, H)
        reqs.append(ServeRequest(i, sc.scene_id, W, H, novel, t))
    return scenes, model, reqs


def device_pyramid(scene: ServeScene, C: int = 32, device="cuda", dtype: str = "bf16"):
    """The scene's feature pyramid, drawn on the device with a seeded torch
    generator: [level][view] tensors [Hf][Wf][C], standard normal."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(scene.seed))
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    return [[torch.randn((Hf, Wf, C), generator=g, device=device, dtype=torch.float32).to(tdt)
             for _ in range(scene.V)] for (Hf, Wf) in scene.feat_hw]


def device_images(scene: ServeScene, block: int = 16, device="cuda"):
    """The scene's V input images, RGBA8 [H][W][4] on the device: bilinear
    colour fields over uniform random bytes on a ``block``-pixel grid (a
    seeded torch generator of its own), alpha 255."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(scene.seed) + 104729)
    H, W = scene.img_hw
    gh, gw = H // block + 2, W // block + 2
    out = []
    for _ in range(scene.V):
        grid = torch.rand((1, 3, gh, gw), generator=g, device=device) * 255.0
        up = torch.nn.functional.interpolate(grid, scale_factor=block, mode="bilinear",
                                             align_corners=False)[0, :, :H, :W]
        im = torch.empty((H, W, 4), dtype=torch.uint8, device=device)
        im[..., :3] = up.permute(1, 2, 0).round().clamp(0, 255).to(torch.uint8)
        im[..., 3] = 255
        out.append(im)
    return out
