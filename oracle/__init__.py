"""FP64 CPU oracle for the Update & Fuse step and the LDM composite.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library.  The arithmetic lives
in ``quark_oracle.c`` (plain double-precision loops, one function per step of
the method); this module builds it with gcc, loads it with ctypes and
marshals NumPy arrays in and out.  It shares no code with the GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "quark_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE double)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fvisibility=hidden",
               "-fno-fast-math", "-ffp-contract=off", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        L.or_reprojection_matrix.restype = ctypes.c_int
        L.or_reproject.restype = ctypes.c_int
        L.or_reproject_T.restype = ctypes.c_int
        L.or_update_fuse.restype = ctypes.c_int
        L.or_render_ibr.restype = ctypes.c_int
        L.or_render_to_views.restype = ctypes.c_int
        L.or_ray_encoding.restype = ctypes.c_int
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later OpenMP regions (n <= 0: unchanged)."""
    lib().or_set_num_threads(int(n))


# --------------------------------------------------------------------------
# Step-level entry points (each maps to one C function)
# --------------------------------------------------------------------------

def scale_intrinsics(K, w0, h0, w1, h1) -> np.ndarray:
    K = _f64(K)
    out = np.zeros(9)
    lib().or_scale_intrinsics(_d(K), int(w0), int(h0), int(w1), int(h1), _d(out))
    return out.reshape(3, 3)


def reprojection_matrix(Kn, En, Km, Em) -> np.ndarray:
    Kn, En, Km, Em = map(_f64, (Kn, En, Km, Em))
    T = np.zeros(16)
    rc = lib().or_reprojection_matrix(_d(Kn), _d(En), _d(Km), _d(Em), _d(T))
    if rc != 0:
        raise ValueError("singular camera matrix")
    return T.reshape(4, 4)


def reproject(Kn, En, Km, Em, u, v, d):
    """Returns ((u_m, v_m), valid)."""
    Kn, En, Km, Em = map(_f64, (Kn, En, Km, Em))
    out = np.zeros(2)
    rc = lib().or_reproject(_d(Kn), _d(En), _d(Km), _d(Em), ctypes.c_double(u),
                            ctypes.c_double(v), ctypes.c_double(d), _d(out))
    if rc < 0:
        raise ValueError("singular camera matrix")
    return (float(out[0]), float(out[1])), bool(rc == 1)


def bilinear(I, u, v) -> np.ndarray:
    I = _f64(I)
    Hf, Wf, C = I.shape
    s = np.zeros(C)
    lib().or_bilinear(_d(I), Hf, Wf, C, ctypes.c_double(u), ctypes.c_double(v), _d(s))
    return s


def rmsnorm(x) -> np.ndarray:
    x = _f64(x)
    y = np.zeros_like(x)
    lib().or_rmsnorm(_d(x), x.shape[0], _d(y))
    return y


def attention(F, S, heads, dh, Wq, Wk, Wv, Wo, folded: bool = False):
    """One layer-pixel: returns (F', p[heads][V]) (p is None when folded)."""
    F, S, Wq, Wk, Wv, Wo = map(_f64, (F, S, Wq, Wk, Wv, Wo))
    C = F.shape[0]
    V, Cf = S.shape
    out = np.zeros(C)
    if folded:
        lib().or_attention_folded(_d(F), C, _d(S), V, Cf, heads, dh, _d(Wq), _d(Wk), _d(Wv),
                                  _d(Wo), _d(out))
        return out, None
    p = np.zeros((heads, V))
    lib().or_attention(_d(F), C, _d(S), V, Cf, heads, dh, _d(Wq), _d(Wk), _d(Wv), _d(Wo),
                       _d(out), _d(p))
    return out, p


def blend_logits(F, S, heads, dh, Wq, Wk) -> np.ndarray:
    """One layer-pixel's blend-weight logits [V] (first head's attention
    logits, before the softmax)."""
    F, S, Wq, Wk = map(_f64, (F, S, Wq, Wk))
    C = F.shape[0]
    V, Cf = S.shape
    out = np.zeros(V)
    lib().or_blend_logits(_d(F), C, _d(S), V, Cf, heads, dh, _d(Wq), _d(Wk), _d(out))
    return out


def decode(Fp, w_sigma, w_depth, W_color, alpha, depth, li, L, near, far, mode=0):
    """Returns (alpha', depth', color'[3])."""
    Fp, w_sigma, w_depth, W_color = map(_f64, (Fp, w_sigma, w_depth, W_color))
    a = ctypes.c_double()
    d = ctypes.c_double()
    c = np.zeros(3)
    lib().or_decode(_d(Fp), Fp.shape[0], _d(w_sigma), _d(w_depth), _d(W_color),
                    ctypes.c_double(alpha), ctypes.c_double(depth), int(li), int(L),
                    ctypes.c_double(near), ctypes.c_double(far), int(mode), ctypes.byref(a),
                    ctypes.byref(d), _d(c))
    return a.value, d.value, c


def composite(color, alpha, back_to_front: bool = False):
    """color [L][...][3], alpha [L][...] -> (rgb [...][3], acc [...])."""
    color = _f64(color)
    alpha = _f64(alpha)
    L = alpha.shape[0]
    pix_shape = alpha.shape[1:]
    npix = int(np.prod(pix_shape)) if pix_shape else 1
    rgb = np.zeros((npix, 3))
    acc = np.zeros(npix)
    if back_to_front:
        lib().or_composite_back_to_front(L, ctypes.c_long(npix), _d(color), _d(alpha), _d(rgb))
        return rgb.reshape(pix_shape + (3,)), None
    lib().or_composite(L, ctypes.c_long(npix), _d(color), _d(alpha), _d(rgb), _d(acc))
    return rgb.reshape(pix_shape + (3,)), acc.reshape(pix_shape)


def composite_backward(color, alpha, d_rgb, d_acc=None):
    """Adjoint of ``composite``: (d_color [L][...][3], d_alpha [L][...]) from
    d_rgb [...][3] and, optionally, d_acc [...] (Sec. 3.1, chain rule)."""
    color = _f64(color)
    alpha = _f64(alpha)
    d_rgb = _f64(d_rgb)
    L = alpha.shape[0]
    pix_shape = alpha.shape[1:]
    npix = int(np.prod(pix_shape)) if pix_shape else 1
    dc = np.zeros((L, npix, 3))
    da = np.zeros((L, npix))
    dA = _f64(d_acc) if d_acc is not None else None
    lib().or_composite_backward(L, ctypes.c_long(npix), _d(color), _d(alpha), _d(d_rgb),
                                _d(dA) if dA is not None else ctypes.cast(None, _dp),
                                _d(dc), _d(da))
    return dc.reshape((L,) + pix_shape + (3,)), da.reshape((L,) + pix_shape)


# --------------------------------------------------------------------------
# Final render: upsample & activate, blend-weight image-based render
# --------------------------------------------------------------------------

def upsample_bilinear(src, H: int, W: int) -> np.ndarray:
    """src [h][w] or [h][w][C] -> [H][W](...) (half-pixel centres, border
    extended)."""
    src = _f64(src)
    squeeze = src.ndim == 2
    if squeeze:
        src = src[..., None]
    h, w, C = src.shape
    dst = np.zeros((H, W, C))
    lib().or_upsample_bilinear(_d(src), h, w, C, int(H), int(W), _d(dst))
    return dst[..., 0] if squeeze else dst


def ibr_activate(xd, xs, xb, li, L, near, far):
    """One layer-pixel's activation: returns (depth, sigma, beta[V])."""
    xb = _f64(xb)
    d = ctypes.c_double()
    sg = ctypes.c_double()
    beta = np.zeros(xb.shape[0])
    lib().or_ibr_activate(ctypes.c_double(xd), ctypes.c_double(xs), _d(xb), xb.shape[0],
                          int(li), int(L), ctypes.c_double(near), ctypes.c_double(far),
                          ctypes.byref(d), ctypes.byref(sg), _d(beta))
    return d.value, sg.value, beta


def image_rgb(img) -> np.ndarray:
    """An RGBA8 image [H][W][4] as the RGB values in [0, 1] the render reads."""
    return np.ascontiguousarray(np.asarray(img)[..., :3], dtype=np.float64) / 255.0


def render_ibr(in_cams, images, novel, near, far, depth_logit, sigma_logit, blend_logit,
               H: int, W: int, *, rows: Optional[Sequence[int]] = None,
               want_layers: bool = False) -> Dict[str, np.ndarray]:
    """The final render on the given output rows (default: all).  ``images``
    are RGBA8 arrays [Hi][Wi][4] (or float RGB [Hi][Wi][3] in [0, 1]); the
    logits are [L][h][w] (depth, density) and [L][h][w][V] (blend)."""
    V = len(in_cams)
    img64 = [image_rgb(im) if np.asarray(im).dtype == np.uint8 else _f64(im) for im in images]
    dl, sl, bl = _f64(depth_logit), _f64(sigma_logit), _f64(blend_logit)
    L, h, w = dl.shape
    rows = np.arange(H, dtype=np.int32) if rows is None else np.asarray(rows, dtype=np.int32)
    R = int(rows.shape[0])
    Kin = _f64(np.stack([c.K for c in in_cams]))
    Ein = _f64(np.stack([c.E for c in in_cams]))
    cam_wh = np.ascontiguousarray([[c.width, c.height] for c in in_cams], dtype=np.int32)
    img_hw = np.ascontiguousarray([[im.shape[0], im.shape[1]] for im in img64], dtype=np.int32)
    iptrs = (_dp * V)(*[_d(im) for im in img64])
    nov_wh = np.array([novel.width, novel.height], dtype=np.int32)
    Kn, En = _f64(novel.K), _f64(novel.E)
    rgb = np.zeros((R, W, 3))
    acc = np.zeros((R, W))
    dmap = np.zeros((R, W))
    lc = np.zeros((L, R, W, 3)) if want_layers else None
    rc = lib().or_render_ibr(
        V, _d(Kin), _d(Ein), cam_wh.ctypes.data_as(_ip), iptrs, img_hw.ctypes.data_as(_ip),
        _d(Kn), _d(En), nov_wh.ctypes.data_as(_ip), ctypes.c_double(near), ctypes.c_double(far),
        L, h, w, _d(dl), _d(sl), _d(bl), int(H), int(W), rows.ctypes.data_as(_ip), R,
        _d(rgb), _d(acc), _d(dmap), _d(lc) if lc is not None else ctypes.cast(None, _dp))
    if rc != 0:
        raise ValueError("oracle render_ibr failed (singular camera?)")
    out = {"rgb": rgb, "acc": acc, "depth": dmap, "rows": rows}
    if lc is not None:
        out["layer_color"] = lc
    return out


# --------------------------------------------------------------------------
# Render to input views (projection operator P_theta and per-view composite)
# --------------------------------------------------------------------------

def splat_layer(T, depth, val, Hm: int, Wm: int) -> np.ndarray:
    """P_theta of one layer: val [H][W] or [H][W][C] at depth [H][W] (novel
    grid) into an (Hm, Wm) view grid through the 4x4 chain T."""
    T, depth, val = _f64(T), _f64(depth), _f64(val)
    squeeze = val.ndim == 2
    if squeeze:
        val = val[..., None]
    H, W, C = val.shape
    out = np.zeros((Hm, Wm, C))
    lib().or_splat_layer(_d(T), H, W, _d(depth), _d(val), C, int(Hm), int(Wm), _d(out))
    return out[..., 0] if squeeze else out


def render_to_views(in_cams, novel, depth, alpha, color, view_hw) -> Dict[str, list]:
    """Eq. 2 for every view: depth, alpha [L][H][W], color [L][H][W][3]
    (novel grid); view_hw [V] of (Hm, Wm).  Returns {"img": [V] [Hm][Wm][3],
    "acc": [V] [Hm][Wm]}."""
    V = len(in_cams)
    depth, alpha, color = _f64(depth), _f64(alpha), _f64(color)
    L, H, W = depth.shape
    Kin = _f64(np.stack([c.K for c in in_cams]))
    Ein = _f64(np.stack([c.E for c in in_cams]))
    cam_wh = np.ascontiguousarray([[c.width, c.height] for c in in_cams], dtype=np.int32)
    vhw = np.ascontiguousarray(view_hw, dtype=np.int32).reshape(V, 2)
    imgs = [np.zeros((int(h), int(w), 3)) for h, w in vhw]
    accs = [np.zeros((int(h), int(w))) for h, w in vhw]
    iptr = (_dp * V)(*[_d(a) for a in imgs])
    aptr = (_dp * V)(*[_d(a) for a in accs])
    nov_wh = np.array([novel.width, novel.height], dtype=np.int32)
    rc = lib().or_render_to_views(V, _d(Kin), _d(Ein), cam_wh.ctypes.data_as(_ip),
                                  vhw.ctypes.data_as(_ip), _d(_f64(novel.K)), _d(_f64(novel.E)),
                                  nov_wh.ctypes.data_as(_ip), L, H, W, _d(depth), _d(alpha),
                                  _d(color), iptr, aptr)
    if rc != 0:
        raise ValueError("oracle render_to_views failed (singular camera?)")
    return {"img": imgs, "acc": accs}


# --------------------------------------------------------------------------
# Residual CNN block of a fusion block
# --------------------------------------------------------------------------

def residual_conv(F, W1, W2) -> np.ndarray:
    """V' = V + W2 * gelu(W1 * N(V)) per layer (N the per-pixel RMS
    normalisation): F [L][H][W][C] (float32, or bfloat16 bit patterns), W1,
    W2 [3][3][C][C]."""
    F = _as_f64_array(F)
    W1, W2 = _f64(W1), _f64(W2)
    L, H, W, C = F.shape
    out = np.zeros_like(F)
    lib().or_residual_conv(L, H, W, C, _d(F), _d(W1), _d(W2), _d(out))
    return out


def layer_collapse(F, W1, W2) -> np.ndarray:
    """out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2: F
    [L][H][W][C] (L even; float32 or bfloat16 bits), W1 [2C][C], W2 [C][C]."""
    F = _as_f64_array(F)
    W1, W2 = _f64(W1), _f64(W2)
    L, H, W, C = F.shape
    out = np.zeros((L // 2, H, W, C))
    lib().or_layer_collapse(L, H, W, C, _d(F), _d(W1), _d(W2), _d(out))
    return out


def ray_encoding(cam, novel, near, far, Wr, Hf: int, Wf: int, want_delta: bool = False):
    """The ray-direction encoding of ``cam``'s pixels on an (Hf, Wf) grid:
    returns out [Hf][Wf][C] (and the NDC difference [Hf][Wf][2])."""
    Wr = _f64(Wr)
    C = Wr.shape[1]
    out = np.zeros((Hf, Wf, C))
    dl = np.zeros((Hf, Wf, 2)) if want_delta else None
    cwh = np.array([cam.width, cam.height], dtype=np.int32)
    nwh = np.array([novel.width, novel.height], dtype=np.int32)
    rc = lib().or_ray_encoding(_d(_f64(cam.K)), _d(_f64(cam.E)), cwh.ctypes.data_as(_ip), int(Hf),
                               int(Wf), _d(_f64(novel.K)), _d(_f64(novel.E)),
                               nwh.ctypes.data_as(_ip), ctypes.c_double(near),
                               ctypes.c_double(far), _d(Wr), C, _d(out),
                               _d(dl) if dl is not None else ctypes.cast(None, _dp))
    if rc != 0:
        raise ValueError("oracle ray_encoding failed (singular camera?)")
    return (out, dl) if want_delta else out


def upsample2x(src):
    """Bilinear upsampling by two of src [N][H][W][C] (half-pixel centres,
    border extended): the general resampling at (2H, 2W), per n."""
    src = _f64(src)
    return np.stack([upsample_bilinear(s, 2 * s.shape[0], 2 * s.shape[1]) for s in src])


def decode_volume(F, w_sigma, w_depth, W_color, near, far):
    """The absolute decode (Sec. 3.2.2-3.2.3, the paper's depth anchors) of
    every layer-pixel of F [L][H][W][C]: returns (depth, alpha, color)."""
    F = _as_f64_array(F)
    L, H, W, _ = F.shape
    depth, alpha, color = np.zeros((L, H, W)), np.zeros((L, H, W)), np.zeros((L, H, W, 3))
    for li in range(L):
        for y in range(H):
            for x in range(W):
                a, d, c = decode(F[li, y, x], w_sigma, w_depth, W_color, 0.5, 1.0, li, L, near,
                                 far, mode=1)
                depth[li, y, x], alpha[li, y, x], color[li, y, x] = d, a, c
    return depth, alpha, color


def ray_encoding_lowres(cam, novel, near, far, Wr, low_hw, Hf: int, Wf: int):
    """The paper's form of the ray-direction encoding (Sec. 3.2.2, "Encode
    Input Images"): the 8-octave sinusoids evaluated once on the
    low-resolution grid ``low_hw`` = (h, w), bilinearly upsampled to the
    (Hf, Wf) map grid, then projected by Wr: returns [Hf][Wf][C]."""
    h, w = int(low_hw[0]), int(low_hw[1])
    e = ray_encoding(cam, novel, near, far, np.eye(32), h, w)
    return upsample_bilinear(e, Hf, Wf) @ _f64(Wr)


# --------------------------------------------------------------------------
# Whole step over a scene level
# --------------------------------------------------------------------------

def _as_f64_array(a: np.ndarray) -> np.ndarray:
    if a.dtype == np.uint16:          # bfloat16 bit patterns -> exact values
        return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def update_fuse(in_cams, novel, near, far, level, *, F=None, depth=None, alpha=None,
                rows: Optional[Sequence[int]] = None, mode: int = 0, attn_form: int = 0,
                want_samples: bool = False, feats64: Optional[List[np.ndarray]] = None,
                want_logits: bool = False) -> Dict[str, np.ndarray]:
    """One Update & Fuse step of ``level`` (a ``synth.Level``) on the given
    rows (default: all).  ``F``/``depth``/``alpha`` override the level's state
    (full-size arrays, used for multi-step runs)."""
    V = len(in_cams)
    L, H, W, C, Cf = level.L, level.H, level.W, level.C, level.Cf
    rows = np.arange(H, dtype=np.int32) if rows is None else np.asarray(rows, dtype=np.int32)
    R = int(rows.shape[0])
    Kin = _f64(np.stack([c.K for c in in_cams]))
    Ein = _f64(np.stack([c.E for c in in_cams]))
    cam_wh = np.ascontiguousarray([[c.width, c.height] for c in in_cams], dtype=np.int32)
    if feats64 is None:
        feats64 = [_as_f64_array(f) for f in level.feats]
    feat_hw = np.ascontiguousarray([[f.shape[0], f.shape[1]] for f in feats64], dtype=np.int32)
    fptrs = (_dp * V)(*[_d(f) for f in feats64])
    F64 = _as_f64_array(level.F if F is None else F)
    d64 = _as_f64_array(level.depth if depth is None else depth)
    a64 = _as_f64_array(level.alpha if alpha is None else alpha)
    w = {k: _f64(v) for k, v in level.weights.items()}
    nov_wh = np.array([novel.width, novel.height], dtype=np.int32)
    Kn, En = _f64(novel.K), _f64(novel.E)
    F_out = np.zeros((L, R, W, C))
    d_out = np.zeros((L, R, W))
    a_out = np.zeros((L, R, W))
    c_out = np.zeros((L, R, W, 3))
    s_out = np.zeros((L, R, W, V, Cf)) if want_samples else None
    g_out = np.zeros((L, R, W, V)) if want_logits else None
    rc = lib().or_update_fuse(
        V, _d(Kin), _d(Ein), cam_wh.ctypes.data_as(_ip), fptrs, feat_hw.ctypes.data_as(_ip), Cf,
        _d(Kn), _d(En), nov_wh.ctypes.data_as(_ip), ctypes.c_double(near), ctypes.c_double(far),
        L, H, W, C, _d(F64), _d(d64), _d(a64), level.heads, level.head_dim,
        _d(w["Wq"]), _d(w["Wk"]), _d(w["Wv"]), _d(w["Wo"]), _d(w["w_sigma"]), _d(w["w_depth"]),
        _d(w["W_color"]), int(mode), int(attn_form), rows.ctypes.data_as(_ip), R,
        _d(F_out), _d(d_out), _d(a_out), _d(c_out),
        _d(s_out) if s_out is not None else ctypes.cast(None, _dp),
        _d(g_out) if g_out is not None else ctypes.cast(None, _dp))
    if rc != 0:
        raise ValueError("oracle update_fuse failed (singular camera?)")
    out = {"F": F_out, "depth": d_out, "alpha": a_out, "color": c_out, "rows": rows}
    if s_out is not None:
        out["samples"] = s_out
    if g_out is not None:
        out["blend_logit"] = g_out
    return out


def run_level(scene, level, *, steps: Optional[int] = None, rows=None, mode: int = 0,
              attn_form: int = 0, composite_out: Optional[bool] = None):
    """``steps`` Update & Fuse steps of one level on the given rows, then (if
    requested) the composite of the last step.  Multi-step runs feed
    (F', depth', alpha') back in; layer-pixels are independent, so sampled rows
    are exact."""
    steps = scene.steps if steps is None else steps
    composite_out = level.composite if composite_out is None else composite_out
    feats64 = [_as_f64_array(f) for f in level.feats]
    H = level.H
    rows_arr = np.arange(H, dtype=np.int32) if rows is None else np.asarray(rows, dtype=np.int32)
    F = _as_f64_array(level.F)
    d = _as_f64_array(level.depth)
    a = _as_f64_array(level.alpha)
    out = None
    for s in range(steps):
        out = update_fuse(scene.in_cams, scene.novel, scene.near, scene.far, level, F=F,
                          depth=d, alpha=a, rows=rows_arr, mode=mode, attn_form=attn_form,
                          feats64=feats64)
        if s + 1 < steps:
            # write the sampled rows back into full-size state for the next step
            F = F.copy(); d = d.copy(); a = a.copy()
            F[:, rows_arr] = out["F"]
            d[:, rows_arr] = out["depth"]
            a[:, rows_arr] = out["alpha"]
    if composite_out:
        rgb, acc = composite(out["color"], out["alpha"])
        out["rgb"] = rgb
        out["acc"] = acc
    return out


def run_chain(ch, attn_form: int = 0):
    """The chained steps of a ``synth.ChainScene`` (Sec. 3.2.2 iterative
    updates): step i > 0 takes step i - 1's output features, collapses their
    layers and / or upsamples them by two as its transition asks; every step
    decodes its input features (the absolute decode), runs Update & Fuse with
    the absolute decode and, if it has one, its residual CNN block; the last
    step's output LDM (decoded after the block) is composited.  Returns the
    per-step outputs and the final rgb / acc."""
    F = _as_f64_array(ch.F0)
    outs = []
    n = len(ch.steps)
    for i, st in enumerate(ch.steps):
        if i > 0:
            F = outs[-1]["F_next"]
            if st.collapse:
                F = layer_collapse(F, *ch.collapse_w[i])
            if st.upsample:
                F = upsample2x(F)
        w = ch.weights[i]
        d, a, _ = decode_volume(F, w["w_sigma"], w["w_depth"], w["W_color"], ch.near, ch.far)
        out = update_fuse(ch.in_cams, ch.novel, ch.near, ch.far, ch.level(i), F=F, depth=d,
                          alpha=a, mode=1, attn_form=attn_form)
        out["F_in"], out["depth_in"], out["alpha_in"] = F, d, a
        out["F_next"] = out["F"]
        if st.conv:
            out["F_conv"] = residual_conv(out["F"], *ch.conv_w[i])
            out["F_next"] = out["F_conv"]
            if i == n - 1:
                out["depth"], out["alpha"], out["color"] = decode_volume(
                    out["F_conv"], w["w_sigma"], w["w_depth"], w["W_color"], ch.near, ch.far)
        outs.append(out)
    rgb, acc = composite(outs[-1]["color"], outs[-1]["alpha"])
    return outs, rgb, acc


def volume_logits(F, w_sigma, w_depth):
    """The final LDM's unactivated attributes (Sec. 3.2.3: linear
    projections, activated only after the render's upsampling): returns
    (depth_logit, sigma_logit) = (F . w_depth, F . w_sigma) per layer-pixel."""
    F = _as_f64_array(F)
    return F @ _f64(w_depth), F @ _f64(w_sigma)


def encode_pyramid(pl):
    """Every pyramid level's maps plus their ray-direction encoding (Sec.
    3.2.1; the paper's low-resolution form, one projection per level)."""
    ch = pl.chain
    out = []
    for k, lvl in enumerate(ch.feats):
        enc = []
        for m, f in enumerate(lvl):
            f64 = _as_f64_array(f)
            Hf, Wf = f64.shape[:2]
            enc.append(f64 + ray_encoding_lowres(ch.in_cams[m], ch.novel, ch.near, ch.far,
                                                 pl.Wr[k], pl.low_hw, Hf, Wf))
        out.append(enc)
    return out


def run_pipeline(pl, attn_form: int = 0, rows: Optional[Sequence[int]] = None):
    """The whole frame of a ``synth.PipelineScene``: the ray-encoded pyramid;
    the learned initialisation (f0 broadcast, flat layers at the anchors,
    alpha 1/2) as the first step's LDM; the chained steps (transition,
    absolute decode of the step's input, Update & Fuse, residual CNN block),
    the last of which also gives the blend-weight logits of its attention;
    the unactivated decode of the final feature volume; and the final render
    (Eq. 1: upsample, activate, blend the input images, composite) at the
    output grid, on ``rows`` of it (default all).  Returns (per-step outputs,
    render outputs, encoded pyramid)."""
    ch = pl.chain
    feats = encode_pyramid(pl)
    s0 = ch.steps[0]
    F, d, a = ldm_init(s0.L, s0.H, s0.W, pl.f0, ch.near, ch.far)
    outs = []
    n = len(ch.steps)
    for i, st in enumerate(ch.steps):
        w = ch.weights[i]
        if i > 0:
            F = outs[-1]["F_next"]
            if st.collapse:
                F = layer_collapse(F, *ch.collapse_w[i])
            if st.upsample:
                F = upsample2x(F)
            d, a, _ = decode_volume(F, w["w_sigma"], w["w_depth"], w["W_color"], ch.near, ch.far)
        out = update_fuse(ch.in_cams, ch.novel, ch.near, ch.far, ch.level(i), F=F, depth=d,
                          alpha=a, mode=1, attn_form=attn_form, feats64=feats[st.level],
                          want_logits=(i == n - 1))
        out["F_in"], out["depth_in"], out["alpha_in"] = F, d, a
        out["F_next"] = residual_conv(out["F"], *ch.conv_w[i]) if st.conv else out["F"]
        outs.append(out)
    w = ch.weights[-1]
    dl, sl = volume_logits(outs[-1]["F_next"], w["w_sigma"], w["w_depth"])
    H, W = pl.out_hw
    r = render_ibr(ch.in_cams, pl.images, ch.novel, ch.near, ch.far, dl, sl,
                   outs[-1]["blend_logit"], H, W, rows=rows)
    r["depth_logit"], r["sigma_logit"] = dl, sl
    return outs, r, feats


def run_scene(scene, *, rows_per_level=None, mode: int = 0, attn_form: int = 0):
    """All levels of a scene.  ``rows_per_level`` is a list (one entry per
    level, None = all rows)."""
    res = []
    for i, lvl in enumerate(scene.levels):
        rows = None if rows_per_level is None else rows_per_level[i]
        res.append(run_level(scene, lvl, rows=rows, mode=mode, attn_form=attn_form))
    return res


def update_fuse_backward(in_cams, novel, near, far, level, *, d_rgb=None, dF_out=None,
                         d_depth_out=None, d_alpha_out=None, rows=None, mode: int = 0,
                         F=None, depth=None, alpha=None, feats64=None):
    """Adjoint of one Update & Fuse step + composite (standard form).

    Upstream gradients are full-size arrays (or None); only ``rows`` (default
    all) are processed and every other row's upstream gradient counts as
    zero, so the result is the exact gradient of a loss restricted to those
    rows.  Returns a dict of float64 gradients: F, depth, alpha, feats (list),
    Wq, Wk, Wv, Wo, w_sigma, w_depth, W_color."""
    V = len(in_cams)
    L, H, W, C, Cf = level.L, level.H, level.W, level.C, level.Cf
    rows = np.arange(H, dtype=np.int32) if rows is None else np.asarray(rows, dtype=np.int32)
    Kin = _f64(np.stack([c.K for c in in_cams]))
    Ein = _f64(np.stack([c.E for c in in_cams]))
    cam_wh = np.ascontiguousarray([[c.width, c.height] for c in in_cams], dtype=np.int32)
    if feats64 is None:
        feats64 = [_as_f64_array(f) for f in level.feats]
    feat_hw = np.ascontiguousarray([[f.shape[0], f.shape[1]] for f in feats64], dtype=np.int32)
    fptrs = (_dp * V)(*[_d(f) for f in feats64])
    F64 = _as_f64_array(level.F if F is None else F)
    d64 = _as_f64_array(level.depth if depth is None else depth)
    a64 = _as_f64_array(level.alpha if alpha is None else alpha)
    w = {k: _f64(v) for k, v in level.weights.items()}
    nov_wh = np.array([novel.width, novel.height], dtype=np.int32)
    Kn, En = _f64(novel.K), _f64(novel.E)
    null = ctypes.cast(None, _dp)
    ups = [None if a is None else _f64(a) for a in (d_rgb, dF_out, d_depth_out, d_alpha_out)]
    g = {"F": np.zeros_like(F64), "depth": np.zeros_like(d64), "alpha": np.zeros_like(a64),
         "feats": [np.zeros_like(f) for f in feats64]}
    for k in ("Wq", "Wk", "Wv", "Wo", "w_sigma", "w_depth", "W_color"):
        g[k] = np.zeros_like(w[k])
    dIptrs = (_dp * V)(*[_d(a) for a in g["feats"]])
    rc = lib().or_update_fuse_backward(
        V, _d(Kin), _d(Ein), cam_wh.ctypes.data_as(_ip), fptrs, feat_hw.ctypes.data_as(_ip), Cf,
        _d(Kn), _d(En), nov_wh.ctypes.data_as(_ip), ctypes.c_double(near), ctypes.c_double(far),
        L, H, W, C, _d(F64), _d(d64), _d(a64), level.heads, level.head_dim,
        _d(w["Wq"]), _d(w["Wk"]), _d(w["Wv"]), _d(w["Wo"]), _d(w["w_sigma"]), _d(w["w_depth"]),
        _d(w["W_color"]), int(mode), rows.ctypes.data_as(_ip), int(rows.shape[0]),
        *[null if a is None else _d(a) for a in ups],
        _d(g["F"]), _d(g["depth"]), _d(g["alpha"]), dIptrs,
        _d(g["Wq"]), _d(g["Wk"]), _d(g["Wv"]), _d(g["Wo"]), _d(g["w_sigma"]), _d(g["w_depth"]),
        _d(g["W_color"]))
    if rc != 0:
        raise ValueError("oracle backward failed (singular camera?)")
    return g


def sample_coordinates(in_cams, novel, level, depth=None):
    """Sample coordinate (u_m, v_m) of every layer-pixel in every view, NaN
    where the point is behind the view: array [L][H][W][V][2].  Used to keep
    finite-difference probes away from the kinks of bilinear sampling."""
    L, H, W = level.L, level.H, level.W
    d = _as_f64_array(level.depth if depth is None else depth)
    out = np.full((L, H, W, len(in_cams), 2), np.nan)
    Kn = scale_intrinsics(novel.K, novel.width, novel.height, W, H)
    for m, cam in enumerate(in_cams):
        Hf, Wf = level.feats[m].shape[:2]
        Km = scale_intrinsics(cam.K, cam.width, cam.height, Wf, Hf)
        T = reprojection_matrix(Kn, novel.E, Km, cam.E).reshape(16)
        uv = np.zeros(2)
        for li in range(L):
            for y in range(H):
                for x in range(W):
                    ok = lib().or_reproject_T(_d(T), ctypes.c_double(x + 0.5),
                                              ctypes.c_double(y + 0.5),
                                              ctypes.c_double(d[li, y, x]), _d(uv))
                    if ok == 1:
                        out[li, y, x, m] = uv
    return out


def ldm_init(L: int, H: int, W: int, f0, near: float, far: float):
    """The learned initialisation of an LDM (Sec. 3.2, "Initialization"):
    the single C-channel feature f0 broadcast to every layer-pixel, each layer
    flat at its depth anchor (Sec. 3.2.3: the paper's layer l sits at
    disparity fraction (l - 1/2)/L of the band, storage layer i = L - l with
    0 nearest), alpha one half (the paper leaves it unstated; reading).
    Returns (F [L][H][W][C], depth [L][H][W], alpha [L][H][W]) in float64."""
    f0 = _f64(f0)
    band = 1.0 / near - 1.0 / far
    depth = np.empty((L, H, W))
    for i in range(L):
        l_paper = L - i
        delta = (l_paper - 0.5) / L
        depth[i] = 1.0 / (delta * band + 1.0 / far)
    F = np.broadcast_to(f0, (L, H, W, f0.shape[0])).copy()
    alpha = np.full((L, H, W), 0.5)
    return F, depth, alpha
