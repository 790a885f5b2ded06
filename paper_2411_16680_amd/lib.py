"""Thin ctypes binding of libquark (C-ABI in include/quark.h).

Argument marshalling only: every step of the Update & Fuse path runs in the
library's HIP kernels.  Device buffers are torch tensors on a ROCm device
(torch supplies memory and streams).  There is no fallback: if the library is
missing or a call fails, a ``QuarkError`` is raised.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libquark.so")

QK_OK, QK_EINVAL, QK_ESHAPE, QK_EDTYPE, QK_ENOMEM, QK_EHIP, QK_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "QK_OK", -1: "QK_EINVAL", -2: "QK_ESHAPE", -3: "QK_EDTYPE", -4: "QK_ENOMEM",
                -5: "QK_EHIP", -6: "QK_EUNSUPPORTED"}
QK_F32, QK_BF16 = 0, 1
PREC = {"fp32": 0, "bf16": 1, "bf16_fp8proj": 2}
ATTN = {"standard": 0, "folded": 1}
MODE = {"residual": 0, "paper": 1}

# symbols include/quark.h declares (checked by the CPU tests)
EXPORTS = ["qk_context_create", "qk_context_destroy", "qk_context_weights_static", "qk_update_fuse", "qk_update_fuse_check",
           "qk_update_fuse_noalloc", "qk_batch_update_fuse", "qk_batch_update_fuse_check",
           "qk_update_fuse_backward", "qk_update_fuse_backward_check", "qk_ldm_init",
           "qk_composite", "qk_composite_backward", "qk_composite_backward_check",
           "qk_render_ibr", "qk_render_ibr_check", "qk_render_to_views",
           "qk_render_to_views_check", "qk_residual_conv", "qk_residual_conv_check",
           "qk_layer_collapse", "qk_layer_collapse_check", "qk_ray_encoding",
           "qk_ray_encoding_check", "qk_upsample2x", "qk_upsample2x_check", "qk_ldm_decode",
           "qk_ldm_decode_check", "qk_ldm_decode_logits", "qk_ldm_decode_logits_check",
           "qk_camera_tables", "qk_last_error", "qk_version"]


class QuarkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class qk_camera(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double * 9), ("E", ctypes.c_double * 16),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class qk_feature_map(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("C", ctypes.c_int32)]


class qk_feature_map_inout(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("src", ctypes.c_void_p)]


class qk_image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class qk_ldm_logits(ctypes.Structure):
    _fields_ = [("depth_logit", ctypes.c_void_p), ("sigma_logit", ctypes.c_void_p),
                ("blend_logit", ctypes.c_void_p), ("L", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("V", ctypes.c_int32)]


class qk_ldm_decoded(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("color", ctypes.c_void_p),
                ("L", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class qk_view_image(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32)]


class qk_ldm(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("L", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("C", ctypes.c_int32), ("dtype", ctypes.c_int)]


class qk_weights(ctypes.Structure):
    _fields_ = [("Wq", ctypes.c_void_p), ("Wk", ctypes.c_void_p), ("Wv", ctypes.c_void_p),
                ("Wo", ctypes.c_void_p), ("w_sigma", ctypes.c_void_p),
                ("w_depth", ctypes.c_void_p), ("W_color", ctypes.c_void_p),
                ("C", ctypes.c_int32), ("C_feat", ctypes.c_int32), ("heads", ctypes.c_int32),
                ("head_dim", ctypes.c_int32)]


class qk_request_desc(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int32), ("in_cams", ctypes.c_void_p), ("feats", ctypes.c_void_p),
                ("novel", ctypes.c_void_p), ("near_", ctypes.c_float), ("far_", ctypes.c_float),
                ("weights", ctypes.c_void_p), ("update_mode", ctypes.c_int),
                ("ldm_in", ctypes.c_void_p), ("ldm_out", ctypes.c_void_p),
                ("rgb_out", ctypes.c_void_p), ("acc_alpha_out", ctypes.c_void_p),
                ("blend_logit_out", ctypes.c_void_p)]


class qk_weight_grads(ctypes.Structure):
    _fields_ = [("Wq", ctypes.c_void_p), ("Wk", ctypes.c_void_p), ("Wv", ctypes.c_void_p),
                ("Wo", ctypes.c_void_p), ("w_sigma", ctypes.c_void_p),
                ("w_depth", ctypes.c_void_p), ("W_color", ctypes.c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libquark.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QuarkError(QK_EINVAL, f"{LIB_PATH} not built (run python -m paper_2411_16680_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.qk_last_error.restype = ctypes.c_char_p
    L.qk_version.restype = ctypes.c_char_p
    P = ctypes.POINTER
    L.qk_context_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(ctypes.c_void_p)]
    L.qk_context_destroy.argtypes = [ctypes.c_void_p]
    L.qk_context_weights_static.argtypes = [ctypes.c_void_p, ctypes.c_int]
    uf_args = [ctypes.c_int32, P(qk_camera), P(qk_feature_map), P(qk_camera), ctypes.c_float,
               ctypes.c_float, P(qk_weights), ctypes.c_int, ctypes.c_int, ctypes.c_int,
               P(qk_ldm), P(qk_ldm), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.qk_update_fuse.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + uf_args
    L.qk_update_fuse_check.argtypes = uf_args
    L.qk_update_fuse_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + uf_args
    L.qk_batch_update_fuse.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       P(qk_request_desc), ctypes.c_int, ctypes.c_int]
    L.qk_batch_update_fuse_check.argtypes = [ctypes.c_int32, P(qk_request_desc), ctypes.c_int,
                                             ctypes.c_int]
    bwd_args = [ctypes.c_int32, P(qk_camera), P(qk_feature_map), P(qk_camera), ctypes.c_float,
                ctypes.c_float, P(qk_weights), ctypes.c_int, P(qk_ldm), P(qk_ldm), ctypes.c_void_p,
                P(qk_ldm), P(qk_ldm), P(ctypes.c_void_p), P(qk_weight_grads)]
    L.qk_update_fuse_backward.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + bwd_args
    L.qk_update_fuse_backward_check.argtypes = bwd_args
    L.qk_ldm_init.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                              ctypes.c_float, P(qk_ldm)]
    L.qk_composite.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p]
    cb_args = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32] + [ctypes.c_void_p] * 6
    L.qk_composite_backward.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + cb_args
    L.qk_composite_backward_check.argtypes = cb_args
    L.qk_camera_tables.argtypes = [ctypes.c_int32, P(qk_camera), P(ctypes.c_int32), P(qk_camera),
                                   ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double)]
    render_args = [ctypes.c_int32, P(qk_camera), P(qk_image), P(qk_camera), ctypes.c_float,
                   ctypes.c_float, P(qk_ldm_logits), ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.qk_render_ibr.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + render_args
    L.qk_render_ibr_check.argtypes = render_args
    views_args = [ctypes.c_int32, P(qk_camera), P(qk_camera), P(qk_ldm_decoded), P(qk_view_image)]
    L.qk_render_to_views.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + views_args
    L.qk_render_to_views_check.argtypes = views_args
    conv_args = [P(qk_ldm), ctypes.c_void_p, ctypes.c_void_p, P(qk_ldm)]
    L.qk_residual_conv.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + conv_args
    L.qk_residual_conv_check.argtypes = conv_args
    L.qk_layer_collapse.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + conv_args
    L.qk_layer_collapse_check.argtypes = conv_args
    ray_args = [ctypes.c_int32, P(qk_camera), P(qk_camera), ctypes.c_float, ctypes.c_float,
                ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                P(qk_feature_map_inout)]
    L.qk_ray_encoding.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + ray_args
    L.qk_ray_encoding_check.argtypes = ray_args
    up_args = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
               ctypes.c_int32, ctypes.c_int]
    L.qk_upsample2x.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + up_args
    L.qk_upsample2x_check.argtypes = up_args
    dec_args = [P(qk_ldm), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                ctypes.c_float, ctypes.c_void_p]
    L.qk_ldm_decode.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + dec_args
    L.qk_ldm_decode_check.argtypes = dec_args
    lg_args = [P(qk_ldm), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.qk_ldm_decode_logits.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + lg_args
    L.qk_ldm_decode_logits_check.argtypes = lg_args
    for name in ("qk_context_create", "qk_context_destroy", "qk_context_weights_static", "qk_update_fuse",
                 "qk_update_fuse_noalloc", "qk_batch_update_fuse", "qk_batch_update_fuse_check", "qk_update_fuse_check", "qk_update_fuse_backward",
                 "qk_update_fuse_backward_check", "qk_ldm_init", "qk_composite",
                 "qk_composite_backward", "qk_composite_backward_check", "qk_render_ibr",
                 "qk_render_ibr_check", "qk_render_to_views",
                 "qk_render_to_views_check", "qk_residual_conv", "qk_residual_conv_check",
                 "qk_layer_collapse", "qk_layer_collapse_check", "qk_ray_encoding",
                 "qk_ray_encoding_check", "qk_upsample2x", "qk_upsample2x_check",
                 "qk_ldm_decode", "qk_ldm_decode_check", "qk_ldm_decode_logits",
                 "qk_ldm_decode_logits_check", "qk_camera_tables"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int):
    if st != QK_OK:
        raise QuarkError(st, load().qk_last_error().decode())


def version() -> str:
    return load().qk_version().decode()


# --------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------

def make_camera(cam) -> qk_camera:
    c = qk_camera()
    K = np.ascontiguousarray(cam.K, dtype=np.float64).reshape(9)
    E = np.ascontiguousarray(cam.E, dtype=np.float64).reshape(16)
    for i in range(9):
        c.K[i] = float(K[i])
    for i in range(16):
        c.E[i] = float(E[i])
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _fmap(f) -> "qk_feature_map":
    """One view's feature map [H][W][C] (its dtype and C as the tensor has
    them; the library checks them against the call's precision and
    weights)."""
    return qk_feature_map(_ptr(f), _dtype_code(f), int(f.shape[0]), int(f.shape[1]),
                          int(f.shape[2]) if len(f.shape) > 2 else 0)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.bfloat16:
        return QK_BF16
    if t.dtype == torch.float32:
        return QK_F32
    return 99


def make_ldm(F, depth, alpha) -> qk_ldm:
    """F: [L][H][W][C] (float32 or bfloat16) or None; depth, alpha: [L][H][W] float32
    (either may be None where the call allows it; the grid comes from the others)."""
    ref = depth if depth is not None else alpha
    L, H, W = (int(s) for s in (ref.shape if ref is not None else F.shape[:3]))
    C = int(F.shape[-1]) if F is not None else 0
    return qk_ldm(_ptr(F), _ptr(depth), _ptr(alpha), L, H, W, C,
                  _dtype_code(F) if F is not None else QK_F32)


def make_weights(w: Dict, heads: int = 1, head_dim: Optional[int] = None) -> qk_weights:
    C = int(w["Wq"].shape[0])
    Cf = int(w["Wk"].shape[0])
    hd = int(w["Wq"].shape[1])
    head_dim = hd // heads if head_dim is None else head_dim
    return qk_weights(_ptr(w["Wq"]), _ptr(w["Wk"]), _ptr(w["Wv"]), _ptr(w["Wo"]),
                      _ptr(w["w_sigma"]), _ptr(w["w_depth"]), _ptr(w["W_color"]), C, Cf, heads,
                      head_dim)


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Context:
    """A libquark context bound to one device."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        """workspace_bytes: cap on the context's device workspaces (0: none)."""
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.qk_context_create(int(device), int(workspace_bytes), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def weights_static(self, enable: bool = True):
        """Declare the weight masters static (qk_context_weights_static): the
        context keeps the copies it derives from them; calling it again
        drops them (after a device synchronisation)."""
        _check(self._lib.qk_context_weights_static(self.handle, 1 if enable else 0))

    def close(self):
        if self.handle:
            self._lib.qk_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _uf_args(in_cams, feats, novel, near, far, weights, precision, attn_form, mode, ldm_in,
             ldm_out, rgb_out, acc_out, blend_out=None):
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    fm = (qk_feature_map * V)(*[_fmap(f)
                                 for f in feats])
    nov = make_camera(novel)
    wts = weights if isinstance(weights, qk_weights) else make_weights(weights)
    lin = ldm_in if isinstance(ldm_in, qk_ldm) else make_ldm(*ldm_in)
    lout = ldm_out if isinstance(ldm_out, qk_ldm) else make_ldm(*ldm_out)
    if not lout.F:                   # F' not written: channel count and dtype follow the input
        lout.C, lout.dtype = lin.C, lin.dtype
    keep = (cams, fm, nov, wts, lin, lout)
    args = [V, cams, fm, ctypes.byref(nov), float(near), float(far), ctypes.byref(wts),
            PREC[precision] if isinstance(precision, str) else int(precision),
            ATTN[attn_form] if isinstance(attn_form, str) else int(attn_form),
            MODE[mode] if isinstance(mode, str) else int(mode),
            ctypes.byref(lin), ctypes.byref(lout), _ptr(rgb_out), _ptr(acc_out),
            _ptr(blend_out)]
    return args, keep


def update_fuse(ctx: Context, in_cams, feats, novel, near, far, weights, ldm_in, ldm_out, *,
                precision="fp32", attn_form="standard", mode="residual", rgb_out=None,
                acc_out=None, blend_logit_out=None, stream=None):
    """qk_update_fuse.  ``ldm_in``/``ldm_out`` are (F, depth, alpha) tuples of
    device tensors (or prebuilt qk_ldm); ``feats`` a list of [Hf][Wf][C]
    device tensors; ``weights`` a dict of float32 device tensors;
    ``blend_logit_out`` an optional [L][H][W][V] float32 tensor."""
    args, keep = _uf_args(in_cams, feats, novel, near, far, weights, precision, attn_form, mode,
                          ldm_in, ldm_out, rgb_out, acc_out, blend_logit_out)
    _check(ctx._lib.qk_update_fuse(ctx.handle, _stream_handle(stream), *args))


def update_fuse_noalloc(ctx: Context, in_cams, feats, novel, near, far, weights, ldm_in, ldm_out,
                        *, precision="fp32", attn_form="standard", mode="residual", rgb_out=None,
                        acc_out=None, blend_logit_out=None, stream=None):
    """qk_update_fuse_noalloc: qk_update_fuse with the device's fixed scratch
    instead of allocated workspaces (same arguments as ``update_fuse``)."""
    args, keep = _uf_args(in_cams, feats, novel, near, far, weights, precision, attn_form, mode,
                          ldm_in, ldm_out, rgb_out, acc_out, blend_logit_out)
    _check(ctx._lib.qk_update_fuse_noalloc(ctx.handle, _stream_handle(stream), *args))


def update_fuse_check(in_cams, feats, novel, near, far, weights, ldm_in, ldm_out, *,
                      precision="fp32", attn_form="standard", mode="residual", rgb_out=None,
                      acc_out=None, blend_logit_out=None) -> int:
    """qk_update_fuse_check: the status qk_update_fuse would return (no device use)."""
    args, keep = _uf_args(in_cams, feats, novel, near, far, weights, precision, attn_form, mode,
                          ldm_in, ldm_out, rgb_out, acc_out, blend_logit_out)
    return int(load().qk_update_fuse_check(*args))


class Request:
    """One request of a batched Update & Fuse: the keyword arguments of
    ``update_fuse`` for one level (precision and attention form are the
    batch's)."""

    def __init__(self, in_cams, feats, novel, near, far, weights, ldm_in, ldm_out, *,
                 mode="residual", rgb_out=None, acc_out=None, blend_logit_out=None):
        V = len(in_cams)
        self.cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
        self.fm = (qk_feature_map * V)(*[_fmap(f) for f in feats])
        self.nov = make_camera(novel)
        self.wts = weights if isinstance(weights, qk_weights) else make_weights(weights)
        self.lin = ldm_in if isinstance(ldm_in, qk_ldm) else make_ldm(*ldm_in)
        self.lout = ldm_out if isinstance(ldm_out, qk_ldm) else make_ldm(*ldm_out)
        if not self.lout.F:
            self.lout.C, self.lout.dtype = self.lin.C, self.lin.dtype
        self.desc = qk_request_desc(
            V, ctypes.addressof(self.cams), ctypes.addressof(self.fm),
            ctypes.addressof(self.nov), float(near), float(far), ctypes.addressof(self.wts),
            MODE[mode] if isinstance(mode, str) else int(mode), ctypes.addressof(self.lin),
            ctypes.addressof(self.lout), _ptr(rgb_out), _ptr(acc_out), _ptr(blend_logit_out))


def _batch_args(requests, precision, attn_form):
    arr = (qk_request_desc * len(requests))(*[r.desc for r in requests])
    return (len(requests), arr, PREC[precision] if isinstance(precision, str) else int(precision),
            ATTN[attn_form] if isinstance(attn_form, str) else int(attn_form)), arr


def batch_update_fuse(ctx: Context, requests, *, precision="bf16", attn_form="standard",
                      stream=None):
    """qk_batch_update_fuse: ``requests`` a list of ``Request``; one launch."""
    args, keep = _batch_args(requests, precision, attn_form)
    _check(ctx._lib.qk_batch_update_fuse(ctx.handle, _stream_handle(stream), *args))


def batch_update_fuse_check(requests, *, precision="bf16", attn_form="standard") -> int:
    args, keep = _batch_args(requests, precision, attn_form)
    return int(load().qk_batch_update_fuse_check(*args))


WEIGHT_NAMES = ("Wq", "Wk", "Wv", "Wo", "w_sigma", "w_depth", "W_color")


def make_weight_grads(dw: Dict) -> qk_weight_grads:
    return qk_weight_grads(*[_ptr(dw[k]) for k in WEIGHT_NAMES])


def _bwd_args(in_cams, feats, novel, near, far, weights, mode, ldm_in, ldm_out, d_rgb, d_out,
              d_in, d_feats, d_weights):
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    fm = (qk_feature_map * V)(*[_fmap(f)
                                 for f in feats])
    nov = make_camera(novel)
    wts = weights if isinstance(weights, qk_weights) else make_weights(weights)
    lin = ldm_in if isinstance(ldm_in, qk_ldm) else make_ldm(*ldm_in)
    lout = None
    if ldm_out is not None:
        lout = ldm_out if isinstance(ldm_out, qk_ldm) else make_ldm(*ldm_out)
    dout = None
    if d_out is not None:
        dout = d_out if isinstance(d_out, qk_ldm) else _grad_ldm(lin, *d_out)
    din = d_in if isinstance(d_in, qk_ldm) else make_ldm(*d_in)
    dfe = (ctypes.c_void_p * V)(*[_ptr(t) for t in d_feats])
    dw = d_weights if isinstance(d_weights, qk_weight_grads) else make_weight_grads(d_weights)
    keep = (cams, fm, nov, wts, lin, lout, dout, din, dfe, dw)
    args = [V, cams, fm, ctypes.byref(nov), float(near), float(far), ctypes.byref(wts),
            MODE[mode] if isinstance(mode, str) else int(mode), ctypes.byref(lin),
            ctypes.byref(lout) if lout is not None else None, _ptr(d_rgb),
            ctypes.byref(dout) if dout is not None else None, ctypes.byref(din), dfe,
            ctypes.byref(dw)]
    return args, keep


def _grad_ldm(like: qk_ldm, dF, d_depth, d_alpha) -> qk_ldm:
    """An LDM of upstream gradients; any of the three may be None (zero)."""
    return qk_ldm(_ptr(dF), _ptr(d_depth), _ptr(d_alpha), like.L, like.H, like.W, like.C, QK_F32)


def update_fuse_backward(ctx: Context, in_cams, feats, novel, near, far, weights, ldm_in,
                         ldm_out, d_in, d_feats, d_weights, *, d_rgb=None, d_out=None,
                         mode="residual", stream=None):
    """qk_update_fuse_backward.  ``ldm_in``/``ldm_out`` are the forward's (F,
    depth, alpha) input and output tuples; ``d_out`` an optional (dF', ddepth',
    dalpha') tuple whose entries may be None; ``d_in`` the (dF, ddepth, dalpha)
    tuple written; ``d_feats`` a list of [Hf][Wf][C] float32 tensors and
    ``d_weights`` a dict with the keys of the weights, both written."""
    args, keep = _bwd_args(in_cams, feats, novel, near, far, weights, mode, ldm_in, ldm_out,
                           d_rgb, d_out, d_in, d_feats, d_weights)
    _check(ctx._lib.qk_update_fuse_backward(ctx.handle, _stream_handle(stream), *args))


def update_fuse_backward_check(in_cams, feats, novel, near, far, weights, ldm_in, ldm_out, d_in,
                               d_feats, d_weights, *, d_rgb=None, d_out=None,
                               mode="residual") -> int:
    """qk_update_fuse_backward_check: the status the backward would return."""
    args, keep = _bwd_args(in_cams, feats, novel, near, far, weights, mode, ldm_in, ldm_out,
                           d_rgb, d_out, d_in, d_feats, d_weights)
    return int(load().qk_update_fuse_backward_check(*args))


def ldm_init(ctx: Context, f0, near, far, ldm, stream=None):
    """qk_ldm_init: fill ``ldm`` = (F, depth, alpha) with the learned
    initialisation (f0 broadcast, layers at their anchors, alpha 1/2)."""
    l = ldm if isinstance(ldm, qk_ldm) else make_ldm(*ldm)
    _check(ctx._lib.qk_ldm_init(ctx.handle, _stream_handle(stream), _ptr(f0), float(near),
                                float(far), ctypes.byref(l)))


def composite(ctx: Context, color, alpha, rgb_out, acc_out=None, stream=None):
    L, H, W = (int(s) for s in alpha.shape)
    _check(ctx._lib.qk_composite(ctx.handle, _stream_handle(stream), L, H, W, _ptr(color),
                                 _ptr(alpha), _ptr(rgb_out), _ptr(acc_out)))


def _cb_args(color, alpha, d_rgb, d_acc, d_color, d_alpha):
    L, H, W = (int(s) for s in alpha.shape)
    return (L, H, W, _ptr(color), _ptr(alpha), _ptr(d_rgb), _ptr(d_acc), _ptr(d_color),
            _ptr(d_alpha))


def composite_backward(ctx: Context, color, alpha, d_rgb, d_alpha, d_color=None, d_acc=None,
                       stream=None):
    """qk_composite_backward: color [L][H][W][3], alpha [L][H][W], d_rgb
    [H][W][3] (and d_acc [H][W] or None) float32 device tensors ->
    d_color [L][H][W][3] (or None), d_alpha [L][H][W]."""
    _check(ctx._lib.qk_composite_backward(ctx.handle, _stream_handle(stream),
                                          *_cb_args(color, alpha, d_rgb, d_acc, d_color, d_alpha)))


def composite_backward_check(color, alpha, d_rgb, d_alpha, d_color=None, d_acc=None) -> int:
    return int(load().qk_composite_backward_check(*_cb_args(color, alpha, d_rgb, d_acc, d_color,
                                                            d_alpha)))


def _render_args(in_cams, images, novel, near, far, logits, H, W, rgb_out, acc_out, depth_out):
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    imgs = (qk_image * V)(*[qk_image(_ptr(im), int(im.shape[0]), int(im.shape[1]))
                            for im in images])
    dl, sl, bl = logits
    L, h, w = (int(s) for s in dl.shape)
    lg = qk_ldm_logits(_ptr(dl), _ptr(sl), _ptr(bl), L, h, w,
                       int(bl.shape[3]) if len(bl.shape) == 4 else -1)
    nov = make_camera(novel)
    args = (V, cams, imgs, ctypes.byref(nov), ctypes.c_float(near), ctypes.c_float(far),
            ctypes.byref(lg), int(H), int(W), _ptr(rgb_out), _ptr(acc_out), _ptr(depth_out))
    return args, (cams, imgs, lg, nov)


def render_ibr(ctx: Context, in_cams, images, novel, near, far, logits, rgb_out, *,
               acc_out=None, depth_out=None, stream=None):
    """qk_render_ibr: images are RGBA8 device tensors [Hi][Wi][4] (uint8);
    logits = (depth_logit [L][h][w], sigma_logit [L][h][w],
    blend_logit [L][h][w][V]) float32; rgb_out [H][W][3] float32 sets the
    output grid."""
    H, W = int(rgb_out.shape[0]), int(rgb_out.shape[1])
    args, keep = _render_args(in_cams, images, novel, near, far, logits, H, W, rgb_out, acc_out,
                              depth_out)
    _check(ctx._lib.qk_render_ibr(ctx.handle, _stream_handle(stream), *args))


def render_ibr_check(in_cams, images, novel, near, far, logits, H, W, rgb_out, *, acc_out=None,
                     depth_out=None) -> int:
    """qk_render_ibr_check: the status qk_render_ibr would return (no device use)."""
    args, keep = _render_args(in_cams, images, novel, near, far, logits, H, W, rgb_out, acc_out,
                              depth_out)
    return int(load().qk_render_ibr_check(*args))


def _views_args(in_cams, novel, depth, alpha, color, rgb_outs, acc_outs):
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    L, H, W = (int(s) for s in depth.shape)
    ld = qk_ldm_decoded(_ptr(depth), _ptr(alpha), _ptr(color), L, H, W)
    accs = [None] * V if acc_outs is None else list(acc_outs)
    views = (qk_view_image * V)(*[qk_view_image(_ptr(r), _ptr(a), int(r.shape[0]), int(r.shape[1]))
                                  for r, a in zip(rgb_outs, accs)])
    nov = make_camera(novel)
    return (V, cams, ctypes.byref(nov), ctypes.byref(ld), views), (cams, ld, views, nov)


def render_to_views(ctx: Context, in_cams, novel, depth, alpha, color, rgb_outs, acc_outs=None,
                    stream=None):
    """qk_render_to_views: depth, alpha [L][H][W], color [L][H][W][3] float32
    device tensors; rgb_outs[m] [Hm][Wm][3] (sets view m's grid), acc_outs[m]
    [Hm][Wm] or None."""
    args, keep = _views_args(in_cams, novel, depth, alpha, color, rgb_outs, acc_outs)
    _check(ctx._lib.qk_render_to_views(ctx.handle, _stream_handle(stream), *args))


def render_to_views_check(in_cams, novel, depth, alpha, color, rgb_outs, acc_outs=None) -> int:
    """qk_render_to_views_check: the status qk_render_to_views would return."""
    args, keep = _views_args(in_cams, novel, depth, alpha, color, rgb_outs, acc_outs)
    return int(load().qk_render_to_views_check(*args))


def _volume(F) -> qk_ldm:
    L, H, W, C = (int(s) for s in F.shape)
    return qk_ldm(_ptr(F), None, None, L, H, W, C, _dtype_code(F))


def residual_conv(ctx: Context, F_in, W1, W2, F_out, stream=None):
    """qk_residual_conv: F_out = F_in + W2 * gelu(W1 * N(F_in)) per layer;
    F_in, F_out [L][H][W][32] bfloat16 device tensors, W1, W2 [3][3][32][32]
    float32."""
    a, b = _volume(F_in), _volume(F_out)
    _check(ctx._lib.qk_residual_conv(ctx.handle, _stream_handle(stream), ctypes.byref(a),
                                     _ptr(W1), _ptr(W2), ctypes.byref(b)))


def residual_conv_check(F_in, W1, W2, F_out) -> int:
    a, b = _volume(F_in), _volume(F_out)
    return int(load().qk_residual_conv_check(ctypes.byref(a), _ptr(W1), _ptr(W2), ctypes.byref(b)))


def layer_collapse(ctx: Context, F_in, W1, W2, F_out, stream=None):
    """qk_layer_collapse: F_out[j] = (F_in[2j] + F_in[2j+1]) / 2 +
    relu([F_in[2j], F_in[2j+1]] W1) W2; bfloat16 device tensors
    [L][H][W][32] -> [L/2][H][W][32], W1 [64][32], W2 [32][32] float32."""
    a, b = _volume(F_in), _volume(F_out)
    _check(ctx._lib.qk_layer_collapse(ctx.handle, _stream_handle(stream), ctypes.byref(a),
                                      _ptr(W1), _ptr(W2), ctypes.byref(b)))


def layer_collapse_check(F_in, W1, W2, F_out) -> int:
    a, b = _volume(F_in), _volume(F_out)
    return int(load().qk_layer_collapse_check(ctypes.byref(a), _ptr(W1), _ptr(W2),
                                              ctypes.byref(b)))


def _ray_args(in_cams, novel, near, far, Wr, feats, low_hw, src=None):
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    srcs = [None] * len(feats) if src is None else list(src)
    if len(srcs) != len(feats):
        raise ValueError("src needs one map per feature map")
    for f, s_ in zip(feats, srcs):
        if s_ is not None and (tuple(s_.shape) != tuple(f.shape) or s_.dtype != f.dtype):
            raise ValueError("a source map needs its feature map's shape and dtype")
    maps = (qk_feature_map_inout * V)(*[qk_feature_map_inout(_ptr(f), int(f.shape[0]),
                                                             int(f.shape[1]), _ptr(s))
                                        for f, s in zip(feats, srcs)])
    nov = make_camera(novel)
    C = int(Wr.shape[1]) if Wr is not None else 0
    lh, lw = (0, 0) if low_hw is None else (int(low_hw[0]), int(low_hw[1]))
    return ((V, cams, ctypes.byref(nov), float(near), float(far), _ptr(Wr), C,
             _dtype_code(feats[0]), lh, lw, maps), (cams, maps, nov))


def ray_encoding(ctx: Context, in_cams, novel, near: float, far: float, Wr, feats, low_hw=None,
                 stream=None, src=None):
    """qk_ray_encoding: adds each view's ray-direction encoding to its
    feature map; Wr [32][C] float32, feats[m] [Hf][Wf][C] float32 or
    bfloat16 device tensors (one dtype); low_hw = (h, w) evaluates the
    encoding on that grid and upsamples it (the paper's form), None per
    pixel.  src (optional, one per map, entries may be None): the maps read,
    the encoded result going to feats; without it the maps are encoded in
    place."""
    args, keep = _ray_args(in_cams, novel, near, far, Wr, feats, low_hw, src)
    _check(ctx._lib.qk_ray_encoding(ctx.handle, _stream_handle(stream), *args))


def ray_encoding_check(in_cams, novel, near: float, far: float, Wr, feats, low_hw=None,
                       src=None) -> int:
    """qk_ray_encoding_check: the status qk_ray_encoding would return."""
    args, keep = _ray_args(in_cams, novel, near, far, Wr, feats, low_hw, src)
    return int(load().qk_ray_encoding_check(*args))


def _up_args(src, dst):
    shape = tuple(int(d) for d in src.shape)
    N, H, W, C = shape if len(shape) == 4 else (1,) + shape
    return (_ptr(src), _ptr(dst), N, H, W, C, _dtype_code(src))


def upsample2x(ctx: Context, src, dst, stream=None):
    """qk_upsample2x: src [N][H][W][C] (or [H][W][C]) -> dst [N][2H][2W][C],
    float32 or bfloat16 device tensors."""
    _check(ctx._lib.qk_upsample2x(ctx.handle, _stream_handle(stream), *_up_args(src, dst)))


def upsample2x_check(src, dst) -> int:
    return int(load().qk_upsample2x_check(*_up_args(src, dst)))


def _dec_args(F, depth, alpha, w_sigma, w_depth, W_color, near, far, color_out):
    L, H, W, C = (int(d) for d in F.shape)
    ldm = qk_ldm(_ptr(F), _ptr(depth), _ptr(alpha), L, H, W, C, _dtype_code(F))
    return (ctypes.byref(ldm), _ptr(w_sigma), _ptr(w_depth), _ptr(W_color), float(near),
            float(far), _ptr(color_out)), ldm


def ldm_decode(ctx: Context, F, depth, alpha, w_sigma, w_depth, W_color, near: float, far: float,
               color_out=None, stream=None):
    """qk_ldm_decode: F [L][H][W][C] float32 / bfloat16 -> depth, alpha
    [L][H][W] (and color_out [L][H][W][3] if given), the absolute decode."""
    args, keep = _dec_args(F, depth, alpha, w_sigma, w_depth, W_color, near, far, color_out)
    _check(ctx._lib.qk_ldm_decode(ctx.handle, _stream_handle(stream), *args))


def ldm_decode_check(F, depth, alpha, w_sigma, w_depth, W_color, near, far, color_out=None) -> int:
    args, keep = _dec_args(F, depth, alpha, w_sigma, w_depth, W_color, near, far, color_out)
    return int(load().qk_ldm_decode_check(*args))


def _lg_args(F, w_sigma, w_depth, depth_logit, sigma_logit):
    L, H, W, C = (int(d) for d in F.shape)
    ldm = qk_ldm(_ptr(F), None, None, L, H, W, C, _dtype_code(F))
    return (ctypes.byref(ldm), _ptr(w_sigma), _ptr(w_depth), _ptr(depth_logit),
            _ptr(sigma_logit)), ldm


def ldm_logits(ctx: Context, F, w_sigma, w_depth, depth_logit, sigma_logit, stream=None):
    """qk_ldm_decode_logits: F [L][H][W][C] float32 / bfloat16 -> the unactivated
    depth_logit, sigma_logit [L][H][W] float32 (the render's inputs)."""
    args, keep = _lg_args(F, w_sigma, w_depth, depth_logit, sigma_logit)
    _check(ctx._lib.qk_ldm_decode_logits(ctx.handle, _stream_handle(stream), *args))


def ldm_logits_check(F, w_sigma, w_depth, depth_logit, sigma_logit) -> int:
    args, keep = _lg_args(F, w_sigma, w_depth, depth_logit, sigma_logit)
    return int(load().qk_ldm_decode_logits_check(*args))


def camera_tables(in_cams, feat_hw: Sequence, novel, H: int, W: int) -> np.ndarray:
    """qk_camera_tables: per-view [12] = A (3x3 row-major) then b, in double."""
    V = len(in_cams)
    cams = (qk_camera * V)(*[make_camera(c) for c in in_cams])
    hw = np.ascontiguousarray(feat_hw, dtype=np.int32).reshape(V, 2)
    out = np.zeros((V, 12))
    nov = make_camera(novel)
    _check(load().qk_camera_tables(V, cams, hw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   ctypes.byref(nov), int(H), int(W),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out
