"""C-ABI contract on the CPU: the library loads, exports every symbol the
header declares, composes the camera tables in double exactly like the
oracle's independent 4x4 chain, and rejects bad arguments before touching a
device."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="session", autouse=True)
def built_library():
    if not os.path.exists(lib.LIB_PATH):
        from paper_2411_16680_amd import build
        build.build()
    return lib.load()


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "quark.h")).read()
    declared = sorted(set(re.findall(r"QK_API\s+[\w\s\*]*?\b(qk_\w+)\s*\(", hdr)))
    assert declared, "no declarations found"
    assert sorted(lib.EXPORTS) == declared
    L = lib.load()
    for name in declared:
        assert hasattr(L, name), name
    assert "gfx950" in lib.version()


def _random_rig(seed):
    r = np.random.default_rng(seed)
    sc = synth.make_custom(V=5, H=33, W=47, C=8, L=2, seed=seed, hfov=75.0)
    return sc


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_camera_tables_match_oracle_chain(seed):
    sc = _random_rig(seed)
    H, W = 33, 47
    feat_hw = [(17, 23)] * sc.V          # feature grid differs from the LDM grid
    tab = lib.camera_tables(sc.in_cams, feat_hw, sc.novel, H, W)
    r = np.random.default_rng(seed + 10)
    for m, cam in enumerate(sc.in_cams):
        A = tab[m, :9].reshape(3, 3)
        b = tab[m, 9:]
        Kn = oracle.scale_intrinsics(sc.novel.K, sc.novel.width, sc.novel.height, W, H)
        Km = oracle.scale_intrinsics(cam.K, cam.width, cam.height, 23, 17)
        for _ in range(20):
            u, v, d = r.uniform(0, W), r.uniform(0, H), r.uniform(0.5, 20)
            pz = A[2] @ [u, v, 1] + b[2] / d
            (um, vm), ok = oracle.reproject(Kn, sc.novel.E, Km, cam.E, u, v, d)
            assert ok == (pz > 1e-6)
            if ok:
                px = A[0] @ [u, v, 1] + b[0] / d
                py = A[1] @ [u, v, 1] + b[1] / d
                assert abs(px / pz - um) < 1e-9 and abs(py / pz - vm) < 1e-9


# ---------------------------------------------------------------- validation

class _FakeT:
    """Stands in for a device tensor: only the pointer value and shape are
    read by the argument checks (no device memory is touched)."""

    def __init__(self, shape, addr=0x100000, dtype=None):
        import torch
        self.shape = shape
        self._addr = addr
        self.dtype = dtype or torch.float32

    def data_ptr(self):
        return self._addr


def _args(C=16, L=4, H=12, W=20, V=3, dtype="f32", heads=1, head_dim=None, Cf=None):
    import torch
    sc = synth.make_custom(V=V, H=H, W=W, C=C, L=L, seed=4)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    Cf = C if Cf is None else Cf
    hd = heads * (C if head_dim is None else head_dim)
    feats = [_FakeT((H, W, Cf), 0x200000 + 0x10000 * i, tdt) for i in range(V)]
    F = _FakeT((L, H, W, C), 0x300000, tdt)
    d = _FakeT((L, H, W), 0x400000)
    a = _FakeT((L, H, W), 0x500000)
    w = {"Wq": _FakeT((C, hd), 0x600000), "Wk": _FakeT((Cf, hd), 0x610000),
         "Wv": _FakeT((Cf, hd), 0x620000), "Wo": _FakeT((hd, C), 0x630000),
         "w_sigma": _FakeT((C,), 0x640000), "w_depth": _FakeT((C,), 0x650000),
         "W_color": _FakeT((C, 3), 0x660000)}
    wts = lib.make_weights(w, heads=heads)
    return sc, feats, wts, (F, d, a)


def _check(sc, feats, wts, ldm, **kw):
    return lib.update_fuse_check(sc.in_cams, feats, sc.novel, sc.near, sc.far, wts, ldm, ldm, **kw)


def test_feature_maps_carry_dtype_and_channels():
    """Each map states its dtype and C; one that disagrees with the
    precision's storage type or the weights' C_feat is rejected before any
    launch."""
    import torch
    sc, feats, wts, ldm = _args(C=16, dtype="bf16")
    assert _check(sc, feats, wts, ldm, precision="bf16") == lib.QK_OK
    wrong = list(feats)
    wrong[1] = _FakeT((12, 20, 16), 0x210000, torch.float32)
    assert _check(sc, wrong, wts, ldm, precision="bf16") == lib.QK_EDTYPE
    assert "feature map 1" in lib.load().qk_last_error().decode()
    wrong[1] = _FakeT((12, 20, 8), 0x210000, torch.bfloat16)
    assert _check(sc, wrong, wts, ldm, precision="bf16") == lib.QK_ESHAPE
    assert "C_feat" in lib.load().qk_last_error().decode()
    # float32 maps under a bfloat16 precision, and the reverse
    sc, feats, wts, ldm = _args(C=16)
    assert _check(sc, feats, wts, ldm) == lib.QK_OK
    bf = [_FakeT((12, 20, 16), 0x200000 + 0x10000 * i, torch.bfloat16) for i in range(3)]
    assert _check(sc, bf, wts, ldm) == lib.QK_EDTYPE


def test_valid_arguments_pass():
    for C in (8, 16, 32, 64):
        sc, feats, wts, ldm = _args(C=C)
        assert _check(sc, feats, wts, ldm) == lib.QK_OK
        sc, feats, wts, ldm = _args(C=C, dtype="bf16")
        assert _check(sc, feats, wts, ldm, precision="bf16") == lib.QK_OK
        assert _check(sc, feats, wts, ldm, precision="bf16_fp8proj") == lib.QK_OK
        assert _check(sc, feats, wts, ldm, precision=3) == lib.QK_EINVAL


def test_rejections():
    sc, feats, wts, ldm = _args()
    # precision / dtype mismatch
    assert _check(sc, feats, wts, ldm, precision="bf16") == lib.QK_EDTYPE
    assert _check(sc, feats, wts, ldm, precision="bf16_fp8proj") == lib.QK_EDTYPE
    # unsupported channel count and heads
    sc2, f2, w2, l2 = _args(C=24)
    assert _check(sc2, f2, w2, l2) == lib.QK_EUNSUPPORTED
    sc2, f2, w2, l2 = _args(C=16, heads=2, head_dim=8)
    assert _check(sc2, f2, w2, l2) == lib.QK_EUNSUPPORTED

    # misaligned feature buffer
    F, d, a = ldm
    bad = (_FakeT(F.shape, F._addr + 4), d, a)
    assert _check(sc, feats, wts, bad) == lib.QK_EINVAL
    # NULL weight
    w_null = lib.qk_weights.from_buffer_copy(wts)
    w_null.Wk = None
    assert _check(sc, feats, w_null, ldm) == lib.QK_EINVAL
    # near >= far
    assert lib.update_fuse_check(sc.in_cams, feats, sc.novel, 5.0, 5.0, wts, ldm, ldm) == lib.QK_EINVAL
    # bad camera: K last row
    bad_cam = synth.Camera(sc.novel.K.copy(), sc.novel.E.copy(), sc.novel.width, sc.novel.height)
    bad_cam.K[2, 2] = 2.0
    assert lib.update_fuse_check(sc.in_cams, feats, bad_cam, sc.near, sc.far, wts, ldm,
                                 ldm) == lib.QK_EINVAL
    # out LDM with different dims
    out = (_FakeT((2, 12, 20, 16), 0x700000), _FakeT((2, 12, 20), 0x710000),
           _FakeT((2, 12, 20), 0x720000))
    assert lib.update_fuse_check(sc.in_cams, feats, sc.novel, sc.near, sc.far, wts, ldm,
                                 out) == lib.QK_ESHAPE
    # a feature map of 1 GiB or more (float32: 4096 x 4096 x 16) is refused,
    # one just under it passes
    big = list(feats)
    big[1] = _FakeT((4096, 4096, 16), feats[1]._addr)
    assert _check(sc, big, wts, ldm) == lib.QK_EUNSUPPORTED
    assert "1 GiB" in lib.load().qk_last_error().decode()
    big[1] = _FakeT((4095, 4096, 16), feats[1]._addr)
    assert _check(sc, big, wts, ldm) == lib.QK_OK
    # acc without rgb
    assert _check(sc, feats, wts, ldm, acc_out=_FakeT((12, 20))) == lib.QK_EINVAL
    msg = lib.load().qk_last_error().decode()
    assert "rgb" in msg



def test_heads():
    """Several heads at C >= 32 with heads x head_dim == C and head_dim 16,
    32 (or 8 at C = 32); the folded form at C = 32 without e4m3 projections."""
    for C, heads, hd in ((32, 4, 8), (32, 2, 16), (64, 4, 16), (64, 2, 32), (32, 1, 32)):
        sc, f, w, l = _args(C=C, heads=heads, head_dim=hd)
        assert _check(sc, f, w, l) == lib.QK_OK, (C, heads, hd)
        sc, f, w, l = _args(C=C, heads=heads, head_dim=hd, dtype="bf16")
        assert _check(sc, f, w, l, precision="bf16") == lib.QK_OK
        assert _check(sc, f, w, l, precision="bf16_fp8proj") == lib.QK_OK
    for C, heads, hd in ((64, 8, 8), (32, 4, 16), (32, 2, 8), (16, 2, 8), (8, 2, 4)):
        sc, f, w, l = _args(C=C, heads=heads, head_dim=hd)
        assert _check(sc, f, w, l) == lib.QK_EUNSUPPORTED, (C, heads, hd)
    # the folded form of several heads: C = 32, not with e4m3 projections
    sc, f, w, l = _args(C=32, heads=4, head_dim=8)
    assert _check(sc, f, w, l, attn_form="folded") == lib.QK_OK
    sc, f, w, l = _args(C=32, heads=2, head_dim=16, dtype="bf16")
    assert _check(sc, f, w, l, attn_form="folded", precision="bf16") == lib.QK_OK
    assert _check(sc, f, w, l, attn_form="folded", precision="bf16_fp8proj") == lib.QK_EUNSUPPORTED
    sc, f, w, l = _args(C=64, heads=4, head_dim=16)
    assert _check(sc, f, w, l, attn_form="folded") == lib.QK_EUNSUPPORTED
    assert "folded" in lib.load().qk_last_error().decode()


def test_blend_logit_output_checks():
    sc, feats, wts, ldm = _args(C=32, L=2, H=6, W=10, V=3)
    bl = _FakeT((2, 6, 10, 3), 0x800000)
    assert _check(sc, feats, wts, ldm, blend_logit_out=bl) == lib.QK_OK
    assert _check(sc, feats, wts, ldm, blend_logit_out=_FakeT((2, 6, 10, 3), 0x800002)) == \
        lib.QK_EINVAL
    sc, f, w, l = _args(C=32, heads=4, head_dim=8, L=2, H=6, W=10, V=3)
    assert _check(sc, f, w, l, blend_logit_out=bl) == lib.QK_EUNSUPPORTED
    assert "one attention head" in lib.load().qk_last_error().decode()


def test_ldm_decode_logits_checks():
    import torch
    F = _FakeT((4, 5, 6, 32), 0x300000, torch.bfloat16)
    ws, wd = _FakeT((32,), 0x500000), _FakeT((32,), 0x510000)
    dl, sl = _FakeT((4, 5, 6), 0x400000), _FakeT((4, 5, 6), 0x410000)
    assert lib.ldm_logits_check(F, ws, wd, dl, sl) == lib.QK_OK
    assert lib.ldm_logits_check(F, ws, wd, None, sl) == lib.QK_EINVAL
    assert lib.ldm_logits_check(F, ws, wd, dl, _FakeT((4, 5, 6), 0x400000 + 64)) == lib.QK_EINVAL
    assert "overlaps" in lib.load().qk_last_error().decode()
    assert lib.ldm_logits_check(_FakeT((4, 5, 6, 24), 0x300000), ws, wd, dl, sl) == \
        lib.QK_EUNSUPPORTED
    assert lib.ldm_logits_check(_FakeT((4, 5, 6, 32), 0x300000, torch.float16), ws, wd, dl,
                                sl) == lib.QK_EDTYPE


def test_null_context_rejected_before_device_use():
    sc, feats, wts, ldm = _args()
    args, keep = lib._uf_args(sc.in_cams, feats, sc.novel, sc.near, sc.far, wts, "fp32",
                              "standard", "residual", ldm, ldm, None, None)
    assert lib.load().qk_update_fuse(None, None, *args) == lib.QK_EINVAL
    assert lib.load().qk_composite(None, None, 1, 1, 1, None, None, None, None) == lib.QK_EINVAL


def test_context_create_without_gpu_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = lib.load().qk_context_create(0, 0, ctypes.byref(h))
    assert st in (lib.QK_EHIP, lib.QK_EINVAL)
    with pytest.raises(lib.QuarkError):
        lib.Context(0)


# ------------------------------------------------------- backward validation

def _bwd_check(sc, feats, wts, ldm, *, C=16, L=4, H=12, W=20, d_rgb=True, dfe=None, d_in=None,
               ldm_out=True, mode="residual"):
    V = len(feats)
    dfe = dfe if dfe is not None else [_FakeT(f.shape, 0x800000 + 0x10000 * i)
                                       for i, f in enumerate(feats)]
    d_in = d_in if d_in is not None else (_FakeT((L, H, W, C), 0x900000),
                                          _FakeT((L, H, W), 0x910000),
                                          _FakeT((L, H, W), 0x920000))
    dw = {k: _FakeT((1,), 0xa00000 + 0x1000 * i) for i, k in enumerate(lib.WEIGHT_NAMES)}
    out = ldm if ldm_out else None
    return lib.update_fuse_backward_check(sc.in_cams, feats, sc.novel, sc.near, sc.far, wts, ldm,
                                          out, d_in, dfe, dw,
                                          d_rgb=_FakeT((H, W, 3), 0xb00000) if d_rgb else None,
                                          mode=mode)


def test_backward_valid_arguments_pass():
    for C in (8, 16):
        sc, feats, wts, ldm = _args(C=C)
        assert _bwd_check(sc, feats, wts, ldm, C=C) == lib.QK_OK
        assert _bwd_check(sc, feats, wts, ldm, C=C, d_rgb=False, ldm_out=False) == lib.QK_OK
        assert _bwd_check(sc, feats, wts, ldm, C=C, mode="paper") == lib.QK_OK


def test_backward_rejections():
    sc, feats, wts, ldm = _args(C=32)
    assert _bwd_check(sc, feats, wts, ldm, C=32) == lib.QK_EUNSUPPORTED
    sc, feats, wts, ldm = _args(C=16, dtype="bf16")
    assert _bwd_check(sc, feats, wts, ldm) == lib.QK_EDTYPE
    sc, feats, wts, ldm = _args(C=16)
    # d_rgb needs the forward's outputs
    assert _bwd_check(sc, feats, wts, ldm, ldm_out=False) == lib.QK_EINVAL
    # misaligned feature-map gradient
    dfe = [_FakeT(f.shape, 0x800004 + 0x10000 * i) for i, f in enumerate(feats)]
    assert _bwd_check(sc, feats, wts, ldm, dfe=dfe) == lib.QK_EINVAL
    # NULL gradient output
    d_in = (_FakeT((4, 12, 20, 16), 0x900000), None, _FakeT((4, 12, 20), 0x920000))
    assert _bwd_check(sc, feats, wts, ldm, d_in=d_in) == lib.QK_EINVAL
    # gradient LDM with other dims
    d_in = (_FakeT((4, 12, 21, 16), 0x900000), _FakeT((4, 12, 21), 0x910000),
            _FakeT((4, 12, 21), 0x920000))
    assert _bwd_check(sc, feats, wts, ldm, d_in=d_in) == lib.QK_ESHAPE
    # several heads
    sc, feats, wts, ldm = _args(C=16, heads=2, head_dim=8)
    assert _bwd_check(sc, feats, wts, ldm) == lib.QK_EUNSUPPORTED


def test_backward_null_context_rejected():
    sc, feats, wts, ldm = _args()
    dfe = [_FakeT(f.shape, 0x800000 + 0x10000 * i) for i, f in enumerate(feats)]
    dw = {k: _FakeT((1,), 0xa00000 + 0x1000 * i) for i, k in enumerate(lib.WEIGHT_NAMES)}
    d_in = (_FakeT((4, 12, 20, 16), 0x900000), _FakeT((4, 12, 20), 0x910000),
            _FakeT((4, 12, 20), 0x920000))
    args, keep = lib._bwd_args(sc.in_cams, feats, sc.novel, sc.near, sc.far, wts, "residual", ldm,
                               ldm, None, None, d_in, dfe, dw)
    assert lib.load().qk_update_fuse_backward(None, None, *args) == lib.QK_EINVAL


def _render_args(V=3, L=2, h=6, w=10, H=12, W=20, Hi=14, Wi=22):
    import torch
    rs = synth.make_render(V=V, W=W, H=H, L=L, lowres_hw=(h, w), img_hw=(Hi, Wi), seed=2)
    imgs = [_FakeT((Hi, Wi, 4), 0x200000 + 0x10000 * i, torch.uint8) for i in range(V)]
    lg = (_FakeT((L, h, w), 0x300000), _FakeT((L, h, w), 0x310000),
          _FakeT((L, h, w, V), 0x320000))
    rgb = _FakeT((H, W, 3), 0x400000)
    return rs, imgs, lg, rgb


def _rcheck(rs, imgs, lg, rgb, near=None, far=None, **kw):
    return lib.render_ibr_check(rs.in_cams, imgs, rs.novel, rs.near if near is None else near,
                                rs.far if far is None else far, lg, rgb.shape[0], rgb.shape[1],
                                rgb, **kw)


def test_render_valid_arguments_pass():
    rs, imgs, lg, rgb = _render_args()
    assert _rcheck(rs, imgs, lg, rgb) == lib.QK_OK
    assert _rcheck(rs, imgs, lg, rgb, acc_out=_FakeT((12, 20), 0x500000),
                   depth_out=_FakeT((12, 20), 0x510000)) == lib.QK_OK


def test_render_rejections():
    rs, imgs, lg, rgb = _render_args()
    # blend logits for another number of views
    bad = (lg[0], lg[1], _FakeT((2, 6, 10, 4), 0x320000))
    assert _rcheck(rs, imgs, bad, rgb) == lib.QK_ESHAPE
    # misaligned image, NULL logit, misaligned output
    im2 = list(imgs)
    im2[1] = _FakeT(imgs[1].shape, imgs[1]._addr + 2, imgs[1].dtype)
    assert _rcheck(rs, im2, lg, rgb) == lib.QK_EINVAL
    assert "aligned" in lib.load().qk_last_error().decode()
    assert _rcheck(rs, imgs, (lg[0], None, lg[2]), rgb) == lib.QK_EINVAL
    assert _rcheck(rs, imgs, lg, _FakeT((12, 20, 3), 0x400002)) == lib.QK_EINVAL
    # near >= far
    assert _rcheck(rs, imgs, lg, rgb, near=3.0, far=3.0) == lib.QK_EINVAL
    # an image of 1 GiB (16384 x 16384 RGBA8) is refused
    im3 = list(imgs)
    im3[0] = _FakeT((16384, 16384, 4), imgs[0]._addr)
    assert _rcheck(rs, im3, lg, rgb) == lib.QK_EUNSUPPORTED
    # non-positive output grid
    assert lib.render_ibr_check(rs.in_cams, imgs, rs.novel, rs.near, rs.far, lg, 0, 20,
                                rgb) == lib.QK_ESHAPE
    # more than 16 views
    rs17, imgs17, lg17, rgb17 = _render_args(V=17)
    assert _rcheck(rs17, imgs17, lg17, rgb17) == lib.QK_ESHAPE


def test_render_null_context_rejected_before_device_use():
    rs, imgs, lg, rgb = _render_args()
    args, keep = lib._render_args(rs.in_cams, imgs, rs.novel, rs.near, rs.far, lg, 12, 20, rgb,
                                  None, None)
    assert lib.load().qk_render_ibr(None, None, *args) == lib.QK_EINVAL


def _views_args(V=3, L=2, H=12, W=20, Hm=14, Wm=22):
    vs = synth.make_views(V=V, W=W, H=H, L=L, view_hw=(Hm, Wm), seed=2)
    d, a = _FakeT((L, H, W), 0x300000), _FakeT((L, H, W), 0x310000)
    c = _FakeT((L, H, W, 3), 0x320000)
    rgbs = [_FakeT((Hm, Wm, 3), 0x400000 + 0x10000 * m) for m in range(V)]
    return vs, d, a, c, rgbs


def test_views_valid_arguments_pass():
    vs, d, a, c, rgbs = _views_args()
    assert lib.render_to_views_check(vs.in_cams, vs.novel, d, a, c, rgbs) == lib.QK_OK
    accs = [_FakeT((14, 22), 0x500000 + 0x10000 * m) for m in range(3)]
    assert lib.render_to_views_check(vs.in_cams, vs.novel, d, a, c, rgbs, accs) == lib.QK_OK


def test_views_rejections():
    vs, d, a, c, rgbs = _views_args()
    # misaligned LDM buffer, NULL colour, misaligned output
    assert lib.render_to_views_check(vs.in_cams, vs.novel, _FakeT(d.shape, d._addr + 2), a, c,
                                     rgbs) == lib.QK_EINVAL
    assert lib.render_to_views_check(vs.in_cams, vs.novel, d, a, None, rgbs) == lib.QK_EINVAL
    bad = list(rgbs)
    bad[2] = _FakeT(rgbs[2].shape, rgbs[2]._addr + 1)
    assert lib.render_to_views_check(vs.in_cams, vs.novel, d, a, c, bad) == lib.QK_EINVAL
    # empty view grid
    bad[2] = _FakeT((0, 22, 3), rgbs[2]._addr)
    assert lib.render_to_views_check(vs.in_cams, vs.novel, d, a, c, bad) == lib.QK_ESHAPE
    # projected planes of 2^31 floats: 8 layers x 8192 x 8192 x 4
    vs8, d8, a8, c8, _ = _views_args(V=1, L=8)
    huge = [_FakeT((8192, 8192, 3), 0x400000)]
    assert lib.render_to_views_check(vs8.in_cams[:1], vs8.novel, d8, a8, c8,
                                     huge) == lib.QK_EUNSUPPORTED
    # 17 views
    vs17, d17, a17, c17, r17 = _views_args(V=17)
    assert lib.render_to_views_check(vs17.in_cams, vs17.novel, d17, a17, c17,
                                     r17) == lib.QK_ESHAPE


def test_views_null_context_rejected_before_device_use():
    vs, d, a, c, rgbs = _views_args()
    args, keep = lib._views_args(vs.in_cams, vs.novel, d, a, c, rgbs, None)
    assert lib.load().qk_render_to_views(None, None, *args) == lib.QK_EINVAL


def test_residual_conv_checks():
    import torch
    F = _FakeT((2, 9, 13, 32), 0x300000, torch.bfloat16)
    out = _FakeT((2, 9, 13, 32), 0x900000, torch.bfloat16)
    W1, W2 = _FakeT((3, 3, 32, 32), 0x600000), _FakeT((3, 3, 32, 32), 0x610000)
    assert lib.residual_conv_check(F, W1, W2, out) == lib.QK_OK
    # C other than 32, float32 volume, differing dims, overlap, misalignment, NULL
    assert lib.residual_conv_check(_FakeT((2, 9, 13, 16), 0x300000, torch.bfloat16), W1, W2,
                                   _FakeT((2, 9, 13, 16), 0x900000, torch.bfloat16)) == lib.QK_EUNSUPPORTED
    assert lib.residual_conv_check(_FakeT((2, 9, 13, 32), 0x300000), W1, W2,
                                   _FakeT((2, 9, 13, 32), 0x900000)) == lib.QK_EDTYPE
    assert lib.residual_conv_check(F, W1, W2, _FakeT((2, 9, 12, 32), 0x900000,
                                                     torch.bfloat16)) == lib.QK_ESHAPE
    assert lib.residual_conv_check(F, W1, W2, _FakeT((2, 9, 13, 32), 0x300000 + 64,
                                                     torch.bfloat16)) == lib.QK_EINVAL
    assert "overlap" in lib.load().qk_last_error().decode()
    assert lib.residual_conv_check(_FakeT((2, 9, 13, 32), 0x300008, torch.bfloat16), W1, W2,
                                   out) == lib.QK_EINVAL
    assert lib.residual_conv_check(F, None, W2, out) == lib.QK_EINVAL


def test_layer_collapse_checks():
    import torch
    F = _FakeT((4, 9, 13, 32), 0x300000, torch.bfloat16)
    out = _FakeT((2, 9, 13, 32), 0x900000, torch.bfloat16)
    W1, W2 = _FakeT((64, 32), 0x600000), _FakeT((32, 32), 0x610000)
    assert lib.layer_collapse_check(F, W1, W2, out) == lib.QK_OK
    assert lib.layer_collapse_check(_FakeT((3, 9, 13, 32), 0x300000, torch.bfloat16), W1, W2,
                                    out) == lib.QK_ESHAPE
    assert "even" in lib.load().qk_last_error().decode()
    assert lib.layer_collapse_check(F, W1, W2, _FakeT((4, 9, 13, 32), 0x900000,
                                                      torch.bfloat16)) == lib.QK_ESHAPE
    assert lib.layer_collapse_check(_FakeT((4, 9, 13, 16), 0x300000, torch.bfloat16), W1, W2,
                                    _FakeT((2, 9, 13, 16), 0x900000, torch.bfloat16)) == lib.QK_EUNSUPPORTED
    assert lib.layer_collapse_check(F, W1, W2, _FakeT((2, 9, 13, 32), 0x300000 + 4096,
                                                      torch.bfloat16)) == lib.QK_EINVAL
    assert lib.layer_collapse_check(F, None, W2, out) == lib.QK_EINVAL


def test_ray_encoding_checks():
    import torch
    sc = synth.make_custom(V=3, H=12, W=20, C=16, L=2, seed=4)
    cams, nov = sc.in_cams, sc.novel
    Wr = _FakeT((32, 16), 0x600000)
    feats = [_FakeT((9, 13, 16), 0x100000 * (m + 1)) for m in range(3)]
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats) == lib.QK_OK
    bf = [_FakeT((9, 13, 16), 0x100000 * (m + 1), torch.bfloat16) for m in range(3)]
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, bf) == lib.QK_OK
    assert lib.ray_encoding_check(cams, nov, 0.5, 0.5, Wr, feats) == lib.QK_EINVAL
    assert lib.ray_encoding_check(cams, nov, 0.0, 20.0, Wr, feats) == lib.QK_EINVAL
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, _FakeT((32, 12), 0x600000),
                                  feats) == lib.QK_EUNSUPPORTED
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, _FakeT((32, 16), 0x600004),
                                  feats) == lib.QK_EINVAL
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr,
                                  [_FakeT((9, 13, 16), 0x100000, torch.float16)] * 3) == lib.QK_EDTYPE
    # overlapping maps race (each is written in place)
    ov = [feats[0], _FakeT((9, 13, 16), 0x100000 + 64), feats[2]]
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, ov) == lib.QK_EINVAL
    assert "overlap" in lib.load().qk_last_error().decode()
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr,
                                  [feats[0], _FakeT((0, 13, 16), 0x200000), feats[2]]) == lib.QK_ESHAPE
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr,
                                  [feats[0], _FakeT((9, 13, 16), 0x200008), feats[2]]) == lib.QK_EINVAL
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, None, feats) == lib.QK_EINVAL
    assert lib.ray_encoding_check(cams * 6, nov, 0.5, 20.0, Wr, feats * 6) == lib.QK_ESHAPE
    # the low-resolution form: both sides positive, or both 0
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, low_hw=(5, 7)) == lib.QK_OK
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, low_hw=(0, 7)) == lib.QK_ESHAPE
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, low_hw=(-1, -1)) == lib.QK_ESHAPE
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats,
                                  low_hw=(1 << 14, 1 << 14)) == lib.QK_EUNSUPPORTED
    # out of place: a source map is read, the encoded map written to data;
    # it may be the map itself, or any buffer that overlaps no map written
    srcs = [_FakeT((9, 13, 16), 0x1000000 * (m + 1)) for m in range(3)]
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, src=srcs) == lib.QK_OK
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats,
                                  src=[feats[0], None, srcs[2]]) == lib.QK_OK
    # two sources may share memory (both only read)
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats,
                                  src=[srcs[0], srcs[0], srcs[0]]) == lib.QK_OK
    for bad in ([srcs[0], feats[0], srcs[2]],                        # another view's map
                [_FakeT((9, 13, 16), 0x100000 + 64), None, None]):   # its own map, shifted
        assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, src=bad) == lib.QK_EINVAL
        assert "source map" in lib.load().qk_last_error().decode()
    assert lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats,
                                  src=[_FakeT((9, 13, 16), 0x1000008), None, None]) == lib.QK_EINVAL
    with pytest.raises(ValueError):
        lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats, src=srcs[:2])
    with pytest.raises(ValueError):
        lib.ray_encoding_check(cams, nov, 0.5, 20.0, Wr, feats,
                               src=[_FakeT((9, 12, 16), 0x1000000), None, None])


def test_upsample2x_and_decode_checks():
    import torch
    src = _FakeT((2, 5, 7, 8), 0x100000)
    dst = _FakeT((2, 10, 14, 8), 0x200000)
    assert lib.upsample2x_check(src, dst) == lib.QK_OK
    assert lib.upsample2x_check(_FakeT((2, 5, 7, 3), 0x100004), _FakeT((2, 10, 14, 3), 0x200000)) == lib.QK_OK
    assert lib.upsample2x_check(_FakeT((2, 5, 7, 8), 0x100004), dst) == lib.QK_EINVAL
    assert lib.upsample2x_check(src, _FakeT((2, 10, 14, 8), 0x100000 + 64)) == lib.QK_EINVAL
    assert "overlap" in lib.load().qk_last_error().decode()
    assert lib.upsample2x_check(_FakeT((0, 5, 7, 8), 0x100000), dst) == lib.QK_ESHAPE
    assert lib.upsample2x_check(_FakeT((2, 5, 7, 8), 0x100000, torch.float16), dst) == lib.QK_EDTYPE
    F = _FakeT((4, 5, 6, 32), 0x300000, torch.bfloat16)
    d, a = _FakeT((4, 5, 6), 0x400000), _FakeT((4, 5, 6), 0x410000)
    ws, wd, wc = _FakeT((32,), 0x500000), _FakeT((32,), 0x510000), _FakeT((32, 3), 0x520000)
    assert lib.ldm_decode_check(F, d, a, ws, wd, wc, 0.5, 20.0) == lib.QK_OK
    assert lib.ldm_decode_check(F, d, a, ws, wd, wc, 0.5, 20.0, color_out=_FakeT((4, 5, 6, 3), 0x600000)) == lib.QK_OK
    assert lib.ldm_decode_check(_FakeT((4, 5, 6, 24), 0x300000), d, a, ws, wd, wc, 0.5, 20.0) == lib.QK_EUNSUPPORTED
    assert lib.ldm_decode_check(F, d, a, ws, wd, wc, 2.0, 1.0) == lib.QK_EINVAL
    assert lib.ldm_decode_check(F, None, a, ws, wd, wc, 0.5, 20.0) == lib.QK_EINVAL
    assert lib.ldm_decode_check(_FakeT((4, 5, 6, 32), 0x300008), d, a, ws, wd, wc, 0.5, 20.0) == lib.QK_EINVAL


def test_composite_backward_checks():
    c, a = _FakeT((3, 4, 5, 3), 0x100000), _FakeT((3, 4, 5), 0x200000)
    g, gA = _FakeT((4, 5, 3), 0x300000), _FakeT((4, 5), 0x310000)
    dc, da = _FakeT((3, 4, 5, 3), 0x400000), _FakeT((3, 4, 5), 0x500000)
    assert lib.composite_backward_check(c, a, g, da, dc, gA) == lib.QK_OK
    assert lib.composite_backward_check(c, a, g, da) == lib.QK_OK         # d_color, d_acc NULL
    assert lib.composite_backward_check(c, a, None, da) == lib.QK_EINVAL
    assert lib.composite_backward_check(c, a, g, None) == lib.QK_EINVAL
    assert lib.composite_backward_check(c, _FakeT((0, 4, 5), 0x200000), g, da) == lib.QK_ESHAPE
    assert lib.composite_backward_check(c, a, _FakeT((4, 5, 3), 0x300002), da) == lib.QK_EINVAL
    # an output on top of an input, or on the other output
    assert lib.composite_backward_check(c, a, g, _FakeT((3, 4, 5), 0x200000 + 16)) == lib.QK_EINVAL
    assert "overlap" in lib.load().qk_last_error().decode()
    assert lib.composite_backward_check(c, a, g, da, _FakeT((3, 4, 5, 3), 0x500000 - 64)) == lib.QK_EINVAL


def test_composite_backward_null_context_rejected():
    import torch
    t3 = torch.zeros((2, 3, 4, 3))
    t1 = torch.zeros((2, 3, 4))
    st = lib.load().qk_composite_backward(None, None, *lib._cb_args(t3, t1, torch.zeros(3, 4, 3),
                                                                    None, None, t1))
    assert st == lib.QK_EINVAL


def test_batch_update_fuse_checks():
    reqs = []
    for i, (H, W, V) in enumerate(((6, 10, 3), (4, 21, 2), (5, 7, 4))):
        sc, f, w, l = _args(C=32, L=2, H=H, W=W, V=V, dtype="bf16")
        reqs.append(lib.Request(sc.in_cams, f, sc.novel, sc.near, sc.far, w, l, l))
    assert lib.batch_update_fuse_check(reqs) == lib.QK_OK
    assert lib.batch_update_fuse_check(reqs, attn_form="folded") == lib.QK_OK
    assert lib.batch_update_fuse_check(reqs, precision="fp32") == lib.QK_EUNSUPPORTED
    assert lib.batch_update_fuse_check([]) == lib.QK_ESHAPE
    assert lib.batch_update_fuse_check(reqs * 22) == lib.QK_ESHAPE          # 66 > 64
    # a request of another width
    sc, f, w, l = _args(C=16, L=2, H=6, W=10, V=3, dtype="bf16")
    assert lib.batch_update_fuse_check(reqs + [lib.Request(sc.in_cams, f, sc.novel, sc.near,
                                                           sc.far, w, l, l)]) == \
        lib.QK_EUNSUPPORTED
    # a bad request is named by its index
    sc, f, w, l = _args(C=32, L=2, H=6, W=10, V=3, dtype="bf16")
    bad = lib.Request(sc.in_cams, f, sc.novel, 5.0, 5.0, w, l, l)
    assert lib.batch_update_fuse_check(reqs[:2] + [bad]) == lib.QK_EINVAL
    assert "request 2" in lib.load().qk_last_error().decode()
    assert lib.load().qk_batch_update_fuse(None, None, *lib._batch_args(reqs, "bf16",
                                                                        "standard")[0]) == \
        lib.QK_EINVAL
