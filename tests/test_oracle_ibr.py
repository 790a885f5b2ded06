"""Pins of the oracle's final render (upsample & activate, blend-weight
image-based render; Sec. 3.1 Eq. 1 and Sec. 3.2.3).

Each function is checked against something other than itself: the
library's bilinear resampler (torch interpolate), closed forms of the
activation, invariants of the blend (identical views, one-hot weights,
identity camera), and an independent float64 re-implementation of the whole
render from torch primitives (interpolate, grid_sample, softmax)."""

import math

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import synth

torch = pytest.importorskip("torch")
Fn = torch.nn.functional


def _interp(a: np.ndarray, H: int, W: int) -> np.ndarray:
    """torch's bilinear resize (half-pixel centres, align_corners=False) of
    a [h][w] or [h][w][C] array."""
    t = torch.from_numpy(np.asarray(a, dtype=np.float64))
    if t.ndim == 2:
        return Fn.interpolate(t[None, None], size=(H, W), mode="bilinear",
                              align_corners=False)[0, 0].numpy()
    out = Fn.interpolate(t.permute(2, 0, 1)[None], size=(H, W), mode="bilinear",
                         align_corners=False)[0]
    return out.permute(1, 2, 0).numpy()


@pytest.mark.parametrize("shape", [((12, 20), (24, 40)), ((5, 7), (15, 21)), ((5, 13), (13, 29)),
                                   ((1, 1), (3, 4)), ((9, 6), (9, 6)), ((2, 3), (7, 11))])
def test_upsample_matches_torch(shape):
    (h, w), (H, W) = shape
    rng = np.random.default_rng(h * 100 + w)
    src = rng.standard_normal((h, w, 3))
    got = oracle.upsample_bilinear(src, H, W)
    ref = _interp(src, H, W)
    assert np.max(np.abs(got - ref)) < 1e-12
    got1 = oracle.upsample_bilinear(src[..., 0], H, W)
    assert np.max(np.abs(got1 - ref[..., 0])) < 1e-12


def test_upsample_identity_and_affine():
    rng = np.random.default_rng(3)
    src = rng.standard_normal((6, 9, 2))
    assert np.array_equal(oracle.upsample_bilinear(src, 6, 9), src)
    # an affine field sampled at pixel centres is reproduced exactly away
    # from the border (where the border value extends outward)
    h, w, H, W = 8, 10, 24, 30
    yy, xx = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    aff = 0.3 * xx - 1.7 * yy + 0.25
    up = oracle.upsample_bilinear(aff, H, W)
    YY, XX = np.meshgrid((np.arange(H) + 0.5) * h / H, (np.arange(W) + 0.5) * w / W, indexing="ij")
    inner = (XX >= 0.5) & (XX <= w - 0.5) & (YY >= 0.5) & (YY <= h - 0.5)
    assert np.max(np.abs(up - (0.3 * XX - 1.7 * YY + 0.25))[inner]) < 1e-12


def test_activation_closed_forms():
    near, far, L = 0.5, 20.0, 4
    band = 1 / near - 1 / far
    xb = np.array([0.3, -1.2, 2.0])
    for li in range(L):
        lp = L - li
        d, s, beta = oracle.ibr_activate(0.0, 0.0, xb, li, L, near, far)
        # x_d = 0 puts the layer at its anchor disparity (lp - 0.5)/L of the band
        assert d == pytest.approx(1.0 / ((lp - 0.5) / L * band + 1 / far), rel=1e-14)
        assert s == pytest.approx(0.5, abs=1e-15)
        e = np.exp(xb - xb.max())
        assert np.allclose(beta, e / e.sum(), rtol=1e-14)
        # saturated tanh reaches the band's edges: the bands tile [1/far, 1/near]
        d_hi, _, _ = oracle.ibr_activate(40.0, 0.0, xb, li, L, near, far)
        d_lo, _, _ = oracle.ibr_activate(-40.0, 0.0, xb, li, L, near, far)
        assert 1 / d_hi == pytest.approx(lp / L * band + 1 / far, rel=1e-14)
        assert 1 / d_lo == pytest.approx((lp - 1) / L * band + 1 / far, rel=1e-14)
    _, s, beta = oracle.ibr_activate(0.0, 1.3, np.zeros(5), 0, L, near, far)
    assert s == pytest.approx(1 / (1 + math.exp(-1.3)), rel=1e-15)
    assert np.allclose(beta, 0.2, rtol=1e-15)
    _, _, b2 = oracle.ibr_activate(0.0, 0.0, xb + 7.5, 0, L, near, far)
    assert np.allclose(b2, beta if False else oracle.ibr_activate(0.0, 0.0, xb, 0, L, near, far)[2],
                       rtol=1e-14)


def _scene(V=3, W=40, H=24, s=2, L=3, img_hw=(30, 50), seed=11):
    return synth.make_render(V=V, W=W, H=H, s=s, L=L, img_hw=img_hw, seed=seed)


def _render(rs, cams=None, images=None, blend=None, **kw):
    cams = rs.in_cams if cams is None else cams
    images = rs.images if images is None else images
    blend = rs.blend_logit if blend is None else blend
    return oracle.render_ibr(cams, images, rs.novel, rs.near, rs.far, rs.depth_logit,
                             rs.sigma_logit, blend, rs.H, rs.W, **kw)


def test_identity_camera_reproduces_the_image():
    """One input image seen from the novel camera itself, on the output
    grid: every pixel reprojects onto its own centre at any depth, so each
    layer's colour is the pixel's colour and rgb = c (1 - prod(1 - sigma))."""
    rs = _scene(V=1, img_hw=(24, 40))
    cam = synth.Camera(rs.novel.K.copy(), rs.novel.E.copy(), rs.novel.width, rs.novel.height)
    out = _render(rs, cams=[cam], want_layers=True)
    img = oracle.image_rgb(rs.images[0])
    sig = 1 / (1 + np.exp(-_interp(np.moveaxis(rs.sigma_logit, 0, -1), rs.H, rs.W)))  # [H][W][L]
    T = np.prod(1 - sig, axis=-1)
    assert np.max(np.abs(out["layer_color"] - img[None])) < 1e-12
    assert np.max(np.abs(out["rgb"] - img * (1 - T)[..., None])) < 1e-12
    assert np.max(np.abs(out["acc"] - (1 - T))) < 1e-12


def test_identical_views_equal_one_view():
    rs = _scene(V=3)
    one = _render(rs, cams=[rs.in_cams[1]] * 1, images=[rs.images[1]],
                  blend=rs.blend_logit[..., 1:2])
    same = _render(rs, cams=[rs.in_cams[1]] * 3, images=[rs.images[1]] * 3)
    for k in ("rgb", "acc", "depth"):
        assert np.max(np.abs(same[k] - one[k])) < 1e-12


def test_one_hot_blend_selects_a_view():
    rs = _scene(V=3)
    bl = np.zeros_like(rs.blend_logit)
    bl[..., 2] = 80.0
    got = _render(rs, blend=bl)
    ref = _render(rs, cams=[rs.in_cams[2]], images=[rs.images[2]], blend=bl[..., 2:3])
    assert np.max(np.abs(got["rgb"] - ref["rgb"])) < 1e-12


def test_layers_composite_to_the_image():
    rs = _scene(V=2, L=4)
    out = _render(rs, want_layers=True)
    sig = 1 / (1 + np.exp(-np.stack([_interp(rs.sigma_logit[l], rs.H, rs.W) for l in range(4)])))
    rgb, acc = oracle.composite(out["layer_color"], sig)
    assert np.max(np.abs(rgb - out["rgb"])) < 1e-12
    assert np.max(np.abs(acc - out["acc"])) < 1e-12


def test_rows_subset_is_exact():
    rs = _scene(V=2)
    full = _render(rs)
    rows = [0, 5, rs.H - 1]
    part = _render(rs, rows=rows)
    assert np.array_equal(part["rgb"], full["rgb"][rows])


def _scaled_K(cam, w1, h1):
    K = cam.K.copy()
    K[0] *= w1 / cam.width
    K[1] *= h1 / cam.height
    K[2] = cam.K[2]
    return torch.from_numpy(K)


def _torch_render(rs):
    """The render written again from torch float64 primitives: interpolate
    for the upsampling, tanh/sigmoid/softmax for the activation, explicit
    K / E matrices for the back-projection, grid_sample (zero padding,
    align_corners=False) for the image sampling, a loop for "over"."""
    f64 = torch.float64
    V, (L, h, w), H, W = rs.V, rs.depth_logit.shape, rs.H, rs.W
    up = lambda a: Fn.interpolate(torch.from_numpy(a.astype(np.float64))[:, None], size=(H, W),
                                  mode="bilinear", align_corners=False)[:, 0]
    xd, xs = up(rs.depth_logit), up(rs.sigma_logit)                       # [L][H][W]
    xb = Fn.interpolate(torch.from_numpy(rs.blend_logit.astype(np.float64)).permute(0, 3, 1, 2),
                        size=(H, W), mode="bilinear", align_corners=False)  # [L][V][H][W]
    band = 1 / rs.near - 1 / rs.far
    lp = L - torch.arange(L, dtype=f64)
    disp = ((lp - 0.5) / L)[:, None, None] + (0.5 / L) * torch.tanh(xd)
    depth = 1 / (disp * band + 1 / rs.far)
    sig = torch.sigmoid(xs)
    beta = torch.softmax(xb, dim=1)
    Kn = _scaled_K(rs.novel, W, H)
    ys, xs_ = torch.meshgrid(torch.arange(H, dtype=f64) + 0.5, torch.arange(W, dtype=f64) + 0.5,
                             indexing="ij")
    pix = torch.stack([xs_, ys, torch.ones_like(xs_)]).reshape(3, -1)
    rays = torch.linalg.inv(Kn) @ pix
    En_inv = torch.linalg.inv(torch.from_numpy(rs.novel.E))
    colour = torch.zeros((L, 3, H, W), dtype=f64)
    for l in range(L):
        d = depth[l].reshape(-1)
        Xn = torch.cat([rays * d, torch.ones(1, H * W, dtype=f64)])
        for m in range(V):
            cam = rs.in_cams[m]
            img = torch.from_numpy(oracle.image_rgb(rs.images[m])).permute(2, 0, 1)[None]
            Hi, Wi = img.shape[2], img.shape[3]
            Xm = torch.from_numpy(cam.E) @ (En_inv @ Xn)
            P = _scaled_K(cam, Wi, Hi) @ Xm[:3]
            valid = Xm[2] > 1e-6 * d
            um, vm = P[0] / P[2], P[1] / P[2]
            g = torch.stack([2 * um / Wi - 1, 2 * vm / Hi - 1], dim=-1)
            g[~valid] = -10.0
            s = Fn.grid_sample(img, g.reshape(1, H, W, 2), mode="bilinear", padding_mode="zeros",
                               align_corners=False)[0]
            colour[l] += beta[l, m] * s
    T = torch.ones((H, W), dtype=f64)
    rgb = torch.zeros((3, H, W), dtype=f64)
    dmap = torch.zeros((H, W), dtype=f64)
    for l in range(L):
        rgb += T * sig[l] * colour[l]
        dmap += T * sig[l] * depth[l]
        T = T * (1 - sig[l])
    return rgb.permute(1, 2, 0).numpy(), (1 - T).numpy(), dmap.numpy()


@pytest.mark.parametrize("kw", [dict(), dict(V=4, s=3, W=45, H=27, L=2, img_hw=(27, 45), seed=4),
                                dict(V=2, W=33, H=17, L=3, img_hw=(40, 60), seed=9)])
def test_render_matches_torch_reimplementation(kw):
    rs = _scene(**kw)
    out = _render(rs)
    rgb, acc, dmap = _torch_render(rs)
    assert np.max(np.abs(out["rgb"] - rgb)) < 1e-10
    assert np.max(np.abs(out["acc"] - acc)) < 1e-12
    assert np.max(np.abs(out["depth"] - dmap)) < 1e-10
    # the rig's samples fall both inside and outside the images
    assert 0.0 < float(np.mean(out["rgb"] > 0)) <= 1.0
