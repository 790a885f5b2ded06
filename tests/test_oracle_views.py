"""Pins of the oracle's render to input views (Sec. 3.2.2, Eq. 2): the
projection operator P_theta (a bilinear splat) and the per-view composite.

P_theta is pinned as the adjoint of the already pinned back-projection
(reprojection + bilinear sampling): <P x, y> = <x, P^T y> for random x, y.
The render is pinned by an identity-camera closed form (each layer-pixel
lands on its own pixel, so the render is the layers' composite), by mass
conservation of the splat, and by an independent float64 re-implementation
from torch primitives (index_add for the splat, a loop for "over")."""

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import synth

torch = pytest.importorskip("torch")


def _T(novel, cam, H, W, Hm, Wm):
    Kn = oracle.scale_intrinsics(novel.K, novel.width, novel.height, W, H)
    Km = oracle.scale_intrinsics(cam.K, cam.width, cam.height, Wm, Hm)
    return oracle.reprojection_matrix(Kn, novel.E, Km, cam.E)


def _scene(**kw):
    base = dict(V=3, W=36, H=20, L=3, seed=21)
    base.update(kw)
    return synth.make_views(**base)


@pytest.mark.parametrize("kw", [dict(), dict(view_hw=(15, 27)), dict(view_hw=(31, 50), seed=5),
                                dict(arc=4.0, hfov=140.0, seed=9)])
def test_splat_is_the_adjoint_of_sampling(kw):
    vs = _scene(**kw)
    rng = np.random.default_rng(2)
    H, W = vs.depth.shape[1:]
    Hm, Wm = vs.view_hw[0]
    T = _T(vs.novel, vs.in_cams[1], H, W, Hm, Wm)
    x = rng.standard_normal((H, W))
    y = rng.standard_normal((Hm, Wm))
    d = vs.depth[1].astype(np.float64)
    Px = oracle.splat_layer(T, d, x, Hm, Wm)
    # P^T y: sample y at every layer-pixel's projection (the pinned sampling)
    Pty = np.zeros((H, W))
    n_out = 0
    for yy in range(H):
        for xx in range(W):
            uv = np.zeros(2)
            ok = oracle.lib().or_reproject_T(oracle._d(np.ascontiguousarray(T.reshape(16))),
                                             oracle.ctypes.c_double(xx + 0.5),
                                             oracle.ctypes.c_double(yy + 0.5),
                                             oracle.ctypes.c_double(d[yy, xx]), oracle._d(uv))
            if ok == 1:
                Pty[yy, xx] = oracle.bilinear(y[..., None], uv[0], uv[1])[0]
            else:
                n_out += 1
    lhs, rhs = float(np.sum(Px * y)), float(np.sum(x * Pty))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_identity_camera_render_is_the_composite():
    vs = _scene(V=1)
    nov = vs.novel
    cam = synth.Camera(nov.K.copy(), nov.E.copy(), nov.width, nov.height)
    out = oracle.render_to_views([cam], nov, vs.depth, vs.alpha, vs.color, [vs.depth.shape[1:]])
    rgb, acc = oracle.composite(vs.color, vs.alpha)
    assert np.max(np.abs(out["img"][0] - rgb)) < 1e-12
    assert np.max(np.abs(out["acc"][0] - acc)) < 1e-12


def test_splat_conserves_mass_inside_the_view():
    """Bilinear weights sum to one, so a splat whose every tap lands inside
    the view keeps the layer's total: the novel camera itself on a grid twice
    as fine (every point falls between four pixel centres), and on the same
    grid (every point on its own centre)."""
    vs = _scene(V=1)
    H, W = vs.depth.shape[1:]
    nov = vs.novel
    x = np.random.default_rng(4).uniform(size=(H, W))
    for k in (1, 2):
        T = _T(nov, nov, H, W, k * H, k * W)
        Px = oracle.splat_layer(T, vs.depth[0], x, k * H, k * W)
        assert abs(Px.sum() - x.sum()) < 1e-10 * x.sum()
    assert np.allclose(oracle.splat_layer(_T(nov, nov, H, W, H, W), vs.depth[0], x, H, W), x,
                       atol=1e-12)


def _torch_render(vs):
    f64 = torch.float64
    L, H, W = vs.depth.shape
    outs = []
    for m, cam in enumerate(vs.in_cams):
        Hm, Wm = vs.view_hw[m]
        Kn = torch.from_numpy(oracle.scale_intrinsics(vs.novel.K, vs.novel.width,
                                                      vs.novel.height, W, H))
        Km = torch.from_numpy(oracle.scale_intrinsics(cam.K, cam.width, cam.height, Wm, Hm))
        ys, xs = torch.meshgrid(torch.arange(H, dtype=f64) + 0.5, torch.arange(W, dtype=f64) + 0.5,
                                indexing="ij")
        pix = torch.stack([xs, ys, torch.ones_like(xs)]).reshape(3, -1)
        rays = torch.linalg.inv(Kn) @ pix
        En_inv = torch.linalg.inv(torch.from_numpy(vs.novel.E))
        Tr = torch.ones(Hm * Wm, dtype=f64)
        img = torch.zeros(Hm * Wm, 3, dtype=f64)
        for l in range(L):
            d = torch.from_numpy(vs.depth[l].astype(np.float64)).reshape(-1)
            Xn = torch.cat([rays * d, torch.ones(1, H * W, dtype=f64)])
            Xm = torch.from_numpy(cam.E) @ (En_inv @ Xn)
            P = Km @ Xm[:3]
            valid = Xm[2] > 1e-6 * d
            fx_, fy_ = P[0] / P[2] - 0.5, P[1] / P[2] - 0.5
            x0, y0 = torch.floor(fx_), torch.floor(fy_)
            fx, fy = fx_ - x0, fy_ - y0
            vals = torch.cat([torch.from_numpy(vs.color[l].astype(np.float64)).reshape(-1, 3),
                              torch.from_numpy(vs.alpha[l].astype(np.float64)).reshape(-1, 1)], 1)
            acc = torch.zeros(Hm * Wm, 4, dtype=f64)
            for tx, ty, w in ((x0, y0, (1 - fx) * (1 - fy)), (x0 + 1, y0, fx * (1 - fy)),
                              (x0, y0 + 1, (1 - fx) * fy), (x0 + 1, y0 + 1, fx * fy)):
                inside = valid & (tx >= 0) & (tx < Wm) & (ty >= 0) & (ty < Hm)
                idx = (ty[inside] * Wm + tx[inside]).long()
                acc.index_add_(0, idx, vals[inside] * w[inside, None])
            img += (Tr * acc[:, 3])[:, None] * acc[:, :3]
            Tr = Tr * (1 - acc[:, 3])
        outs.append((img.reshape(Hm, Wm, 3).numpy(), (1 - Tr).reshape(Hm, Wm).numpy()))
    return outs


@pytest.mark.parametrize("kw", [dict(), dict(view_hw=(17, 29), L=4, seed=3),
                                dict(arc=4.0, hfov=140.0, seed=9)])
def test_render_matches_torch_reimplementation(kw):
    vs = _scene(**kw)
    out = oracle.render_to_views(vs.in_cams, vs.novel, vs.depth, vs.alpha, vs.color, vs.view_hw)
    ref = _torch_render(vs)
    for m in range(vs.V):
        assert np.max(np.abs(out["img"][m] - ref[m][0])) < 1e-10
        assert np.max(np.abs(out["acc"][m] - ref[m][1])) < 1e-10
    # splats overlap: some view pixels receive more than one layer-pixel
    assert max(float(np.max(a)) for a in out["acc"]) > 0.0
