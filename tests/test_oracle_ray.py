"""Pins of the oracle's ray-direction encoding: a view that is the novel
camera itself gives a zero difference vector everywhere; a view translated
sideways in the novel camera's frame gives the constant difference
(2 f / W)(1/far - 1/near) t_x; one moved along the optical axis gives the
pixel-linear difference -(2 / W)(1/far - 1/near) t_z (u - c_x); and the
sinusoid octaves take their closed-form values at tanh(delta) = 1/2."""

import math

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import synth


def _rig():
    sc = synth.make_custom(V=2, H=18, W=32, C=8, L=1, seed=5)
    return sc.novel


def _moved(novel, t):
    """The novel camera translated by t (its own frame)."""
    E = novel.E.copy()
    R = E[:3, :3]
    c = -R.T @ E[:3, 3] + R.T @ np.asarray(t, dtype=np.float64)
    E[:3, 3] = -R @ c
    return synth.Camera(novel.K.copy(), E, novel.width, novel.height)


NEAR, FAR = 0.5, 20.0


def test_aligned_view_gives_zero_difference():
    nov = _rig()
    Wr = np.random.default_rng(1).standard_normal((32, 16))
    out, dl = oracle.ray_encoding(nov, nov, NEAR, FAR, Wr, 9, 16, want_delta=True)
    assert np.max(np.abs(dl)) < 1e-12
    e0 = np.tile([0.0, 1.0, 0.0, 1.0], 8)
    assert np.max(np.abs(out - e0 @ Wr)) < 1e-12


def test_sideways_translation_gives_a_constant_difference():
    nov = _rig()
    tx = 0.07
    cam = _moved(nov, (tx, 0.0, 0.0))
    _, dl = oracle.ray_encoding(cam, nov, NEAR, FAR, np.zeros((32, 4)), nov.height, nov.width,
                                want_delta=True)
    f = nov.K[0, 0]
    assert np.max(np.abs(dl[..., 0] - 2 * f / nov.width * tx * (1 / FAR - 1 / NEAR))) < 1e-12
    assert np.max(np.abs(dl[..., 1])) < 1e-12


def test_axial_translation_gives_a_pixel_linear_difference():
    nov = _rig()
    tz = -0.2
    cam = _moved(nov, (0.0, 0.0, tz))
    H, W = nov.height, nov.width
    _, dl = oracle.ray_encoding(cam, nov, NEAR, FAR, np.zeros((32, 4)), H, W, want_delta=True)
    u = np.arange(W) + 0.5
    v = np.arange(H) + 0.5
    k = 1 / FAR - 1 / NEAR
    ex = -(2.0 / W) * k * tz * (u - nov.K[0, 2])
    ey = -(2.0 / H) * k * tz * (v - nov.K[1, 2])
    assert np.max(np.abs(dl[..., 0] - ex[None, :])) < 1e-12
    assert np.max(np.abs(dl[..., 1] - ey[:, None])) < 1e-12


def test_octaves_at_one_half():
    """tanh(delta_x) = 1/2, delta_y = 0, identity projection (C = 32)."""
    nov = _rig()
    f = nov.K[0, 0]
    tx = math.atanh(0.5) / (2 * f / nov.width * (1 / FAR - 1 / NEAR))
    cam = _moved(nov, (tx, 0.0, 0.0))
    out = oracle.ray_encoding(cam, nov, NEAR, FAR, np.eye(32), 3, 5)
    e = np.zeros(32)
    for k in range(8):
        e[4 * k + 0] = 1.0 if k == 0 else 0.0          # sin(2^k pi / 2)
        e[4 * k + 1] = 0.0 if k == 0 else (-1.0 if k == 1 else 1.0)
        e[4 * k + 2] = 0.0
        e[4 * k + 3] = 1.0
    assert np.max(np.abs(out - e)) < 1e-12


def test_lowres_form_on_the_map_grid_is_the_per_pixel_form():
    """Upsampling from a grid to itself is the identity, so the paper's
    low-resolution form on the map's own grid is the per-pixel encoding."""
    sc = synth.make_ray(V=3, W=64, H=36, levels=((1, 16),), seed=2)
    for cam in sc.in_cams:
        a = oracle.ray_encoding(cam, sc.novel, NEAR, FAR, sc.Wr[0], 18, 32)
        b = oracle.ray_encoding_lowres(cam, sc.novel, NEAR, FAR, sc.Wr[0], (18, 32), 18, 32)
        assert np.max(np.abs(a - b)) < 1e-12


def test_lowres_form_of_a_constant_difference_is_that_constant():
    """A sideways translation gives one difference vector everywhere; its
    upsampled encoding is the per-pixel one at any grid."""
    nov = _rig()
    cam = _moved(nov, (0.05, 0.0, 0.0))
    Wr = np.random.default_rng(3).standard_normal((32, 8))
    a = oracle.ray_encoding(cam, nov, NEAR, FAR, Wr, 27, 48)
    b = oracle.ray_encoding_lowres(cam, nov, NEAR, FAR, Wr, (4, 7), 27, 48)
    assert np.max(np.abs(a - b)) < 1e-12
    assert np.max(np.abs(a - a[0, 0])) < 1e-12


def test_lowres_form_interpolates_between_low_res_centres():
    """At a map pixel whose centre falls midway between two low-res centres
    (an exact 2x upsampling: the map's second pixel sits at low-res
    coordinate 0.25, its third at 0.75) the result is the bilinear mix of
    the per-pixel encodings evaluated at those low-res centres."""
    sc = synth.make_ray(V=2, W=64, H=36, levels=((1, 8),), seed=8)
    cam, Wr = sc.in_cams[1], sc.Wr[0]
    lo = oracle.ray_encoding(cam, sc.novel, NEAR, FAR, Wr, 9, 16)
    up = oracle.ray_encoding_lowres(cam, sc.novel, NEAR, FAR, Wr, (9, 16), 18, 32)
    # map pixel (y=3, x=5) sits at low-res (1.25, 2.25) -> weights 3/4, 1/4
    ref = (0.75 * (0.75 * lo[1, 2] + 0.25 * lo[1, 3]) + 0.25 * (0.75 * lo[2, 2] + 0.25 * lo[2, 3]))
    assert np.max(np.abs(up[3, 5] - ref)) < 1e-12
