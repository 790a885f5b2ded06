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
