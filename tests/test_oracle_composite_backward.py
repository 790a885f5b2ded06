"""Pins of the oracle's composite adjoint (Sec. 3.1, the over operator O,
differentiated by the chain rule): central differences of the oracle's own
forward composite, and closed forms for one layer, an opaque front layer and
fully transparent layers."""

import numpy as np

import oracle

RNG = np.random.default_rng(2024)


def _fd(color, alpha, g, gA, h=1e-6):
    """Central differences of <g, rgb> + <gA, acc> in every colour and alpha."""
    def loss(c, a):
        rgb, acc = oracle.composite(c, a)
        return float(np.sum(g * rgb) + np.sum(gA * acc))
    dc = np.zeros_like(color)
    da = np.zeros_like(alpha)
    for idx in np.ndindex(color.shape):
        cp, cm = color.copy(), color.copy()
        cp[idx] += h; cm[idx] -= h
        dc[idx] = (loss(cp, alpha) - loss(cm, alpha)) / (2 * h)
    for idx in np.ndindex(alpha.shape):
        ap, am = alpha.copy(), alpha.copy()
        ap[idx] += h; am[idx] -= h
        da[idx] = (loss(color, ap) - loss(color, am)) / (2 * h)
    return dc, da


def test_composite_backward_central_differences():
    L, n = 5, 7
    color = RNG.uniform(0, 1, (L, n, 3))
    alpha = RNG.uniform(0.05, 0.95, (L, n))
    g = RNG.standard_normal((n, 3))
    gA = RNG.standard_normal(n)
    dc, da = oracle.composite_backward(color, alpha, g, gA)
    dc_fd, da_fd = _fd(color, alpha, g, gA)
    np.testing.assert_allclose(dc, dc_fd, atol=1e-8)
    np.testing.assert_allclose(da, da_fd, atol=1e-8)
    # without d_acc the accumulated-alpha term is absent
    dc0, da0 = oracle.composite_backward(color, alpha, g)
    dc_fd0, da_fd0 = _fd(color, alpha, g, np.zeros(n))
    np.testing.assert_allclose(dc0, dc_fd0, atol=1e-8)
    np.testing.assert_allclose(da0, da_fd0, atol=1e-8)


def test_composite_backward_one_layer_closed_form():
    n = 11
    color = RNG.uniform(0, 1, (1, n, 3)); alpha = RNG.uniform(0, 1, (1, n))
    g = RNG.standard_normal((n, 3)); gA = RNG.standard_normal(n)
    dc, da = oracle.composite_backward(color, alpha, g, gA)
    # rgb = a c, acc = a
    np.testing.assert_allclose(dc[0], g * alpha[0][:, None], atol=1e-15)
    np.testing.assert_allclose(da[0], np.sum(g * color[0], axis=1) + gA, atol=1e-15)


def test_composite_backward_opaque_front_and_transparent_layers():
    L, n = 4, 6
    color = RNG.uniform(0, 1, (L, n, 3)); alpha = RNG.uniform(0, 1, (L, n))
    g = RNG.standard_normal((n, 3)); gA = RNG.standard_normal(n)
    a1 = alpha.copy(); a1[0] = 1.0
    dc, da = oracle.composite_backward(color, a1, g, gA)
    # everything behind an opaque layer is invisible: zero gradient
    np.testing.assert_array_equal(dc[1:], 0.0)
    np.testing.assert_array_equal(da[1:], 0.0)
    # the front layer: d rgb/d a0 = c0 - B1 (B1 the rest composited alone),
    # d acc/d a0 = prod_{l>0}(1 - a_l)
    B1, _ = oracle.composite(color[1:], a1[1:])
    P1 = np.prod(1.0 - a1[1:], axis=0)
    np.testing.assert_allclose(da[0], np.sum(g * (color[0] - B1), axis=1) + gA * P1, atol=1e-14)
    # all layers transparent: T = 1 throughout, d rgb/d a_l = c_l, d acc/d a_l = 1
    dc0, da0 = oracle.composite_backward(color, np.zeros((L, n)), g, gA)
    np.testing.assert_array_equal(dc0, 0.0)
    np.testing.assert_allclose(da0, np.sum(g[None] * color, axis=2) + gA[None], atol=1e-14)
