"""Pins of the oracle's residual CNN block (Sec. 3.3: V' = V +
Conv(gelu(Conv(N(V)))) per LDM layer, 3x3 kernels, zero padding, N the
per-pixel RMS normalisation of the attention's pre-norm, gelu the exact
x Phi(x)): against the library's convolution, normalisation and GELU
(torch conv2d, rms_norm and gelu in float64), and closed forms for a zero
second kernel, a centre-tap identity and the border count of an all-ones
kernel on a constant image."""

import math

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import synth

torch = pytest.importorskip("torch")


def _torch_block(F, W1, W2):
    """The block from torch.nn.functional (conv2d is a cross-correlation, as
    written in the oracle): weights [3][3][ci][co] -> [co][ci][3][3]."""
    x = torch.from_numpy(np.asarray(F, dtype=np.float64))                      # L H W C
    n = torch.nn.functional.rms_norm(x, (x.shape[-1],), eps=1e-6).permute(0, 3, 1, 2)
    k1 = torch.from_numpy(np.asarray(W1, dtype=np.float64)).permute(3, 2, 0, 1)
    k2 = torch.from_numpy(np.asarray(W2, dtype=np.float64)).permute(3, 2, 0, 1)
    h = torch.nn.functional.gelu(torch.nn.functional.conv2d(n, k1, padding=1))
    y = x.permute(0, 3, 1, 2) + torch.nn.functional.conv2d(h, k2, padding=1)
    return y.permute(0, 2, 3, 1).numpy()


@pytest.mark.parametrize("shape", [(2, 9, 13, 8), (1, 5, 7, 16), (3, 4, 17, 32), (1, 1, 1, 8)])
def test_matches_torch(shape):
    L, H, W, C = shape
    F, W1, W2 = synth.make_conv_block(L=L, H=H, W=W, C=C, seed=H * W + C, dtype="f32")
    got = oracle.residual_conv(F, W1, W2)
    ref = _torch_block(F, W1, W2)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_zero_second_kernel_is_identity():
    F, W1, W2 = synth.make_conv_block(L=2, H=6, W=9, C=16, seed=3, dtype="f32")
    assert np.array_equal(oracle.residual_conv(F, W1, np.zeros_like(W2)), F.astype(np.float64))


def test_centre_tap_identity_gives_gelu_of_the_normalised_input():
    """W1 = W2 = identity at the centre tap: V' = V + gelu(N(V))."""
    C = 8
    F, _, _ = synth.make_conv_block(L=2, H=5, W=6, C=C, seed=4, dtype="f32")
    I = np.zeros((3, 3, C, C))
    I[1, 1] = np.eye(C)
    F64 = F.astype(np.float64)
    n = F64 / np.sqrt(np.mean(F64 ** 2, axis=-1, keepdims=True) + 1e-6)
    gelu = np.vectorize(lambda v: 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))))
    assert np.max(np.abs(oracle.residual_conv(F, I, I) - (F64 + gelu(n)))) < 1e-14


def test_zero_padding_counts_inside_taps():
    """A constant image normalises to 1 / sqrt(1 + 1e-6) per channel; an
    all-ones first kernel sums, per pixel, the taps inside the grid times C
    (9 inside, 6 on an edge, 4 at a corner) -- so large that gelu passes it
    unchanged -- and a centre-tap identity second kernel passes that on."""
    L, H, W, C = 1, 4, 5, 8
    F = np.ones((L, H, W, C), dtype=np.float32)
    ones = np.ones((3, 3, C, C))
    I = np.zeros((3, 3, C, C))
    I[1, 1] = np.eye(C)
    out = oracle.residual_conv(F, ones, I) - 1.0
    taps = np.full((H, W), 9.0)
    taps[0, :] = taps[-1, :] = 6.0
    taps[:, 0] = taps[:, -1] = 6.0
    taps[0, 0] = taps[0, -1] = taps[-1, 0] = taps[-1, -1] = 4.0
    assert np.max(np.abs(out[0, ..., 0] - taps * C / math.sqrt(1.0 + 1e-6))) < 1e-12
