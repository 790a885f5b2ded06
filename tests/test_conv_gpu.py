"""Parity of the residual CNN block (qk_residual_conv: F' = F + W2 *
gelu(W1 * N(F)) per layer, N the per-pixel RMS normalisation, 3x3, zero
padding) against the FP64 oracle, through the C-ABI.

Bar (bfloat16 storage and operands, float32 accumulation):
|F'_gpu - F'_oracle| <= 2e-2 + 1e-2 |F'|.  The kernels are rounded to
bfloat16 (2^-9 relative per product, 288 products per output with random
signs), so are the normalised input and the GELU output feeding the
convolutions, and the sum once more at the store (2^-9 |F'|); with
unit-variance features and 1/sqrt(fan_in) weights the two chained sums
carry ~5e-3 typical, the bound is ~4 of those."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[conv]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _gpu(ctx, F, W1, W2):
    Fd = torch.from_numpy(F.view(np.int16)).cuda().view(torch.bfloat16)
    out = torch.full_like(Fd, float("nan"))
    lib.residual_conv(ctx, Fd, torch.from_numpy(W1).cuda(), torch.from_numpy(W2).cuda(), out)
    torch.cuda.synchronize()
    return out.float().cpu().numpy()


def _compare(name, got, ref):
    err = np.abs(got - ref)
    ratio = float(np.max(err / (2e-2 + 1e-2 * np.abs(ref))))
    _say(name, f"max-abs {float(err.max()):.3g} rms {float(np.sqrt(np.mean(err ** 2))):.3g} "
               f"error / bound {ratio:.3g}")
    assert np.all(np.isfinite(got))
    assert ratio <= 1.0, (name, ratio)


@pytest.mark.parametrize("shape", [(2, 9, 13), (1, 1, 1), (3, 17, 35), (2, 8, 16), (1, 24, 7),
                                   (1, 40, 64)])
def test_conv_parity(ctx, shape):
    L, H, W = shape
    F, W1, W2 = synth.make_conv_block(L=L, H=H, W=W, seed=L * 1000 + H * 31 + W)
    _compare(f"L{L}-{H}x{W}", _gpu(ctx, F, W1, W2), oracle.residual_conv(F, W1, W2))


def test_conv_full_size_sampled_layers(ctx):
    """The benchmark's volume (16 layers of 480x270, C = 32), checked on its
    first and last layers (layers are independent)."""
    F, W1, W2 = synth.make_conv_block()
    got = _gpu(ctx, F, W1, W2)
    for l in (0, F.shape[0] - 1):
        _compare(f"480x270-layer{l}", got[l:l + 1], oracle.residual_conv(F[l:l + 1], W1, W2))


def test_conv_identity_kernels(ctx):
    """Centre-tap identities: F' = F + gelu(N(F)) up to three bfloat16
    roundings, each at most 2^-8 of its value: the normalised input (through
    gelu, whose slope is below 1.13), the GELU output and the sum."""
    import math
    C = 32
    F, _, _ = synth.make_conv_block(L=2, H=11, W=21, seed=5)
    I = np.zeros((3, 3, C, C), dtype=np.float32)
    I[1, 1] = np.eye(C, dtype=np.float32)
    got = _gpu(ctx, F, I, I)
    Fv = synth.bf16_bits_to_f32(F).astype(np.float64)
    n = Fv / np.sqrt(np.mean(Fv ** 2, axis=-1, keepdims=True) + 1e-6)
    g = np.vectorize(lambda v: 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))))(n)
    ref = Fv + g
    bound = 2.0 ** -8 * (np.abs(ref) + 1.13 * np.abs(n) + np.abs(g)) + 1e-6
    assert np.max(np.abs(got - ref) / bound) <= 1.0
