"""Parity of the layer collapse (qk_layer_collapse) against the FP64 oracle,
through the C-ABI.

Bar (bfloat16 storage and operands, float32 accumulation):
|out_gpu - out_oracle| <= 2e-2 + 1e-2 |out| -- the matrices rounded to
bfloat16 (2^-9 relative per product, 64 then 32 products per output), the
ReLU output rounded as an operand, the result rounded at the store."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[collapse]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _gpu(ctx, F, W1, W2):
    Fd = torch.from_numpy(F.view(np.int16)).cuda().view(torch.bfloat16)
    L, H, W, C = F.shape
    out = torch.full((L // 2, H, W, C), float("nan"), device="cuda", dtype=torch.bfloat16)
    lib.layer_collapse(ctx, Fd, torch.from_numpy(W1).cuda(), torch.from_numpy(W2).cuda(), out)
    torch.cuda.synchronize()
    return out.float().cpu().numpy()


@pytest.mark.parametrize("shape", [(2, 3, 5), (4, 7, 9), (6, 1, 1), (2, 17, 33), (16, 270, 480)])
def test_collapse_parity(ctx, shape):
    L, H, W = shape
    F, W1, W2 = synth.make_collapse(L=L, H=H, W=W, seed=L * 7 + H + W)
    got = _gpu(ctx, F, W1, W2)
    ref = oracle.layer_collapse(F, W1, W2)
    err = np.abs(got - ref)
    ratio = float(np.max(err / (2e-2 + 1e-2 * np.abs(ref))))
    _say(shape, f"max-abs {float(err.max()):.3g} error / bound {ratio:.3g}")
    assert np.all(np.isfinite(got))
    assert ratio <= 1.0


def test_collapse_zero_w2_is_the_mean(ctx):
    F, W1, W2 = synth.make_collapse(L=4, H=5, W=19, seed=3)
    got = _gpu(ctx, F, W1, np.zeros_like(W2))
    Fv = synth.bf16_bits_to_f32(F).astype(np.float64)
    ref = 0.5 * (Fv[0::2] + Fv[1::2])
    # the mean of two bf16 values rounded once to bf16
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 2.0 ** -8
