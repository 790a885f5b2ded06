"""Pins of the oracle's layer collapse (mean of adjacent layers plus a
residual ReLU MLP of their concatenation): an independent float64
re-implementation with torch matmuls, the pure mean when W2 = 0, and a
selector MLP whose residual is relu of the first layer."""

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import synth

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape", [(2, 3, 5, 8), (4, 7, 9, 32), (6, 1, 1, 16)])
def test_matches_torch(shape):
    L, H, W, C = shape
    F, W1, W2 = synth.make_collapse(L=L, H=H, W=W, C=C, seed=L + H + W + C, dtype="f32")
    got = oracle.layer_collapse(F, W1, W2)
    x = torch.from_numpy(F.astype(np.float64)).reshape(L // 2, 2, H, W, C)
    cat = torch.cat([x[:, 0], x[:, 1]], dim=-1)
    ref = 0.5 * (x[:, 0] + x[:, 1]) + torch.relu(cat @ torch.from_numpy(W1.astype(np.float64))) \
        @ torch.from_numpy(W2.astype(np.float64))
    assert np.max(np.abs(got - ref.numpy())) < 1e-12


def test_zero_w2_is_the_mean():
    F, W1, W2 = synth.make_collapse(L=4, H=3, W=4, C=8, seed=2, dtype="f32")
    got = oracle.layer_collapse(F, W1, np.zeros_like(W2))
    F64 = F.astype(np.float64)
    assert np.array_equal(got, 0.5 * (F64[0::2] + F64[1::2]))


def test_selector_mlp():
    """W1 = [I; 0], W2 = I: out = mean + relu(first layer of the pair)."""
    C = 8
    F, _, _ = synth.make_collapse(L=4, H=2, W=3, C=C, seed=3, dtype="f32")
    W1 = np.vstack([np.eye(C), np.zeros((C, C))])
    got = oracle.layer_collapse(F, W1, np.eye(C))
    F64 = F.astype(np.float64)
    assert np.max(np.abs(got - (0.5 * (F64[0::2] + F64[1::2]) + np.maximum(F64[0::2], 0)))) < 1e-15
