"""GPU parity of qk_composite_backward (the adjoint of the over composite,
Sec. 3.1) against the oracle's FP64 adjoint, itself pinned by central
differences and closed forms.  Bar: per tensor relative L2 error <= 1e-3
and every element within 2e-3 of the tensor's largest entry (the backward
tolerance); the float32 recurrences carry ~1e-7 relative per layer."""

import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[composite-bwd]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _rel(got, ref):
    n = float(np.linalg.norm(ref))
    return float(np.linalg.norm(got - ref)) / max(n, 1e-30)


CASES = [
    # (name, L, H, W, with d_acc, alpha special)
    ("L4-1080p-rows", 4, 7, 1920, True, None),
    ("L32-ragged", 32, 5, 37, True, None),
    ("L1", 1, 3, 11, False, None),
    ("opaque-front", 6, 4, 29, True, "opaque"),
    ("transparent", 5, 4, 23, True, "clear"),
    ("single-pixel", 3, 1, 1, False, None),
]


@pytest.mark.parametrize("name,L,H,W,with_acc,special", CASES, ids=[c[0] for c in CASES])
def test_composite_backward_matches_oracle(ctx, name, L, H, W, with_acc, special):
    _say(name, L, H, W)
    r = np.random.default_rng(zlib.crc32(name.encode()) % 1000)
    color = r.uniform(0, 1, (L, H, W, 3)).astype(np.float32)
    alpha = r.beta(0.5, 0.5, (L, H, W)).astype(np.float32)
    if special == "opaque":
        alpha[0, :, : W // 2] = 1.0
    if special == "clear":
        alpha[:] = 0.0
    g = r.standard_normal((H, W, 3)).astype(np.float32)
    gA = r.standard_normal((H, W)).astype(np.float32) if with_acc else None
    dc_ref, da_ref = oracle.composite_backward(color, alpha, g, gA)
    c_d, a_d, g_d = (torch.from_numpy(x).cuda() for x in (color, alpha, g))
    gA_d = torch.from_numpy(gA).cuda() if with_acc else None
    dc = torch.full_like(c_d, 7.0)
    da = torch.full_like(a_d, 7.0)
    lib.composite_backward(ctx, c_d, a_d, g_d, da, d_color=dc, d_acc=gA_d)
    torch.cuda.synchronize()
    got_c, got_a = dc.cpu().numpy().astype(np.float64), da.cpu().numpy().astype(np.float64)
    for nm, got, ref in (("d_color", got_c, dc_ref), ("d_alpha", got_a, da_ref)):
        rel = _rel(got, ref)
        el = float(np.max(np.abs(got - ref))) / max(float(np.max(np.abs(ref))), 1e-30)
        _say(name, nm, f"rel {rel:.3g} element {el:.3g}")
        if float(np.max(np.abs(ref))) == 0.0:
            assert float(np.max(np.abs(got))) == 0.0, (name, nm)
            continue
        assert rel <= 1e-3 and el <= 2e-3, (name, nm, rel, el)


def test_composite_backward_without_color_gradient(ctx):
    """d_color = NULL computes d_alpha alone (and leaves nothing else written)."""
    r = np.random.default_rng(5)
    L, H, W = 5, 6, 40
    color = r.uniform(0, 1, (L, H, W, 3)).astype(np.float32)
    alpha = r.uniform(0, 1, (L, H, W)).astype(np.float32)
    g = r.standard_normal((H, W, 3)).astype(np.float32)
    _, da_ref = oracle.composite_backward(color, alpha, g)
    da = torch.empty((L, H, W), device="cuda")
    lib.composite_backward(ctx, torch.from_numpy(color).cuda(), torch.from_numpy(alpha).cuda(),
                           torch.from_numpy(g).cuda(), da)
    torch.cuda.synchronize()
    assert _rel(da.cpu().numpy().astype(np.float64), da_ref) <= 1e-3


def test_composite_forward_then_backward_through_torch_autograd(ctx):
    """The adjoint agrees with torch's own float64 autograd of the forward
    composite (a second, independent route to the same derivative)."""
    r = np.random.default_rng(8)
    L, H, W = 6, 3, 17
    color = r.uniform(0, 1, (L, H, W, 3))
    alpha = r.uniform(0, 1, (L, H, W))
    g = r.standard_normal((H, W, 3))
    gA = r.standard_normal((H, W))
    c = torch.tensor(color, requires_grad=True)
    a = torch.tensor(alpha, requires_grad=True)
    T = torch.cumprod(torch.cat([torch.ones(1, H, W, dtype=a.dtype), 1 - a[:-1]]), 0)
    rgb = (T[..., None] * a[..., None] * c).sum(0)
    acc = 1 - torch.prod(1 - a, 0)
    ((rgb * torch.tensor(g)).sum() + (acc * torch.tensor(gA)).sum()).backward()
    dc = torch.empty((L, H, W, 3), device="cuda")
    da = torch.empty((L, H, W), device="cuda")
    f = lambda x: torch.from_numpy(x.astype(np.float32)).cuda()
    lib.composite_backward(ctx, f(color), f(alpha), f(g), da, d_color=dc, d_acc=f(gA))
    torch.cuda.synchronize()
    assert _rel(dc.cpu().numpy().astype(np.float64), c.grad.numpy()) <= 1e-3
    assert _rel(da.cpu().numpy().astype(np.float64), a.grad.numpy()) <= 1e-3
