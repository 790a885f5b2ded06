"""Parity of the resolution transition (qk_upsample2x) and the volume decode
(qk_ldm_decode) against the FP64 oracle, through the C-ABI.

Bars.  Upsampling, float32: |err| <= 1e-6 max|src| (weights 1/4, 3/4 are
exact; two blends of two float roundings each); bfloat16 adds the final
rounding, 2^-8 |ref|.  Decode (float32 arithmetic): alpha and colour within
1e-5, disparity within 1e-5 of the band 1/near - 1/far (a C-term float dot
product, the library tanh, exp and reciprocal, each a few ulps)."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[resample]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _dev(a, dtype):
    if dtype == "bf16":
        bits = synth.f32_to_bf16_bits(np.ascontiguousarray(a, dtype=np.float32))
        return (torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16),
                synth.bf16_bits_to_f32(bits).astype(np.float64))
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    return torch.from_numpy(a32).cuda(), a32.astype(np.float64)


SHAPES = [(1, 1, 1, 8), (3, 5, 7, 8), (2, 9, 13, 32), (4, 3, 4, 64), (2, 6, 5, 1), (3, 4, 6, 3),
          (1, 17, 33, 16), (1, 1, 40, 4), (8, 36, 64, 32)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=["x".join(map(str, s)) for s in SHAPES])
def test_upsample2x_parity(ctx, shape, dtype):
    N, H, W, C = shape
    src = np.random.default_rng(N * 1000 + H * W + C).standard_normal(shape)
    d, exact = _dev(src, dtype)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    out = torch.full((N, 2 * H, 2 * W, C), float("nan"), device="cuda", dtype=tdt)
    lib.upsample2x(ctx, d, out)
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().astype(np.float64)
    ref = oracle.upsample2x(exact)
    bound = 1e-6 * np.max(np.abs(exact)) + (2.0 ** -8 * np.abs(ref) if dtype == "bf16" else 0.0)
    ratio = float(np.max(np.abs(got - ref) / bound))
    _say(shape, dtype, f"error / bound {ratio:.3g}")
    assert np.all(np.isfinite(got)) and ratio <= 1.0


def test_upsample2x_writes_only_its_output(ctx):
    src = torch.randn((2, 5, 6, 8), device="cuda")
    buf = torch.full((2 * 10 * 12 * 8 + 64,), 3.5, device="cuda")
    lib.upsample2x(ctx, src, buf[: 2 * 10 * 12 * 8].view(2, 10, 12, 8))
    torch.cuda.synchronize()
    assert torch.all(buf[2 * 10 * 12 * 8:] == 3.5).item()


DEC = [(4, 5, 9, 8), (3, 7, 11, 32), (2, 3, 4, 64), (1, 1, 1, 16), (6, 36, 64, 32)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("shape", DEC, ids=["x".join(map(str, s)) for s in DEC])
def test_ldm_decode_parity(ctx, shape, dtype):
    L, H, W, C = shape
    rng = np.random.default_rng(L + 7 * C)
    F = rng.standard_normal(shape)
    ws, wd = rng.standard_normal(C) / np.sqrt(C), rng.standard_normal(C) / np.sqrt(C)
    Wc = rng.standard_normal((C, 3)) / np.sqrt(C)
    near, far = 0.5, 20.0
    Fd, Fx = _dev(F, dtype)
    depth = torch.empty((L, H, W), device="cuda")
    alpha = torch.empty((L, H, W), device="cuda")
    color = torch.empty((L, H, W, 3), device="cuda")
    w = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in (ws, wd, Wc)]
    lib.ldm_decode(ctx, Fd, depth, alpha, *w, near, far, color_out=color)
    torch.cuda.synchronize()
    # the oracle decodes with the float32 weights the kernel reads
    w64 = [t.cpu().numpy().astype(np.float64) for t in w]
    if H * W * L > 4000:                       # sampled rows at the larger size
        rows = [0, H // 2, H - 1]
        dr, ar, cr = oracle.decode_volume(Fx[:, rows], *w64, near, far)
        sel = lambda t: t.cpu().numpy()[:, rows]
    else:
        dr, ar, cr = oracle.decode_volume(Fx, *w64, near, far)
        sel = lambda t: t.cpu().numpy()
    band = 1 / near - 1 / far
    e_disp = float(np.max(np.abs(1 / sel(depth) - 1 / dr))) / band
    e_a = float(np.max(np.abs(sel(alpha) - ar)))
    e_c = float(np.max(np.abs(sel(color) - cr)))
    _say(shape, dtype, f"disp/band {e_disp:.3g} alpha {e_a:.3g} colour {e_c:.3g}")
    assert e_disp <= 1e-5 and e_a <= 1e-5 and e_c <= 1e-5
