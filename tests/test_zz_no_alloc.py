"""qk_update_fuse_noalloc (the allocation-free variant of qk_update_fuse,
for callers that cannot allocate) against qk_update_fuse through the C-ABI.
The two share every kernel; the variant keeps the folded weights and the
e4m3 scales in the device's fixed scratch instead of the context's
workspaces, so its outputs must equal the existing entry point's bit for
bit.  Each case makes two variant calls in a row, the second on a smaller
input (the scratch keeps the first call's contents), and the small case is
also held to the oracle at the parity bounds of its form."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, runner, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _scene(V, H, W, C, L, seed, bf16, heads=1):
    kw = dict(heads=heads, head_dim=C // heads) if heads > 1 else {}
    sc = synth.make_custom(V=V, H=H, W=W, C=C, L=L, seed=seed, **kw)
    return synth.to_bf16(sc) if bf16 else sc


def _run(ctx, fn, sc, precision, attn):
    lvl = sc.levels[0]
    dl = runner.level_to_device(lvl)
    wts = lib.make_weights(dl.weights, heads=dl.heads)
    fn(ctx, sc.in_cams, dl.feats, sc.novel, sc.near, sc.far, wts, (dl.F, dl.depth, dl.alpha),
       (dl.F_out, dl.depth_out, dl.alpha_out), precision=precision, attn_form=attn,
       rgb_out=dl.rgb, acc_out=dl.acc)
    return dl


def _outs(dl):
    torch.cuda.synchronize()
    return {k: t.float().cpu().numpy() for k, t in
            (("F", dl.F_out), ("depth", dl.depth_out), ("alpha", dl.alpha_out),
             ("rgb", dl.rgb), ("acc", dl.acc))}


CASES = [
    # (name, precision, attention, (V, H, W, C, L, heads) large, then small)
    ("bf16-folded-C64", "bf16", "folded", (5, 9, 150, 64, 3, 1), (3, 4, 37, 64, 2, 1)),
    ("bf16-folded-C32-h4", "bf16", "folded", (4, 8, 200, 32, 4, 4), (2, 3, 45, 32, 2, 4)),
    ("fp32-folded-C16", "fp32", "folded", (4, 6, 130, 16, 3, 1), (3, 5, 21, 16, 2, 1)),
    ("fp8-standard-C32", "bf16_fp8proj", "standard", (6, 7, 160, 32, 3, 1), (2, 4, 30, 32, 2, 1)),
    ("fp8-folded-C8", "bf16_fp8proj", "folded", (5, 6, 300, 8, 4, 1), (3, 2, 50, 8, 3, 1)),
    ("bf16-standard-C16", "bf16", "standard", (4, 5, 120, 16, 3, 1), (2, 3, 19, 16, 2, 1)),
]


@pytest.mark.parametrize("name,prec,attn,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_update_fuse(ctx, name, prec, attn, big, small):
    bf16 = prec != "fp32"
    scenes = [_scene(*shape[:5], seed=300 + i, bf16=bf16, heads=shape[5])
              for i, shape in enumerate((big, small))]
    _say(name, "existing entry point on both inputs")
    ref = [_outs(_run(ctx, lib.update_fuse, sc, prec, attn)) for sc in scenes]
    _say(name, "allocation-free entry point, two calls in a row (large, then small)")
    dls = [_run(ctx, lib.update_fuse_noalloc, sc, prec, attn) for sc in scenes]
    got = [_outs(dl) for dl in dls]
    for i in range(2):
        for k in ref[i]:
            np.testing.assert_array_equal(got[i][k], ref[i][k], err_msg=f"{name} call {i} {k}")
    # the small case against the oracle (parity bounds of its form)
    sc = scenes[1]
    o = oracle.run_level(sc, sc.levels[0], attn_form=1 if attn == "folded" else 0)
    tol = {"fp32": 1e-4, "bf16": 2e-2, "bf16_fp8proj": 8e-2}[prec]
    e = float(np.max(np.abs(got[1]["rgb"].astype(np.float64) - o["rgb"])))
    _say(name, f"small case rgb max-abs vs oracle {e:.3g} (tol {tol})")
    assert e <= tol
