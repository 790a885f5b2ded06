"""Static weights (qk_context_weights_static): the derived copies a context
keeps give the same bits as deriving them per call, new masters are picked
up by pointer, and re-declaring drops the kept copies after masters change
in place."""
import numpy as np
import pytest
import torch

from paper_2411_16680_amd import lib, runner, synth

pytestmark = pytest.mark.gpu


def _level(ctx, sc, dl, attn):
    runner.run_level(ctx, sc, dl, attn_form=attn)
    torch.cuda.synchronize()
    return dl.F_out.float().cpu().numpy().copy(), dl.rgb.cpu().numpy().copy()


@pytest.mark.parametrize("form", ["bf16", "fp32"])
def test_folded_weights_kept(form):
    print("[static] folded level", form, flush=True)
    sc = synth.make_custom(dtype="f32", seed=61, V=4, H=6, W=40, C=32, L=3)
    if form == "bf16":
        sc = synth.to_bf16(sc)
    ref_ctx = lib.Context(0)
    dl = runner.scene_to_device(sc)[0]
    ref = _level(ref_ctx, sc, dl, "folded")
    ctx = lib.Context(0)
    ctx.weights_static(True)
    for _ in range(3):                            # derived once, then kept
        got = _level(ctx, sc, dl, "folded")
        assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    # masters changed in place: re-declaring drops the kept copy
    dl.weights["Wq"].mul_(0.5)
    dl.weights["Wo"].mul_(-1.0)
    ctx.weights_static(True)
    ref2 = _level(ref_ctx, sc, dl, "folded")
    got2 = _level(ctx, sc, dl, "folded")
    assert all(np.array_equal(a, b) for a, b in zip(got2, ref2))


def test_chain_and_frame_with_static_weights():
    print("[static] chain", flush=True)
    ch = synth.make_chain()
    dc = runner.chain_to_device(ch)
    ref_ctx, ctx = lib.Context(0), lib.Context(0)
    ctx.weights_static(True)
    runner.run_chain(ref_ctx, ch, dc, attn_form="auto")
    torch.cuda.synchronize()
    ref = dc.rgb.cpu().numpy().copy()
    for _ in range(2):
        runner.run_chain(ctx, ch, dc, attn_form="auto")
        torch.cuda.synchronize()
        assert np.array_equal(dc.rgb.cpu().numpy(), ref)


def test_static_null_context():
    with pytest.raises(lib.QuarkError) as e:
        lib._check(lib.load().qk_context_weights_static(None, 1))
    assert e.value.status == lib.QK_EINVAL
