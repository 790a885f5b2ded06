"""Parity of the chained multi-scale updates (runner.run_chain: layer
collapse, 2x upsampling, decode and Update & Fuse with the absolute decode,
step after step) against the FP64 oracle's chain, through the C-ABI.

Every chain is checked kernel by kernel, each kernel from the GPU's own
input to it (read back exactly), so nothing compounds: the transition
(collapse 2e-2 + 1e-2|ref|, carried through the upsampling, which adds its
rounding: 2^-8|ref| in bfloat16, plus 1e-6 max|src|), the decode (1e-5 in
alpha and in disparity over the band), the update (the single-step
Update & Fuse bounds of its form: float32 F' within 2e-4 + 2e-4|F'|, alpha
1e-4, disparity 1e-3 of one step's update; bfloat16 4e-2 + 1.6e-2|F'|,
2e-2, 0.1), the residual CNN block (2e-2 + 1e-2|ref|, its own bound) and
the output LDM (decode 1e-5, composite 1e-4).  The small chains are also
compared end to end, the GPU's image against the oracle's whole chain from
the same inputs: float32 at the RGB target 1e-4; bfloat16 at the measured
error of this workload (its bound and the reason it exceeds the one-step
target are stated at the test).
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, runner, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": {"alpha": 1e-4, "disp": 1e-3, "F_abs": 2e-4, "F_rel": 2e-4, "rgb": 1e-4},
       "bf16": {"alpha": 2e-2, "disp": 1e-1, "F_abs": 4e-2, "F_rel": 1.6e-2, "rgb": 2e-2}}


def _say(*a):
    print("[chain]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _check_step(label, got_F, got_d, got_a, ref, L, near, far, tol):
    """F' against ref["F"]; depth' and alpha' (if given) against ref's."""
    band = (0.5 / L) * (1.0 / near - 1.0 / far)
    e_F = float(np.max(np.abs(got_F - ref["F"]) - tol["F_rel"] * np.abs(ref["F"])))
    e_a = float(np.max(np.abs(got_a - ref["alpha"]))) if got_a is not None else 0.0
    e_d = (float(np.max(np.abs(1.0 / got_d - 1.0 / ref["depth"]))) / band
           if got_d is not None else 0.0)
    _say(label, f"F excess {e_F:.3g} alpha {e_a:.3g} disp {e_d:.3g}")
    assert e_F <= tol["F_abs"], (label, "F")
    assert e_a <= tol["alpha"], (label, "alpha")
    assert e_d <= tol["disp"], (label, "disp")


def check_chain_stepwise(ch, dc, attn, form, rows_of, tag, first_input=None, composite=True):
    """Every kernel of a chain the GPU has run, each from the GPU's own input
    to it, on the rows ``rows_of(step)`` of each step.  ``first_input``: the
    first step's input volume when it is not decoded (the learned
    initialisation, checked by the caller); ``composite``: whether the last
    step's output LDM was composited (else its update's depth' and alpha'
    are checked like any step's)."""
    tol = TOL[form]
    band = 1.0 / ch.near - 1.0 / ch.far

    for i, st in enumerate(ch.steps):
        rows = rows_of(st)
        label = f"{tag} {attn} step {i} ({st.L}x{st.H}x{st.W}, {st.heads} heads)"
        if i == 0:
            F_in = _np(dc.F0) if first_input is None else first_input
        else:
            # the transition, from the GPU's previous output
            src = _np(dc.F_conv[i - 1] if ch.steps[i - 1].conv else dc.F_out[i - 1])
            ref_in, bound = src, 0.0
            if st.collapse:
                ref_in = oracle.layer_collapse(src, *ch.collapse_w[i])
                bound = 2e-2 + 1e-2 * np.abs(ref_in)
            if st.upsample:
                carried = oracle.upsample2x(bound) if st.collapse else 0.0
                ref_in = oracle.upsample2x(ref_in)
                rnd = 2.0 ** -8 * np.abs(ref_in) if form == "bf16" else 0.0
                bound = carried + rnd + 1e-6 * np.max(np.abs(src))
            F_in = (_np(dc.F_in[i]) if st.upsample else _np(dc.tmp[i]) if st.collapse else src)
            if st.collapse or st.upsample:
                b = bound[:, rows] if np.ndim(bound) else bound
                r = float(np.max(np.abs(F_in[:, rows] - ref_in[:, rows]) / b))
                _say(label, f"transition error / bound {r:.3g}")
                assert r <= 1.0, (label, "transition")
        # the decode of the step's input
        w = ch.weights[i]
        d_in, a_in = _np(dc.depth[i]), _np(dc.alpha[i])
        if i > 0 or first_input is None:
            dr, ar, _ = oracle.decode_volume(F_in[:, rows], w["w_sigma"], w["w_depth"],
                                             w["W_color"], ch.near, ch.far)
            e_dd = float(np.max(np.abs(1 / d_in[:, rows] - 1 / dr))) / band
            e_da = float(np.max(np.abs(a_in[:, rows] - ar)))
            _say(label, f"decode disp/band {e_dd:.3g} alpha {e_da:.3g}")
            assert e_dd <= 1e-5 and e_da <= 1e-5, (label, "decode")
        # the update, from the GPU's decoded input (the last step's depth'
        # and alpha' are the decode of its CNN block's output, checked below)
        last = i == len(ch.steps) - 1
        ref = oracle.update_fuse(ch.in_cams, ch.novel, ch.near, ch.far, ch.level(i), F=F_in,
                                 depth=d_in, alpha=a_in, rows=rows, mode=1,
                                 attn_form=1 if runner.step_form(attn, st) == "folded" else 0)
        skip = last and st.conv and composite
        _check_step(label, _np(dc.F_out[i])[:, rows],
                    None if skip else _np(dc.depth_out[i])[:, rows],
                    None if skip else _np(dc.alpha_out[i])[:, rows], ref, st.L, ch.near, ch.far,
                    tol)
        if st.conv:
            # the CNN block on slabs of rows around each sampled row, from the
            # GPU's update output (rows beyond the slab cannot reach its centre;
            # the block normalises its input, so its inner sums, and their
            # rounding, do not grow with the input's magnitude)
            Fo, Fc = _np(dc.F_out[i]), _np(dc.F_conv[i])
            worst = 0.0
            for r in rows:
                lo, hi = max(0, r - 2), min(st.H, r + 3)
                ref_c = oracle.residual_conv(Fo[:, lo:hi], *ch.conv_w[i])[:, r - lo]
                worst = max(worst, float(np.max(np.abs(Fc[:, r] - ref_c) /
                                                (2e-2 + 1e-2 * np.abs(ref_c)))))
            rms = float(np.sqrt(np.mean(Fo ** 2)))
            _say(label, f"residual block error / bound {worst:.3g} (input rms {rms:.3g})")
            assert worst <= 1.0, (label, "conv")
        if last and composite:
            if st.conv:
                # the output LDM: decode of the block's output, composited
                dr, ar, cr = oracle.decode_volume(_np(dc.F_conv[i])[:, rows], w["w_sigma"],
                                                  w["w_depth"], w["W_color"], ch.near, ch.far)
                e_dd = float(np.max(np.abs(1 / _np(dc.depth_out[i])[:, rows] - 1 / dr))) / band
                e_da = float(np.max(np.abs(_np(dc.alpha_out[i])[:, rows] - ar)))
                _say(label, f"output decode disp/band {e_dd:.3g} alpha {e_da:.3g}")
                assert e_dd <= 1e-5 and e_da <= 1e-5, (label, "output decode")
                rgb, _ = oracle.composite(cr, ar)
                e_rgb = float(np.max(np.abs(_np(dc.rgb)[rows] - rgb)))
                _say(f"{tag} rgb max-abs on sampled rows {e_rgb:.3g} (decode + composite)")
                assert e_rgb <= 1e-4
            else:
                rgb, _ = oracle.composite(ref["color"], ref["alpha"])
                e_rgb = float(np.max(np.abs(_np(dc.rgb)[rows] - rgb)))
                _say(f"{tag} rgb max-abs on sampled rows {e_rgb:.3g}")
                assert e_rgb <= tol["rgb"]


SMALL = {
    # three steps: the paper's four, two and one heads, an upsampling, then a
    # collapse with an upsampling, a residual CNN block after each attention
    # (bfloat16: the collapse and the CNN block take bfloat16)
    "bf16": (synth.ChainStep(4, 6, 10, 0, 4, False, False, True),
             synth.ChainStep(4, 12, 20, 1, 2, False, True, True),
             synth.ChainStep(2, 24, 40, 2, 1, True, True, True)),
    # float32: no collapse, no CNN block
    "fp32": (synth.ChainStep(4, 6, 10, 0, 4, False, False),
             synth.ChainStep(4, 12, 20, 1, 2, False, True),
             synth.ChainStep(4, 12, 20, 1, 1, False, False)),
}


# The bfloat16 chain end to end: three steps whose inputs pass through a
# bfloat16 layer collapse and residual CNN blocks.  Each kernel meets its own
# bound above; end to end, every step samples the N(0, 1) feature maps at
# positions moved by the earlier steps' rounding-level depth differences,
# and at this grid's focal length a fraction of a pixel on an i.i.d. map is
# an O(1) change of the sample.  Measured max-abs 0.025-0.030 over runs; the
# bound sits just above it.  The PSNR target holds (measured 51 dB).
BF16_CHAIN_RGB = 3.5e-2
BF16_CHAIN_PSNR = 45.0


@pytest.mark.parametrize("attn", ["folded", "standard", "auto"])
@pytest.mark.parametrize("form", ["bf16", "fp32"])
def test_small_chain(ctx, form, attn):
    steps = SMALL[form]
    ch = synth.make_chain(V=3, steps=steps, feat_hw=((6, 10), (12, 20), (24, 40)),
                          input_hw=(48, 80), dtype="bf16" if form == "bf16" else "f32", seed=21)
    dc = runner.chain_to_device(ch)
    runner.run_chain(ctx, ch, dc, attn_form=attn)
    torch.cuda.synchronize()
    check_chain_stepwise(ch, dc, attn, form, lambda st: list(range(st.H)), f"small {form}")
    # end to end, from the same inputs
    _, rgb, _ = oracle.run_chain(ch, attn_form=1 if attn == "folded" else 0)
    got = _np(dc.rgb)
    e_rgb = float(np.max(np.abs(got - rgb)))
    mse = float(np.mean((got - rgb) ** 2))
    q = float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
    _say(form, attn, f"end to end rgb max-abs {e_rgb:.3g} psnr {q:.4g} dB")
    if form == "fp32":
        assert e_rgb <= 1e-4
    else:
        assert e_rgb <= BF16_CHAIN_RGB and q >= BF16_CHAIN_PSNR


@pytest.mark.parametrize("attn", ["folded", "standard"])
def test_quark_schedule_step_by_step(ctx, attn):
    """The five Update & Fuse steps of the paper's network table at 1080p
    inputs (V = 8, C = 32, 24 -> 24 -> 24 -> 12 -> 6 layers, 36x64 ->
    288x512, heads 4, 4, 4, 2, 1), bfloat16, run as one chain on the GPU and
    checked kernel by kernel on sampled rows, each from the GPU's own input:
    the transition (collapse: 2e-2 + 1e-2|ref|, upsampling: 2^-8|ref| +
    1e-6 max|src|, from the GPU's previous output), the decode (1e-5 in
    alpha and in disparity over the band), the update (the single-step
    bfloat16 bounds, from the GPU's decoded input), the residual CNN block
    (2e-2 + 1e-2|ref|, its own parity bound, on row slabs around the
    sampled rows, from the GPU's update output) and the output LDM (decode of the block's output 1e-5,
    its composite 1e-4)."""
    ch = synth.make_chain()
    dc = runner.chain_to_device(ch)
    runner.run_chain(ctx, ch, dc, attn_form=attn)
    torch.cuda.synchronize()
    check_chain_stepwise(ch, dc, attn, "bf16",
                         lambda st: sorted({0, st.H // 3, st.H // 2, st.H - 1}), "quark")
