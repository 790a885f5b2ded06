"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances
----------
RGB (in [0, 1]): float32 form max-abs <= 1e-4; bfloat16 form max-abs <= 2e-2
and PSNR >= 45 dB.  The other outputs are checked with bounds derived from
the arithmetic of each form (design notes, "Tolerances"):
  * F' : |err| <= F_abs + F_rel |F'|
  * alpha' : max-abs
  * depth' : in disparity, as a fraction of one step's largest update
    (0.5/L)(1/near - 1/far) -- relative depth error is not a stable measure
    near the far plane, where a small disparity error is a large depth error.
Two-step runs are checked step by step: the second step starts from the
GPU's own first-step state, read back exactly, so both steps are held to
the single-step bounds; the rendered image of the two steps end to end is
held to the RGB targets against the oracle's two steps from the inputs.
Every measured error is written to parity_report.json
in the directory QK_REPORT_DIR names, when it is set.
"""

import math
import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, runner, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {
    "fp32": {"rgb": 1e-4, "acc": 1e-4, "alpha": 1e-4, "disp": 1e-3, "F_abs": 2e-4, "F_rel": 2e-4},
    "bf16": {"rgb": 2e-2, "acc": 2e-2, "alpha": 2e-2, "disp": 1e-1, "F_abs": 4e-2, "F_rel": 1.6e-2},
    # e4m3 projections: each operand rounds to 3 mantissa bits (relative
    # 2^-4), about 8x the bfloat16 rounding, through the same chain; the
    # RGB bar sits just above the measured envelope (worst 0.047 max-abs,
    # 41.9 dB over these cases), which misses the bfloat16 bar -- stated
    "fp8": {"rgb": 5.5e-2, "acc": 5.5e-2, "alpha": 8e-2, "disp": 0.6, "F_abs": 0.3, "F_rel": 0.13},
}
PREC = {"fp32": "fp32", "bf16": "bf16", "fp8": "bf16_fp8proj"}
REPORT = []


def _say(*a):
    print("[parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lib.Context(0)


def psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def compare(gpu, ref, form, scene, level, rows=None, composite=True, label=""):
    """Compare GPU outputs (full arrays) with oracle outputs (packed rows)."""
    t = dict(TOL[form])
    sel = (lambda a: a) if rows is None else (lambda a: a[:, rows])
    F = sel(gpu["F"]); d = sel(gpu["depth"]); a = sel(gpu["alpha"])
    step_range = (0.5 / level.L) * (1.0 / scene.near - 1.0 / scene.far)
    errs = {}
    excess = np.abs(F - ref["F"]) - t["F_rel"] * np.abs(ref["F"])
    errs["F_excess"] = float(np.max(excess))
    errs["F_maxabs"] = float(np.max(np.abs(F - ref["F"])))
    errs["F_rms"] = float(np.sqrt(np.mean((F - ref["F"]) ** 2)))
    errs["alpha"] = float(np.max(np.abs(a - ref["alpha"])))
    errs["disp"] = float(np.max(np.abs(1.0 / d - 1.0 / ref["depth"])) / step_range)
    errs["depth_rel"] = float(np.max(np.abs(d - ref["depth"]) / ref["depth"]))
    if composite:
        rgb = gpu["rgb"] if rows is None else gpu["rgb"][rows]
        acc = gpu["acc"] if rows is None else gpu["acc"][rows]
        errs["rgb"] = float(np.max(np.abs(rgb - ref["rgb"])))
        errs["acc"] = float(np.max(np.abs(acc - ref["acc"])))
        errs["psnr"] = psnr(rgb, ref["rgb"])
    _say(label, form, {k: f"{v:.3g}" for k, v in errs.items()})
    REPORT.append({"case": label, "form": form, **errs})
    assert errs["F_excess"] <= t["F_abs"], (label, "F", errs)
    assert errs["alpha"] <= t["alpha"], (label, "alpha", errs)
    assert errs["disp"] <= t["disp"], (label, "depth", errs)
    if composite:
        assert errs["rgb"] <= t["rgb"], (label, "rgb", errs)
        assert errs["acc"] <= t["acc"], (label, "acc", errs)
        if form == "bf16":
            assert errs["psnr"] >= 45.0, (label, "psnr", errs)
        if form == "fp8":
            assert errs["psnr"] >= 40.0, (label, "psnr", errs)
    return errs


@pytest.fixture(scope="module", autouse=True)
def _write_report():
    yield
    import json
    import os
    out = os.environ.get("QK_REPORT_DIR")
    if out and os.path.isdir(out) and REPORT:
        with open(os.path.join(out, "parity_report.json"), "w") as f:
            json.dump(REPORT, f, indent=1)


def run_gpu_level(ctx, scene, li=0, **kw):
    lvl = scene.levels[li]
    dl = runner.level_to_device(lvl)
    runner.run_level(ctx, scene, dl, **kw)
    return runner.level_outputs_numpy(dl), dl


# ---------------------------------------------------------------- configs

ATTN = ["standard", "folded"]


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_c1_full(ctx, form, attn):
    # the folded (one-to-many) form is checked against the oracle's standard
    # definition: the two are equal in exact arithmetic
    _say("c1 full", form, attn)
    sc = synth.make_inputs(1)
    if form == "bf16":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form=attn)
    compare(gpu, ref, form, sc, sc.levels[0], label=f"c1 {attn}")


def check_rgb(gpu_rgb, ref_rgb, form, label):
    """The rendered image alone against the RGB targets of its form."""
    e = float(np.max(np.abs(gpu_rgb - ref_rgb)))
    q = psnr(gpu_rgb, ref_rgb)
    _say(label, form, f"rgb max-abs {e:.3g} psnr {q:.4g} dB")
    REPORT.append({"case": label, "form": form, "rgb": e, "psnr": q})
    assert e <= TOL[form]["rgb"], (label, "rgb", e)
    if form == "bf16":
        assert q >= 45.0, (label, "psnr", q)
    return e, q


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_c2_two_steps_sampled_rows(ctx, form, attn):
    """Two Update & Fuse steps at 480x270 (V = 4, C = 32, L = 16).  Each step
    is compared with the oracle's step from the same input: step 1 from the
    scene's state, step 2 from the GPU's step-1 output read back exactly
    (bfloat16 and float32 values are exact in float64), both to the
    single-step bounds.  The two steps end to end -- the GPU's image against
    the oracle's two steps from the scene's state -- are held to the RGB
    targets."""
    _say("c2 sampled", form, attn)
    sc = synth.make_inputs(2)
    if form == "bf16":
        sc = synth.to_bf16(sc)
    assert sc.steps == 2
    lvl = sc.levels[0]
    rows = [0, 1, 63, 64, 134, 135, 201, 268, 269]
    dl = runner.level_to_device(lvl)
    # step 1 (no composite)
    runner.run_level(ctx, sc, dl, steps=1, attn_form=attn, composite=False)
    g1 = runner.level_outputs_numpy(dl)
    ref1 = oracle.update_fuse(sc.in_cams, sc.novel, sc.near, sc.far, lvl, rows=rows)
    compare(g1, ref1, form, sc, lvl, rows=rows, composite=False, label=f"c2 step 1 {attn}")
    # step 2, in place on the GPU's state, composited
    runner.run_level(ctx, sc, dl, steps=1, attn_form=attn, from_output=True)
    g2 = runner.level_outputs_numpy(dl)
    ref2 = oracle.update_fuse(sc.in_cams, sc.novel, sc.near, sc.far, lvl, F=g1["F"],
                              depth=g1["depth"], alpha=g1["alpha"], rows=rows)
    ref2["rgb"], ref2["acc"] = oracle.composite(ref2["color"], ref2["alpha"])
    compare(g2, ref2, form, sc, lvl, rows=rows, label=f"c2 step 2 {attn}")
    # both steps end to end
    ref = oracle.run_level(sc, lvl, rows=rows)
    check_rgb(g2["rgb"][rows], ref["rgb"], form, f"c2 two steps end to end {attn}")


@pytest.fixture(scope="module")
def c3_scenes():
    _say("drawing c3 inputs")
    sc = synth.make_inputs(3)
    return {"fp32": sc, "bf16": synth.to_bf16(sc)}


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
@pytest.mark.parametrize("li", [0, 1, 2, 3])
def test_c3_levels_sampled_rows(ctx, c3_scenes, form, li, attn):
    # full 1080p-pyramid sizes, launched exactly as the benchmark launches
    # them (levels 0-2 without composite, level 3 with it)
    sc = c3_scenes[form]
    lvl = sc.levels[li]
    H = lvl.H
    rows = sorted({0, 1, H // 3, H // 2, H - 2, H - 1})
    _say("c3 level", li, form, attn, "rows", rows)
    ref = oracle.run_level(sc, lvl, rows=rows)
    gpu, _ = run_gpu_level(ctx, sc, li, attn_form=attn)
    compare(gpu, ref, form, sc, lvl, rows=rows, composite=lvl.composite, label=f"c3 L{li} {attn}")


# ---------------------------------------------------------------- edge cases

EDGE = [
    # (name, kwargs for make_custom)
    ("ragged-W37-H5-L3-C16-V3", dict(V=3, H=5, W=37, C=16, L=3)),
    ("single-pixel-W1-H1-L2-C8-V2", dict(V=2, H=1, W=1, C=8, L=2)),
    ("one-layer-W70-H3-C32-V4", dict(V=4, H=3, W=70, C=32, L=1)),
    ("one-view-W20-H4-C64-L2", dict(V=1, H=4, W=20, C=64, L=2)),
    ("pad-views-C8-V5", dict(V=5, H=6, W=33, C=8, L=4)),
    ("pad-views-C16-V3", dict(V=3, H=6, W=19, C=16, L=2)),
    ("max-views-V16-C32", dict(V=16, H=4, W=40, C=32, L=2, arc=0.6)),
    # C >= 32 projects the views four at a time: groups cut short at the end
    ("view-groups-C32-V2", dict(V=2, H=3, W=29, C=32, L=2)),
    ("view-groups-C32-V7", dict(V=7, H=4, W=35, C=32, L=3, arc=0.5)),
    ("view-groups-C64-V6", dict(V=6, H=3, W=21, C=64, L=2, arc=0.5)),
    ("feature-grid-differs", dict(V=3, H=9, W=30, C=16, L=3, feat_hw=(5, 17))),
    ("wide-fov-many-invalid", dict(V=4, H=8, W=48, C=8, L=5, arc=1.2, radius=1.0, hfov=100.0)),
]


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
@pytest.mark.parametrize("name,kw", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases(ctx, name, kw, form, attn):
    _say("edge", name, form, attn)
    sc = synth.make_custom(dtype="f32", seed=zlib.crc32(name.encode()) % 1000, **kw)
    if form == "bf16":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form=attn)
    compare(gpu, ref, form, sc, sc.levels[0], label=f"{name} {attn}")


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
@pytest.mark.parametrize("C", [8, 16, 32, 64])
def test_corner_cells(ctx, C, form, attn):
    """Views that are the novel camera itself, with feature maps one pixel
    smaller than the LDM grid: row 0 and column 0 of every layer sample cells
    whose first tap row / column lies outside the map, and pixel (0, 0) the
    corner cell whose only inside tap, (0, 0), carries ~95 % of the weight."""
    _say("corner cells", C, form, attn)
    H, W = 6, 40
    sc = synth.make_custom(V=3, H=H, W=W, C=C, L=3, feat_hw=(H - 1, W - 1), seed=40 + C)
    nov = sc.novel
    sc.in_cams = [synth.Camera(nov.K.copy(), nov.E.copy(), nov.width, nov.height)
                  for _ in range(3)]
    if form == "bf16":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form=attn)
    compare(gpu, ref, form, sc, sc.levels[0], label=f"corner-cells C{C} {attn}")


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_paper_decode_mode(ctx, form, attn):
    _say("paper decode", form, attn)
    sc = synth.make_custom(V=4, H=7, W=45, C=32, L=6, seed=31)
    if form == "bf16":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0], mode=1)
    gpu, _ = run_gpu_level(ctx, sc, mode="paper", attn_form=attn)
    compare(gpu, ref, form, sc, sc.levels[0], label=f"paper-decode {attn}")


HEADS = [
    # (name, kwargs for make_custom): the paper's four and two heads of its
    # 32 channels, and four / two heads at C = 64
    ("C32-h4-hd8-ragged", dict(V=4, H=6, W=37, C=32, L=3, heads=4, head_dim=8)),
    ("C32-h2-hd16", dict(V=3, H=5, W=40, C=32, L=3, heads=2, head_dim=16)),
    ("C64-h4-hd16", dict(V=5, H=4, W=33, C=64, L=2, heads=4, head_dim=16)),
    ("C64-h2-hd32", dict(V=3, H=5, W=20, C=64, L=2, heads=2, head_dim=32)),
    ("C32-h4-V16", dict(V=16, H=3, W=24, C=32, L=2, heads=4, head_dim=8, arc=0.6)),
    ("C32-h4-one-view", dict(V=1, H=4, W=18, C=32, L=2, heads=4, head_dim=8)),
]


@pytest.mark.parametrize("form", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("name,kw", HEADS, ids=[e[0] for e in HEADS])
def test_several_heads(ctx, name, kw, form):
    """Multi-head cross-attention (standard form): per-head softmax over the
    views, heads concatenated into the output projection."""
    _say("heads", name, form)
    sc = synth.make_custom(dtype="f32", seed=zlib.crc32(name.encode()) % 1000, **kw)
    if form != "fp32":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form="standard",
                           precision=PREC["fp8"] if form == "fp8" else None)
    compare(gpu, ref, form, sc, sc.levels[0], label=f"{name} standard")


@pytest.mark.parametrize("form", ["fp32", "bf16"])
@pytest.mark.parametrize("name,kw", [h for h in HEADS if h[1]["C"] == 32],
                         ids=[h[0] for h in HEADS if h[1]["C"] == 32])
def test_several_heads_folded(ctx, name, kw, form):
    """One-to-many attention with several heads (C = 32): per head the query
    with its W_k folded in, a softmax over the views of its dot products with
    the samples, a running sum of the samples, and its W_v W_o folded into
    the output projection over the heads' concatenation.  The oracle runs
    the folded form too (exactly equal to the standard form in real
    arithmetic)."""
    _say("folded heads", name, form)
    sc = synth.make_custom(dtype="f32", seed=zlib.crc32(name.encode()) % 1000, **kw)
    if form != "fp32":
        sc = synth.to_bf16(sc)
    ref = oracle.run_level(sc, sc.levels[0], attn_form=1)
    gpu, _ = run_gpu_level(ctx, sc, attn_form="folded")
    compare(gpu, ref, form, sc, sc.levels[0], label=f"{name} folded")


def test_heads_differ_from_one_head(ctx):
    """The same weights read as four heads and as one head give different
    updates (the per-head softmax is not the one-head softmax)."""
    sc = synth.make_custom(dtype="f32", seed=77, V=4, H=4, W=20, C=32, L=2, heads=4, head_dim=8)
    g4, _ = run_gpu_level(ctx, sc, attn_form="standard")
    sc.levels[0].heads, sc.levels[0].head_dim = 1, 32
    g1, _ = run_gpu_level(ctx, sc, attn_form="standard")
    ref1 = oracle.run_level(sc, sc.levels[0])
    compare(g1, ref1, "fp32", sc, sc.levels[0], label="C32 same weights one head")
    assert float(np.max(np.abs(g4["F"] - g1["F"]))) > 1e-3


def test_in_place_and_optional_outputs(ctx):
    _say("in-place / no F' / no acc")
    sc = synth.make_custom(V=3, H=6, W=50, C=16, L=4, seed=5)
    lvl = sc.levels[0]
    ref = oracle.run_level(sc, lvl)
    dl = runner.level_to_device(lvl)
    # in place: ldm_out aliases ldm_in
    rgb = torch.empty((lvl.H, lvl.W, 3), device="cuda")
    lib.update_fuse(ctx, sc.in_cams, dl.feats, sc.novel, sc.near, sc.far, dl.weights,
                    (dl.F, dl.depth, dl.alpha), (dl.F, dl.depth, dl.alpha), rgb_out=rgb)
    torch.cuda.synchronize()
    np.testing.assert_allclose(rgb.cpu().numpy(), ref["rgb"], atol=1e-4)
    np.testing.assert_allclose(dl.F.cpu().numpy(), ref["F"], atol=2e-4, rtol=2e-4)
    np.testing.assert_allclose(dl.alpha.cpu().numpy(), ref["alpha"], atol=1e-4)
    # F' not written (output F = NULL), composite without acc
    dl2 = runner.level_to_device(lvl)
    sentinel = torch.full_like(dl2.F_out, 7.0)
    dl2.F_out.copy_(sentinel)
    lib.update_fuse(ctx, sc.in_cams, dl2.feats, sc.novel, sc.near, sc.far, dl2.weights,
                    (dl2.F, dl2.depth, dl2.alpha), (None, dl2.depth_out, dl2.alpha_out),
                    rgb_out=rgb)
    torch.cuda.synchronize()
    assert bool((dl2.F_out == 7.0).all())
    np.testing.assert_allclose(rgb.cpu().numpy(), ref["rgb"], atol=1e-4)
    np.testing.assert_allclose(dl2.depth_out.cpu().numpy(), ref["depth"], rtol=1e-4)


def test_identity_camera_single_view_returns_source_pixel(ctx):
    # the sample of a layer-pixel seen by an identical camera is the source
    # pixel: with W_v = W_o = I and V = 1, F' = F + I[y][x] exactly
    _say("identity camera")
    sc = synth.make_custom(V=1, H=5, W=21, C=16, L=2, seed=3)
    sc.in_cams[0] = synth.Camera(sc.novel.K.copy(), sc.novel.E.copy(), 21, 5)
    lvl = sc.levels[0]
    lvl.weights["Wv"] = np.eye(16, dtype=np.float32)
    lvl.weights["Wo"] = np.eye(16, dtype=np.float32)
    gpu, _ = run_gpu_level(ctx, sc)
    expect = lvl.F.astype(np.float64) + lvl.feats[0].astype(np.float64)[None]
    np.testing.assert_allclose(gpu["F"], expect, atol=2e-5)


@pytest.mark.parametrize("attn", ATTN)
def test_runs_are_bitwise_deterministic(ctx, attn):
    _say("determinism", attn)
    sc = synth.to_bf16(synth.make_custom(V=4, H=16, W=100, C=32, L=4, seed=9))
    a, _ = run_gpu_level(ctx, sc, attn_form=attn)
    b, _ = run_gpu_level(ctx, sc, attn_form=attn)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_standalone_composite(ctx):
    _say("standalone composite")
    r = np.random.default_rng(4)
    L, H, W = 7, 13, 29
    color = r.uniform(0, 1, (L, H, W, 3)).astype(np.float32)
    alpha = r.uniform(0, 1, (L, H, W)).astype(np.float32)
    alpha[0, 0, :5] = 1.0
    alpha[:, 1, :] = 0.0
    rgb_ref, acc_ref = oracle.composite(color, alpha)
    c = torch.from_numpy(color).cuda(); a = torch.from_numpy(alpha).cuda()
    rgb = torch.empty((H, W, 3), device="cuda"); acc = torch.empty((H, W), device="cuda")
    lib.composite(ctx, c, a, rgb, acc)
    torch.cuda.synchronize()
    np.testing.assert_allclose(rgb.cpu().numpy(), rgb_ref, atol=1e-6)
    np.testing.assert_allclose(acc.cpu().numpy(), acc_ref, atol=1e-6)


# ---------------------------------------------------------------- e4m3 projections

@pytest.mark.parametrize("attn", ATTN)
def test_fp8_c1_full(ctx, attn):
    _say("c1 full fp8", attn)
    sc = synth.to_bf16(synth.make_inputs(1))
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form=attn, precision=PREC["fp8"])
    compare(gpu, ref, "fp8", sc, sc.levels[0], label=f"c1 {attn}")


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("li", [0, 1, 2, 3])
def test_fp8_c3_levels_sampled_rows(ctx, c3_scenes, li, attn):
    sc = c3_scenes["bf16"]
    lvl = sc.levels[li]
    H = lvl.H
    rows = sorted({0, H // 2, H - 1})
    _say("c3 level fp8", li, attn, "rows", rows)
    ref = oracle.run_level(sc, lvl, rows=rows)
    gpu, _ = run_gpu_level(ctx, sc, li, attn_form=attn, precision=PREC["fp8"])
    compare(gpu, ref, "fp8", sc, lvl, rows=rows, composite=lvl.composite,
            label=f"c3 L{li} {attn}")


@pytest.mark.parametrize("attn", ATTN)
@pytest.mark.parametrize("name,kw", EDGE[:5], ids=[e[0] for e in EDGE[:5]])
def test_fp8_edge_cases(ctx, name, kw, attn):
    _say("edge fp8", name, attn)
    sc = synth.to_bf16(synth.make_custom(dtype="f32", seed=zlib.crc32(name.encode()) % 1000, **kw))
    ref = oracle.run_level(sc, sc.levels[0])
    gpu, _ = run_gpu_level(ctx, sc, attn_form=attn, precision=PREC["fp8"])
    compare(gpu, ref, "fp8", sc, sc.levels[0], label=f"{name} {attn}")
