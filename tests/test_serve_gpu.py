"""Serving on the GPU: a request's image does not depend on what runs beside
it (alone vs mixed in one batch, bitwise), a served 1920x1080 request from
a resident 1080p pyramid matches the FP64 oracle kernel by kernel (the
whole frame's bounds), and the device initialisation matches the oracle's."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, serve, synth

from test_pipeline_gpu import check_pipeline_stepwise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    scenes, model, reqs = synth.make_serving(n_scenes=3, n_requests=6, rate=1000.0, seed=21)
    res = {s.scene_id: (synth.device_pyramid(s), synth.device_images(s)) for s in scenes}
    torch.cuda.synchronize()
    return scenes, model, reqs, res


def _serve(scenes, model, res, reqs, keep=False):
    ex = serve.GpuExecutor({s.scene_id: s for s in scenes}, res, model, n_streams=4,
                           keep_frames=keep)
    srv = serve.Server(ex, budget_bytes=64 << 30)
    jobs = srv.run(reqs)
    torch.cuda.synchronize()
    return {j.req.rid: j for j in jobs}


def test_alone_vs_mixed_bitwise(setup):
    """Requests arriving together are admitted at one poll and run as one
    batch (one launch per Update & Fuse step); each image equals the same
    request served alone, bit for bit."""
    scenes, model, reqs, res = setup
    sizes = synth.SERVE_OUTPUTS
    at0 = []
    for i, r in enumerate(reqs):
        W, H = sizes[i % len(sizes)]
        K = r.novel.K * np.array([[W / r.width], [H / r.height], [1.0]])
        at0.append(synth.ServeRequest(r.rid, r.scene_id, W, H,
                                      synth.Camera(K, r.novel.E.copy(), W, H), 0.0))
    mixed = _serve(scenes, model, res, at0, keep=True)
    assert all(j.status == "done" for j in mixed.values()), [j.error for j in mixed.values()]
    for rid in (0, 2, 4):
        alone = _serve(scenes, model, res, [at0[rid]], keep=True)
        a = alone[rid].frame.rgb.cpu().numpy()
        m = mixed[rid].frame.rgb.cpu().numpy()
        _say("request", rid, at0[rid].width, "x", at0[rid].height, "scene", at0[rid].scene_id,
             "max |alone - mixed|", float(np.max(np.abs(a - m))))
        assert np.array_equal(a, m)


def test_served_1080p_frame_matches_oracle(setup):
    """A served 1920x1080 request (V from its scene, 1080p pyramid resident
    on the device) checked kernel by kernel against the FP64 oracle on
    sampled rows, from the GPU's own input to each kernel."""
    scenes, model, reqs, res = setup
    r = reqs[1]
    W, H = 1920, 1080
    K = r.novel.K * np.array([[W / r.width], [H / r.height], [1.0]])
    req = synth.ServeRequest(0, r.scene_id, W, H, synth.Camera(K, r.novel.E.copy(), W, H), 0.0)
    job = _serve(scenes, model, res, [req], keep=True)[0]
    assert job.status == "done", job.error
    sc = scenes[req.scene_id]
    pyr, images = res[req.scene_id]
    feats = [[synth.f32_to_bf16_bits(f.float().cpu().numpy()) for f in lvl] for lvl in pyr]
    ch = synth.ChainScene(sc.in_cams, req.novel, model.near, model.far, model.C, model.steps,
                          feats, None, model.weights, model.collapse_w, model.conv_w, "bf16")
    pl = synth.PipelineScene(ch, model.f0, model.Wr, model.low_hw,
                             [im.cpu().numpy() for im in images], (H, W))
    check_pipeline_stepwise(pl, job.frame, "auto", "bf16",
                            lambda st: sorted({0, st.H // 2, st.H - 1}),
                            sorted({0, H // 3, H - 1}), f"served {W}x{H} V{sc.V}")


def test_ldm_init_matches_oracle(setup):
    ctx = lib.Context(0)
    L, H, W, C = 5, 7, 33, 16
    f0 = np.random.default_rng(2).standard_normal(C).astype(np.float32)
    for dt, tdt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        F = torch.empty((L, H, W, C), device="cuda", dtype=tdt)
        d = torch.empty((L, H, W), device="cuda")
        a = torch.empty((L, H, W), device="cuda")
        lib.ldm_init(ctx, torch.from_numpy(f0).cuda(), 0.5, 20.0, (F, d, a))
        torch.cuda.synchronize()
        f0_ref = f0 if dt == "f32" else synth.bf16_bits_to_f32(synth.f32_to_bf16_bits(f0))
        Fr, dr, ar = oracle.ldm_init(L, H, W, f0_ref, 0.5, 20.0)
        assert np.array_equal(F.float().cpu().numpy(), Fr.astype(np.float32))
        assert np.allclose(d.cpu().numpy(), dr, rtol=2e-7)
        assert np.array_equal(a.cpu().numpy(), ar.astype(np.float32))
