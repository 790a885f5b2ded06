"""Serving on the GPU: a request's image does not depend on what runs beside
it (alone vs mixed, bitwise), its finest level matches the FP64 oracle run
from the same learned initialisation, and the device initialisation
matches the oracle's."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_16680_amd import lib, serve, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    scenes, model, reqs = synth.make_serving(n_scenes=3, n_requests=8, rate=1000.0, seed=21,
                                             input_hw=(272, 480),
                                             outputs=((320, 184), (640, 360)))
    pyr = {s.scene_id: synth.device_pyramid(s) for s in scenes}
    torch.cuda.synchronize()
    return scenes, model, reqs, pyr


def _serve(scenes, model, pyr, reqs):
    ex = serve.GpuExecutor({s.scene_id: s for s in scenes}, pyr, model, n_streams=4,
                           keep_rgb=True)
    srv = serve.Server(ex, budget_bytes=8 << 30)
    jobs = srv.run(reqs)
    torch.cuda.synchronize()
    return {j.req.rid: j for j in jobs}


def test_alone_vs_mixed_bitwise(setup):
    scenes, model, reqs, pyr = setup
    at0 = [synth.ServeRequest(r.rid, r.scene_id, r.width, r.height, r.novel, 0.0) for r in reqs]
    mixed = _serve(scenes, model, pyr, at0)
    assert all(j.status == "done" for j in mixed.values()), [j.error for j in mixed.values()]
    for rid in (0, 3):
        alone = _serve(scenes, model, pyr, [at0[rid]])
        a = alone[rid].rgb.cpu().numpy()
        m = mixed[rid].rgb.cpu().numpy()
        _say("request", rid, at0[rid].width, "x", at0[rid].height, "max |alone - mixed|",
             float(np.max(np.abs(a - m))))
        assert np.array_equal(a, m)


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


def test_served_image_matches_oracle(setup):
    """The finest level of a served request (learned initialisation, one
    bf16 Update & Fuse step, composite) against the FP64 oracle on the same
    bf16 features and the bf16-rounded initial feature."""
    scenes, model, reqs, pyr = setup
    req = synth.ServeRequest(0, reqs[1].scene_id, 320, 184, reqs[1].novel, 0.0)
    got = _serve(scenes, model, pyr, [req])[0].rgb.cpu().numpy()
    sc = scenes[req.scene_id]
    k, C, L = synth.SERVE_LEVELS[-1]
    H, W = req.height // k, req.width // k
    feats = [f.float().cpu().numpy() for f in pyr[req.scene_id][-1]]
    f0b = synth.f32_to_bf16_bits(model.f0[-1])
    F0, d0, a0 = oracle.ldm_init(L, H, W, synth.bf16_bits_to_f32(f0b), model.near, model.far)
    lvl = synth.Level(L, H, W, C, C, 1, C, feats, d0, a0, F0, model.weights[-1], True)
    out = oracle.update_fuse(sc.in_cams, req.novel, model.near, model.far, lvl)
    rgb, _ = oracle.composite(out["color"], out["alpha"])
    err = float(np.max(np.abs(got - rgb)))
    mse = float(np.mean((got - rgb) ** 2))
    psnr = 10 * np.log10(1.0 / mse) if mse > 0 else float("inf")
    _say("served vs oracle: max abs", err, "psnr", psnr)
    assert err <= 2e-2 and psnr >= 45.0
