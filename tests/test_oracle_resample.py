"""Pins of the oracle's resolution transition and volume decode: the 2x
bilinear upsampling against its closed-form weights (every output a blend
of two rows and two columns with weights 1/4, 3/4, the border row clamping
onto itself) and a constant and an affine field; the volume decode against
the per-pixel decode and its anchor band."""

import numpy as np

import oracle


def _closed_form_2x(src):
    N, H, W, C = src.shape
    out = np.zeros((N, 2 * H, 2 * W, C))
    for Y in range(2 * H):
        y = Y // 2
        ya, yb = (max(y - 1, 0), y) if Y % 2 == 0 else (y, min(y + 1, H - 1))
        wa, wb = (0.25, 0.75) if Y % 2 == 0 else (0.75, 0.25)
        for X in range(2 * W):
            x = X // 2
            xa, xb = (max(x - 1, 0), x) if X % 2 == 0 else (x, min(x + 1, W - 1))
            ua, ub = (0.25, 0.75) if X % 2 == 0 else (0.75, 0.25)
            out[:, Y, X] = (wa * (ua * src[:, ya, xa] + ub * src[:, ya, xb]) +
                            wb * (ua * src[:, yb, xa] + ub * src[:, yb, xb]))
    return out


def test_upsample2x_closed_form_weights():
    rng = np.random.default_rng(3)
    for shape in ((2, 5, 7, 3), (1, 1, 1, 8), (3, 2, 9, 1), (1, 6, 1, 4)):
        src = rng.standard_normal(shape)
        assert np.max(np.abs(oracle.upsample2x(src) - _closed_form_2x(src))) < 1e-14


def test_upsample2x_keeps_constants_and_interior_affine_fields():
    H, W = 6, 9
    const = np.full((1, H, W, 2), 1.25)
    assert np.array_equal(oracle.upsample2x(const), np.full((1, 2 * H, 2 * W, 2), 1.25))
    yy, xx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    aff = (0.3 * xx - 0.7 * yy + 2.0)[None, ..., None]
    up = oracle.upsample2x(aff)[0, ..., 0]
    Y, X = np.meshgrid(np.arange(2 * H) + 0.5, np.arange(2 * W) + 0.5, indexing="ij")
    ref = 0.3 * (X / 2) - 0.7 * (Y / 2) + 2.0
    inner = (slice(1, 2 * H - 1), slice(1, 2 * W - 1))
    assert np.max(np.abs(up[inner] - ref[inner])) < 1e-12


def test_decode_volume_is_the_per_pixel_decode_in_band():
    rng = np.random.default_rng(5)
    L, H, W, C = 3, 2, 4, 8
    F = rng.standard_normal((L, H, W, C))
    ws, wd = rng.standard_normal(C), rng.standard_normal(C)
    Wc = rng.standard_normal((C, 3))
    near, far = 0.5, 20.0
    d, a, c = oracle.decode_volume(F, ws, wd, Wc, near, far)
    band = 1 / near - 1 / far
    for li in range(L):
        xs = F[li] @ ws
        assert np.max(np.abs(a[li] - 1 / (1 + np.exp(-xs)))) < 1e-14
        # layer li sits in its own disparity band of width band / L
        lo = 1 / far + band * (L - li - 1) / L
        assert np.all(1 / d[li] >= lo - 1e-12) and np.all(1 / d[li] <= lo + band / L + 1e-12)
    a1, d1, c1 = oracle.decode(F[1, 1, 2], ws, wd, Wc, 0.5, 1.0, 1, L, near, far, mode=1)
    assert (a1, d1) == (a[1, 1, 2], d[1, 1, 2]) and np.array_equal(c1, c[1, 1, 2])


def test_volume_logits_activate_to_the_decode():
    # the final LDM's unactivated attributes: sigmoid of the density logit is
    # the decoded alpha, and the paper's depth activation of the depth logit
    # is the decoded depth (decode_volume, pinned by the anchor bands)
    r = np.random.default_rng(8)
    L, H, W, C = 3, 2, 4, 8
    F = r.standard_normal((L, H, W, C))
    ws, wd, wc = r.standard_normal(C), r.standard_normal(C), r.standard_normal((C, 3))
    near, far = 0.5, 20.0
    dl, sl = oracle.volume_logits(F, ws, wd)
    d, a, _ = oracle.decode_volume(F, ws, wd, wc, near, far)
    np.testing.assert_allclose(1.0 / (1.0 + np.exp(-sl)), a, rtol=1e-14)
    band = 1.0 / near - 1.0 / far
    li = np.arange(L)[:, None, None]
    delta = (L - li - 0.5) / L
    np.testing.assert_allclose(1.0 / ((delta + 0.5 / L * np.tanh(dl)) * band + 1.0 / far), d,
                               rtol=1e-13)


def test_pipeline_with_zero_ray_projection_starts_from_the_init():
    # with every ray-encoding projection zero the encoded pyramid is the raw
    # one, and the first step's input state is the learned initialisation
    from paper_2411_16680_amd import synth
    pl = synth.make_pipeline(V=2, steps=(synth.ChainStep(2, 3, 5, 0, 1, False, False, False),),
                             feat_hw=((3, 5),), input_hw=(6, 10), dtype="f32", seed=4)
    pl.Wr = [np.zeros_like(w) for w in pl.Wr]
    outs, r, feats = oracle.run_pipeline(pl)
    for m in range(2):
        np.testing.assert_array_equal(feats[0][m], pl.chain.feats[0][m].astype(np.float64))
    F, d, a = oracle.ldm_init(2, 3, 5, pl.f0, pl.chain.near, pl.chain.far)
    np.testing.assert_array_equal(outs[0]["F_in"], F)
    np.testing.assert_array_equal(outs[0]["depth_in"], d)
    assert outs[0]["blend_logit"].shape == (2, 3, 5, 2)
    assert r["rgb"].shape == (6, 10, 3)
