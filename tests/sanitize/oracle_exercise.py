"""Runs the oracle's steps on small inputs with the library at the path
given on the command line (a build under the address and undefined-behaviour
sanitizers); numpy and ctypes only.  Prints "oracle ok" when every call
returned."""

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
from paper_2411_16680_amd import synth  # noqa: E402

oracle._LIB_PATH = sys.argv[1]
oracle._lib = None
oracle.lib()

sc = synth.make_custom(V=3, H=5, W=9, C=16, L=3, seed=3, with_target=True)
lvl = sc.levels[0]
for attn in (0, 1):
    oracle.update_fuse(sc.in_cams, sc.novel, sc.near, sc.far, lvl, attn_form=attn,
                       want_samples=True, want_logits=True)
oracle.run_level(sc, lvl, steps=2, rows=[0, 4])
sc4 = synth.make_custom(V=2, H=3, W=7, C=32, L=2, heads=4, head_dim=8, seed=5)
oracle.update_fuse(sc4.in_cams, sc4.novel, sc4.near, sc4.far, sc4.levels[0], attn_form=1)
G = np.random.default_rng(1).standard_normal((lvl.H, lvl.W, 3))
oracle.update_fuse_backward(sc.in_cams, sc.novel, sc.near, sc.far, lvl, d_rgb=G)
c = np.random.default_rng(2).uniform(0, 1, (4, 6, 3))
a = np.random.default_rng(3).uniform(0, 1, (4, 6))
oracle.composite(c, a)
oracle.composite(c, a, back_to_front=True)
oracle.composite_backward(c, a, np.ones((6, 3)), np.ones(6))
rs = synth.make_render(V=2, W=12, H=8, s=2, L=2, img_hw=(9, 14), seed=4)
oracle.render_ibr(rs.in_cams, rs.images, rs.novel, rs.near, rs.far, *rs.logits, rs.H, rs.W)
oracle.render_to_views(sc.in_cams[:2], sc.novel, np.full((2, 4, 6), 2.0), np.full((2, 4, 6), 0.5),
                       np.full((2, 4, 6, 3), 0.3), [(5, 7), (6, 8)])
F = np.random.default_rng(5).standard_normal((2, 4, 5, 8))
Wc = np.random.default_rng(6).standard_normal((3, 3, 8, 8)) * 0.1
oracle.residual_conv(F, Wc, Wc)
oracle.layer_collapse(F, np.random.default_rng(7).standard_normal((16, 8)),
                      np.random.default_rng(8).standard_normal((8, 8)))
Wr = np.random.default_rng(9).standard_normal((32, 8))
oracle.ray_encoding(sc.in_cams[0], sc.novel, sc.near, sc.far, Wr, 4, 6)
oracle.upsample2x(F)
print("oracle ok", flush=True)
