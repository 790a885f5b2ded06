"""The benchmark's command-line contract that needs no GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.lstrip().startswith("{")


def test_roofline_work_counts_follow_the_attention_form():
    """The algorithmic FLOPs the roofline divides by: the standard form's
    projections on MFMA, or the one-to-many form's two folded projections
    plus its per-view dot products and weighted sums; the headline's
    attention picks the one-to-many form on one-head levels, as the runner
    does."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2411_16680_amd import runner, synth
    sc = synth.make_inputs(1)
    lvl = sc.levels[0]
    N, C, V = lvl.L * lvl.H * lvl.W, lvl.C, sc.V
    assert lvl.heads == 1 and lvl.head_dim == C
    assert bench.level_flops(lvl, V) == 2 * N * (C * C + 2 * V * lvl.Cf * C + C * C)
    assert bench.level_flops(lvl, V, "folded") == 2 * N * (2 * C * C) + 4 * N * V * lvl.Cf
    assert bench.level_form(lvl) == "folded" == runner.step_form(bench.HEADLINE_ATTN, lvl)
