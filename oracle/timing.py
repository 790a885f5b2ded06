"""Timing of the FP64 oracle on the host's cores.  This is test
infrastructure, like the rest of this package, and never part of the
product path.

Cases, each the median of ``repeats`` runs:
  * tiny: two views, 64x48, C=16, L=4, one step and the composite;
  * 480x270: four views, C=32, L=16, two steps and the composite;
  * each level of the 1080p eight-view pyramid (C=64/32/16/8,
    L=32/16/8/4), one step each, the composite on the finest;
  * 960x540: four views, C=16, L=8, the forward step and composite, then
    the adjoint of sum((rgb - target)^2).

Every case runs in full on all threads.  On one thread the large cases
time 1 row and H/16 rows and fit a per-call part plus a per-row part: the oracle
marshals a level's maps to float64 once per call and splits the
layer-pixels over threads in small chunks, so the per-row part is linear
in the rows.  The whole case is then the per-call part plus the per-row
part times H.  Rates are layer-pixel-views per second (L*H*W*V per step).

    python -m oracle.timing [--repeats 3] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import time

import numpy as np

from . import num_threads, run_level, set_num_threads, update_fuse_backward


def _median(fn, repeats: int) -> float:
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts)


def fit_rows(H: int):
    """The two row sets of a fitted timing: one middle row, and H/16 (at
    least 3) evenly spaced rows, enough that the per-row part stands well
    above the timing noise of the per-call part."""
    n = max(3, H // 16)
    return [H // 2], sorted(set(np.linspace(0, H - 1, n).round().astype(int).tolist()))


def fitted_time(t_small: float, n_small: int, t_big: float, n_big: int, H: int) -> float:
    """A per-call part plus a per-row part, fitted to two timed calls on
    n_small < n_big rows, evaluated at H rows."""
    if n_big <= n_small:
        return t_big / n_big * H
    per_row = max(0.0, (t_big - t_small) / (n_big - n_small))
    return max(0.0, t_small - per_row * n_small) + per_row * H


def _fitted(fn_rows, H: int, repeats: int) -> float:
    small, big = fit_rows(H)
    t_small = _median(lambda: fn_rows(small), repeats)
    t_big = _median(lambda: fn_rows(big), repeats)
    return fitted_time(t_small, len(small), t_big, len(big), H)


def _cases():
    from paper_2411_16680_amd import synth
    out = []
    sc1 = synth.make_inputs(1)
    out.append(("tiny 64x48 V2 C16 L4", sc1, [(sc1.levels[0], 1)], None))
    sc2 = synth.make_inputs(2)
    out.append(("480x270 V4 C32 L16, 2 steps", sc2, [(sc2.levels[0], 2)], None))
    sc3 = synth.to_bf16(synth.make_inputs(3))
    for i, lvl in enumerate(sc3.levels):
        out.append((f"1080p pyramid level {i}: {lvl.W}x{lvl.H} V8 C{lvl.C} L{lvl.L}",
                    sc3, [(lvl, 1)], None))
    sc4 = synth.make_inputs(4, "f32")
    out.append(("960x540 V4 C16 L8, forward + adjoint", sc4, [(sc4.levels[0], 1)], sc4.target))
    return out


def _run(scene, lvl, steps, target, rows):
    res = run_level(scene, lvl, steps=steps, rows=rows)
    if target is not None:
        t = target if rows is None else target[rows]
        d_rgb = np.zeros((lvl.H, lvl.W, 3))
        sel = slice(None) if rows is None else rows
        d_rgb[sel] = 2.0 * (res["rgb"] - t)
        update_fuse_backward(scene.in_cams, scene.novel, scene.near, scene.far, lvl,
                             d_rgb=d_rgb, rows=rows)


def time_cases(repeats: int = 3, one_thread: bool = True):
    threads = num_threads()
    rows_out = []
    for name, scene, parts, target in _cases():
        (lvl, steps), = parts
        lpv = float(lvl.L) * lvl.H * lvl.W * len(scene.in_cams) * steps
        t_all = _median(lambda: _run(scene, lvl, steps, target, None), repeats)
        entry = {"case": name, "threads": threads, "s": t_all, "lpv_per_s": lpv / t_all}
        if one_thread:
            set_num_threads(1)
            try:
                if lvl.H <= 64:
                    t1 = _median(lambda: _run(scene, lvl, steps, target, None), repeats)
                    how = "full"
                else:
                    t1 = _fitted(lambda rows: _run(scene, lvl, steps, target, rows),
                                 lvl.H, repeats)
                    how = f"fitted from 1 and {len(fit_rows(lvl.H)[1])} rows"
            finally:
                set_num_threads(threads)
            entry.update({"s_one_thread": t1, "lpv_per_s_one_thread": lpv / t1,
                          "one_thread_how": how})
        rows_out.append(entry)
        print(json.dumps(entry), flush=True)
    return rows_out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--no-one-thread", action="store_true")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    res = time_cases(args.repeats, not args.no_one_thread)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    print(f"\nhost: {model}, {usable} usable cores, oracle threads {num_threads()}")
    print("| case | s (all threads) | layer-pixel-views/s | s (1 thread) | 1 thread |")
    print("|---|---|---|---|---|")
    for e in res:
        print(f"| {e['case']} | {e['s']:.3g} | {e['lpv_per_s']:.3g} | "
              f"{e.get('s_one_thread', float('nan')):.3g} | {e.get('one_thread_how', '-')} |")
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"host": model, "usable_cpus": usable, "cases": res}, f, indent=1)


if __name__ == "__main__":
    main()
