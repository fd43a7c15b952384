"""Benchmark of the HDP hot path on one MI355X.

Workload: one synthetic 1344x1104 RGB pair with labels 0..255 (slanted planes,
shaped like the paper's full-size benchmark images), HDP with a 4-layer graph
pyramid (S=2, L=3), +-4 predicted window, beta=19/20, sigma=0.1.  One step =
the whole top-down loop: pyramid, then per layer interval prediction,
disparity forest, restricted cost, two-pass aggregation and WTA.

Prints one JSON line.  `value` is the full-range-equivalent throughput
N*(dmax+1)/step_time in Mpix*disp/s (the rate at which disparity maps of this
size and range are produced); the full-range MST baseline on the same pair is
reported beside it.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="both", choices=["both", "hdp", "full"],
                    help="profiling aid: time only the HDP loop or only the full-range path")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1509_08197_amd import hdp, scenes

    torch.cuda.set_device(0)
    pair = scenes.workload(2)
    Hh, Ww = pair.shape
    dmax = pair.dmax
    shapes = [(Hh, Ww, dmax)]
    P = scenes.HDP_PARAMS[2]
    L_rgb = torch.from_numpy(pair.left.reshape(-1, 3).copy()).cuda()
    R_rgb = torch.from_numpy(pair.right.reshape(-1, 3).copy()).cuda()
    N = Hh * Ww

    def hdp_step():
        return hdp.hdp_stereo(L_rgb, R_rgb, shapes, S=P["S"], L=P["L"], window=P["window"],
                              beta=P["beta"])

    def full_step():
        return hdp.full_range(L_rgb, R_rgb, shapes)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_hdp = timed(hdp_step, args.steps, args.warmup) if args.mode != "full" else float("nan")
    t_full = (timed(full_step, max(2, args.steps // 4), 1) if args.mode != "hdp"
              else float("nan"))

    res = hdp_step()
    torch.cuda.synchronize()
    alg_entries = sum(r.forest.n * r.forest.width for r in res)
    out = {
        "metric": "aggregated Mpix*disp/s (full-range-equivalent, HDP single pair)",
        "value": N * (dmax + 1) / t_hdp / 1e6,
        "unit": "Mpix*disp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_hdp * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single pair 1344x1104, labels 0..255, HDP L=3 S=2 w=4 beta=19/20",
                   "global_batch": 1},
        "full_range": {"ms_per_step": t_full * 1e3,
                       "value": N * (dmax + 1) / t_full / 1e6,
                       "speedup_hdp_over_full": t_full / t_hdp},
        "hdp_algorithmic_entries": int(alg_entries),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
