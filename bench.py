"""Benchmark of the HDP hot path on one MI355X.

Workload: one synthetic 1344x1104 RGB pair with labels 0..255 (slanted planes,
shaped like the paper's full-size benchmark images), HDP with a 4-layer graph
pyramid (S=2, L=3), +-4 predicted window, beta=19/20, sigma=0.1.  One step =
the whole top-down loop, captured once as a HIP graph and replayed: pyramid,
then per layer interval prediction, disparity forest, restricted cost,
two-pass aggregation and WTA.  Inputs are resident in HBM before timing.

Prints one JSON line.  `value` is the algorithmic aggregation rate: the sum,
over the layers of one step and over their pixels, of the width of the
pixel's tree interval (the (pixel, label) entries the method aggregates),
divided by the step time, in Mpix*disp/s.  Beside it: the
full-range-equivalent rate N*(dmax+1)/step time, the per-layer search ratio,
the full-range MST path on the same pair (with the roofline of its passes),
the roofline of the dominant kernel (the fused up pass), the batched
workloads with their own rooflines,
the adjoint ratios, and the FP64 CPU oracle timed on the host together with
the label agreement between the two.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Rows of at least this many labels read the right image packed in 8 bytes a
# pixel in the fused up pass (kPackRightMinWidth in aggregate.hip).
PACK_RIGHT_MIN_WIDTH = 64
NEAR_TIE_REL = 1e-5



def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="both", choices=["both", "hdp", "full", "batched"],
                    help="profiling aid: time only the HDP loop, only the full-range path "
                         "or only the batched workloads")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and adjoint workloads (profiling aid)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in tile schedule")
    ap.add_argument("--parts", action="store_true",
                    help="also time every part of the HDP step as its own captured graph")
    ap.add_argument("--workload", default="all", choices=["all", "uneven32", "road64"],
                    help="profiling aid for --mode batched: run one batched workload only "
                         "(and not the adjoint workload)")
    return ap.parse_args()


def upload(pairs):
    import numpy as np
    import torch
    L = torch.from_numpy(np.concatenate([p.left.reshape(-1, 3) for p in pairs])).cuda()
    R = torch.from_numpy(np.concatenate([p.right.reshape(-1, 3) for p in pairs])).cuda()
    shapes = [(p.shape[0], p.shape[1], p.dmax) for p in pairs]
    return L, R, shapes


# --- byte models -------------------------------------------------------------------------

def layer_entries(forest) -> int:
    """Algorithmic (pixel, label) entries of one layer: the sum over pixels of the
    width of the pixel's tree interval (padding columns of the row layout excluded)."""
    import torch
    lo = forest.array("lo")
    hi = forest.array("hi")
    return int(torch.sum((hi - lo + 1).to(torch.int64)).item())


def pass_bytes_alg(forest, up: bool) -> float:
    """Algorithmic HBM bytes of one fused matching pass: 4 B per entry for the up
    pass (the cost is computed in place: write U), 8 B per entry for the down pass
    (read U, write the aggregated cost), 12 B of tree metadata per node and pass,
    and in the down pass 4 B per pixel for its label (the winner-takes-all is
    fused into it)."""
    e, n = layer_entries(forest), forest.n
    if up:
        return 4.0 * e + 12.0 * n
    return 8.0 * e + 12.0 * n + 4.0 * n


def pass_bytes_kernel(forest, up: bool) -> float:
    """Bytes the kernel's own data layout moves in one fused matching pass (rows
    of `width` labels, padding included): both passes read the previous-phase row
    of every chain head (4 B per label) and 21 B per row of coefficients and
    links; the up pass writes U (4 B per entry), reads the row's pixel, column and
    interval (12 B), its left and right image pixels (32 B; 24 B where the
    right image is read packed) and 8 B per light child; the down pass reads U
    and writes the aggregated volume (8 B per entry) and, for the fused
    winner-takes-all, the row's pixel and interval (8 B) and its label (4 B)."""
    import torch
    n, w = forest.n, forest.width
    heavy = forest.array("heavy")
    prow = forest.array("prow")
    heads = int(torch.count_nonzero((heavy == 0) & (prow >= 0)).item())
    common = 4.0 * heads * w + 21.0 * n
    if up:
        img = 16.0 + (8.0 if w >= PACK_RIGHT_MIN_WIDTH else 16.0)
        return common + 4.0 * n * w + (12.0 + img) * n + 8.0 * heads
    return common + 8.0 * n * w + 12.0 * n


def measured_traffic(workload: str):
    """HBM bytes per launch of the up and down passes from the committed counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain copy
    of known size), or None once the kernel's sources (the pass and the matching
    cost it inlines) have changed since."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "k_pass_traffic.json")))
        w = rec["workloads"][workload]
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return w


def pass_roofline(hdp, step_eager, reps=5):
    """HIP events around every up- and down-pass launch of `reps` eager runs of
    a step (on the launch's own stream); bytes from the forests of those runs."""
    out = {}
    for cls, up in (("up_pass", True), ("down_pass", False)):
        hdp.timer_arm(cls)
        for _ in range(reps):
            r = step_eager()
        ms, launches = hdp.timer_read()
        hdp.timer_arm(None)
        forests = [x.forest for x in r]
        alg = reps * sum(pass_bytes_alg(f, up) for f in forests)
        ker = reps * sum(pass_bytes_kernel(f, up) for f in forests)
        out[cls] = dict(secs=ms * 1e-3, launches=launches, alg=alg, ker=ker)
    return out


def roofline_entry(rec, kernel, traffic):
    secs, n = rec["secs"], rec["launches"]
    achieved = rec["alg"] / secs / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "launches": n, "avg_launch_us": secs / n * 1e6,
            "algorithmic_bytes_per_launch": rec["alg"] / n,
            "kernel_layout_bytes_per_launch": rec["ker"] / n,
            "kernel_layout_frac": rec["ker"] / secs / 1e9 / HBM_PEAK_GBS}


def rooflines(rl, traffic_key):
    tr = measured_traffic(traffic_key)
    up = roofline_entry(rl["up_pass"], "k_pass_s<up, fused cost> (leaf-to-root pass, cost "
                                       "computed in the pass)", tr and tr.get("up_pass"))
    down = roofline_entry(rl["down_pass"], "k_pass_s<down> (root-to-leaf pass, winner-takes-all "
                                           "fused)",
                          tr and tr.get("down_pass"))
    both = {k: rl["up_pass"][k] + rl["down_pass"][k] for k in ("secs", "launches", "alg", "ker")}
    b = roofline_entry(both, "k_pass_s, both passes", None)
    up["both_passes"] = {k: b[k] for k in ("achieved", "frac", "launches", "avg_launch_us",
                                           "algorithmic_bytes_per_launch")}
    up["down_pass"] = {k: down[k] for k in ("achieved", "frac", "traffic", "launches",
                                            "avg_launch_us", "algorithmic_bytes_per_launch")}
    return up


def per_layer_stats(res):
    """Per layer: pixels, label range, row width and the search ratio R_l =
    mean tree-interval width / (1 + d_l) (Section 4.2)."""
    out = []
    for r in res:
        f = r.forest
        e = layer_entries(f)
        d = max(s[2] for s in r.shapes)
        out.append({"layer": r.level, "pixels": f.n, "dmax": d, "row_width": f.width,
                    "entries": e, "search_ratio": e / f.n / (d + 1)})
    return out


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the box has one GPU "
                                   "and the multi-GPU path is not built (pairs would shard "
                                   "across GPUs with no collective); --gpus must be 1"}))
        sys.exit(2)
    # every input is drawn before the first GPU call (the host pool forks)
    from paper_1509_08197_amd import scenes
    pair = scenes.workload(2)
    extras = not args.no_extra and args.mode in ("both", "batched")
    if extras:
        scenes.prefetch({"all": [3, 4, 5], "uneven32": [3], "road64": [5]}[args.workload])

    import torch

    from paper_1509_08197_amd import hdp

    torch.cuda.set_device(0)
    Hh, Ww = pair.shape
    dmax = pair.dmax
    shapes = [(Hh, Ww, dmax)]
    P = scenes.HDP_PARAMS[2]
    L_rgb = torch.from_numpy(pair.left.reshape(-1, 3).copy()).cuda()
    R_rgb = torch.from_numpy(pair.right.reshape(-1, 3).copy()).cuda()
    N = Hh * Ww

    def hdp_eager(ws=None):
        return hdp.hdp_stereo(L_rgb, R_rgb, shapes, S=P["S"], L=P["L"], window=P["window"],
                              beta=P["beta"], ws=ws)

    def full_eager(ws=None):
        return hdp.full_range(L_rgb, R_rgb, shapes, ws=ws)

    nan = float("nan")
    out = {"metric": "aggregated Mpix*disp/s (algorithmic: per-pixel tree-interval widths "
                     "summed over the layers of the HDP step, single pair)",
           "value": nan, "unit": "Mpix*disp/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": nan, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "single pair 1344x1104 RGB, labels 0..255, HDP pyramid "
                                  "L=3 S=2, window 4, beta 19/20, sigma 0.1",
                      "global_batch": 1}}

    from paper_1509_08197_amd import tuner
    hdp_sched = full_sched = None
    if not args.no_tune and args.mode in ("both", "hdp", "full"):
        # schedules picked by timing whole captured steps (one width at a time)
        probe = hdp_eager()
        widths = sorted({r.forest.width for r in probe}, key=lambda w: -sum(
            r.forest.n for r in probe if r.forest.width == w))
        del probe
        if args.mode != "full":
            hdp_sched = tuner.tune_step(hdp_eager, widths)
        if args.mode != "hdp":
            full_sched = tuner.tune_step(full_eager, [dmax + 1])
        out["schedule"] = {"hdp": {str(k): v for k, v in (hdp_sched or {}).items()},
                           "full_range": {str(k): v for k, v in (full_sched or {}).items()}}
        torch.cuda.empty_cache()

    def use(sched):
        for wdt, s in (sched or {}).items():
            hdp.set_schedule(wdt, *(int(x) for x in s.split("x")))

    res = None
    if args.mode in ("both", "hdp"):
        # the timed step is a whole-step HIP graph replay (captured once)
        use(hdp_sched)
        step = hdp.CapturedStep(hdp_eager)
        t_hdp = timed(step.replay, args.steps, args.warmup)
        del step
        res = hdp_eager()
        torch.cuda.synchronize()
        layers = per_layer_stats(res)
        alg = sum(x["entries"] for x in layers)
        padded = sum(r.forest.n * r.forest.width for r in res)
        out["value"] = alg / t_hdp / 1e6
        out["ms_per_step"] = t_hdp * 1e3
        out["hdp_algorithmic"] = {
            "entries_per_step": int(alg), "padded_entries_per_step": int(padded),
            "full_range_equivalent_Mpix_disp_per_s": N * (dmax + 1) / t_hdp / 1e6,
            "search_ratio_vs_full": alg / (N * (dmax + 1)), "layers": layers}
        out["roofline"] = rooflines(pass_roofline(hdp, hdp_eager), "hdp_1344x1104")
        out["roofline"]["working_set_MB"] = working_set_mb(res)
        if args.parts:
            out["parts_us"] = time_parts(hdp, L_rgb, R_rgb, shapes, P, res)

    if args.mode in ("both", "full"):
        use(full_sched)
        fstep = hdp.CapturedStep(full_eager)
        t_full = timed(fstep.replay, max(2, args.steps // 4), 1)
        out["full_range"] = {"ms_per_step": t_full * 1e3,
                             "Mpix_disp_per_s": N * (dmax + 1) / t_full / 1e6}
        if args.mode == "both":
            out["full_range"]["speedup_hdp_over_full"] = t_full / (out["ms_per_step"] * 1e-3)
        del fstep
        # the full-range step runs the same fused passes on one 256-label layer
        out["full_range"]["roofline"] = rooflines(
            pass_roofline(hdp, lambda: [full_eager()], reps=3), "full_1344x1104")

    if extras:
        use(hdp_sched)
        out["batched"] = bench_batched(hdp, scenes, args)
        if args.workload == "all":
            out["adjoint"] = bench_adjoint(hdp, scenes, args)

    if not args.no_cpu_baseline and args.mode == "both":
        from oracle import oracle
        t0 = time.perf_counter()
        ores = oracle.hdp_stereo(pair.left, pair.right, dmax, S=P["S"], L=P["L"],
                                 window=P["window"], beta=P["beta"])
        t_cpu = time.perf_counter() - t0
        alg_cpu = sum(x["entries"] for x in out["hdp_algorithmic"]["layers"])
        out["cpu_baseline"] = {"value": alg_cpu / t_cpu / 1e6, "unit": "Mpix*disp/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "one whole HDP step of the same 1344x1104 pair "
                                         "(FP64, single-threaded C), same algorithmic entries",
                               "seconds": t_cpu,
                               "host_cores_available": len(os.sched_getaffinity(0))}
        out["parity"] = label_agreement(res, ores)
    print(json.dumps(out))


def working_set_mb(res):
    """Bytes the fused passes of one step touch (images, U and aggregated
    volumes, forest rows), to compare with the 256 MB last-level cache."""
    tot = 0
    for r in res:
        f = r.forest
        tot += 2 * 4 * f.n * f.width + 2 * 16 * f.n + 48 * f.n
    return tot / 1e6


def label_agreement(res, ores):
    """Per layer: labels that differ between the GPU step and the FP64 oracle's
    step, and the oracle's near-ties (two best aggregated costs within 1e-5)."""
    import numpy as np
    out = []
    for l, r in enumerate(res):
        g = r.disp.cpu().numpy()
        o = ores[l]["disp"].ravel()
        c1, c2 = ores[l]["c1"], ores[l]["c2"]
        near = (c2 - c1) <= NEAR_TIE_REL * np.abs(c1)
        out.append({"layer": l, "label_differences": int((g != o).sum()),
                    "oracle_near_ties": int(near.sum()),
                    "differences_at_near_ties": int(((g != o) & near).sum())})
    return out


def time_parts(hdp, L_rgb, R_rgb, shapes, P, res):
    """Every part of the HDP step captured as its own graph and replayed (us)."""
    S, L, w, beta = P["S"], P["L"], P["window"], P["beta"]
    lv = hdp.level_shapes(shapes, S, L)
    lp, rp = hdp.pyramid_views(L_rgb, R_rgb, shapes, S, L)
    parts = {}

    def t(name, fn):
        g = hdp.CapturedStep(fn)
        parts[name] = timed(g.replay, 20, 3) * 1e6

    t("pyramid", lambda ws: hdp.pyramid_views(L_rgb, R_rgb, shapes, S, L))
    for l in range(L, -1, -1):
        f = res[l].forest
        if l < L:
            mw = min(S + 2 * w, max(d for _, _, d in lv[l]) + 1)
            t(f"layer{l}_predict_range",
              lambda ws, l=l: hdp.predict_range(res[l + 1].disp, lv[l + 1], lv[l], S, w))
            t(f"layer{l}_tree", lambda ws, l=l, mw=mw: hdp.build_tree(
                lp[l], lv[l], l, res[l].pix_lo, res[l].pix_hi, max_width=mw, beta=beta,
                ws=ws["tree"], level_order=False))
        else:
            t(f"layer{l}_tree", lambda ws, l=l: hdp.build_tree(lp[l], lv[l], l, ws=ws["tree"],
                                                               level_order=False))
        t(f"layer{l}_matching", lambda ws, l=l, f=f: hdp.match_layer(lp[l], rp[l], lv[l], f,
                                                                   ws=ws["agg"]))
    return parts


def bench_batched(hdp, scenes, args):
    """Uneven batches in one captured graph: 32 pairs (320-1392 x 240-1110,
    64-256 labels) HDP forward; 64 road pairs 1242x375 HDP forward and forward +
    adjoint.  Each with the roofline of its fused passes (eager runs)."""
    import torch
    res = {}
    if args.workload in ("all", "uneven32"):
        res["uneven32_hdp_fwd"] = bench_uneven32(hdp, scenes, args)
    if args.workload in ("all", "road64"):
        res["road64_hdp_fwd_bwd"] = bench_road64(hdp, scenes, args)
    return res


def bench_uneven32(hdp, scenes, args):
    """32 uneven pairs (320-1392 x 240-1110, 64-256 labels), HDP forward."""
    import torch
    pairs = scenes.workload_batch(3)
    L, R, shapes = upload(pairs)
    P3 = scenes.HDP_PARAMS[3]

    def step3(ws=None):
        return hdp.hdp_stereo(L, R, shapes, S=P3["S"], L=P3["L"], window=P3["window"],
                              beta=P3["beta"], ws=ws)
    g3 = hdp.CapturedStep(step3)
    t3 = timed(g3.replay, max(3, args.steps // 2), 2)
    del g3
    r3 = step3()
    torch.cuda.synchronize()
    alg3 = sum(layer_entries(r.forest) for r in r3)
    full3 = sum(h * w * (d + 1) for h, w, d in shapes)
    res = {
        "pairs": len(shapes), "Mpix": sum(h * w for h, w, _ in shapes) / 1e6,
        "ms_per_step": t3 * 1e3, "Mpix_disp_per_s": alg3 / t3 / 1e6,
        "entries_per_step": alg3,
        "Mpix_disp_per_s_full_range_equiv": full3 / t3 / 1e6,
        "layers": per_layer_stats(r3),
        "roofline": rooflines(pass_roofline(hdp, step3, reps=3), "uneven32")}
    res["roofline"]["working_set_MB"] = working_set_mb(r3)
    del r3, L, R
    torch.cuda.empty_cache()
    return res


def bench_road64(hdp, scenes, args):
    """64 road pairs 1242x375, labels 0..191: HDP forward, and forward +
    adjoint (against the fused forward and the forward keeping its volumes)."""
    import torch
    pairs = scenes.workload_batch(5)
    L, R, shapes = upload(pairs)
    P5 = scenes.HDP_PARAMS[5]
    full5 = sum(h * w * (d + 1) for h, w, d in shapes)
    probe = hdp.hdp_stereo(L, R, shapes, S=P5["S"], L=P5["L"], window=P5["window"],
                           beta=P5["beta"], keep=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    G = [torch.randn(r.agg.shape, device="cuda", generator=gen) for r in probe]
    del probe

    def fwd5(ws=None):  # what the loop runs: fused matching
        return hdp.hdp_stereo(L, R, shapes, S=P5["S"], L=P5["L"], window=P5["window"],
                              beta=P5["beta"], ws=ws)

    def fwd5_keep(ws=None):  # cost and aggregated volumes kept for the adjoint
        return hdp.hdp_stereo(L, R, shapes, S=P5["S"], L=P5["L"], window=P5["window"],
                              beta=P5["beta"], keep=True, ws=ws)

    def fwdbwd5(ws=None):
        out = fwd5_keep(ws)
        agg_ws = ws["agg"] if ws else None
        grads = [hdp.aggregate_backward(r.forest, r.cost, r.agg, G[i], 0.1, want_w=False,
                                        ws=agg_ws) for i, r in enumerate(out)]
        return out, grads
    times = {}
    for name, fn in (("fwd", fwd5), ("fwd_keep", fwd5_keep), ("fwd_bwd", fwdbwd5)):
        g = hdp.CapturedStep(fn)
        times[name] = timed(g.replay, max(3, args.steps // 2), 2)
        del g
    r5 = fwd5()
    torch.cuda.synchronize()
    alg5 = sum(layer_entries(r.forest) for r in r5)
    res = {
        "pairs": len(shapes), "Mpix": sum(h * w for h, w, _ in shapes) / 1e6,
        "fwd_ms": times["fwd"] * 1e3, "fwd_keep_ms": times["fwd_keep"] * 1e3,
        "fwd_bwd_ms": times["fwd_bwd"] * 1e3,
        "fwd_bwd_over_fwd": times["fwd_bwd"] / times["fwd"],
        "fwd_bwd_over_fwd_keep": times["fwd_bwd"] / times["fwd_keep"],
        "Mpix_disp_per_s_fwd": alg5 / times["fwd"] / 1e6, "entries_per_step": alg5,
        "Mpix_disp_per_s_full_range_equiv_fwd": full5 / times["fwd"] / 1e6,
        "layers": per_layer_stats(r5),
        "roofline": rooflines(pass_roofline(hdp, fwd5, reps=3), "road64")}
    res["roofline"]["working_set_MB"] = working_set_mb(r5)
    del r5, L, R
    torch.cuda.empty_cache()
    return res


def bench_adjoint(hdp, scenes, args):
    """8 pairs 640x480, labels 0..127, full-range forest: aggregation forward
    vs forward + adjoint (dL/dC, dL/dw, dL/dsigma; U kept as the checkpoint)."""
    import torch
    pairs = scenes.workload_batch(4)
    L, R, shapes = upload(pairs)
    lp = hdp.pyramid(L, shapes, 2, 0)
    rp = hdp.pyramid(R, shapes, 2, 0)
    f = hdp.build_tree(lp[0], shapes, 0)
    cost = hdp.cost_volume(lp[0], rp[0], shapes, f)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    g = torch.randn(cost.shape, device="cuda", generator=gen)

    def fwd(ws=None):
        return hdp.aggregate(f, cost, 0.1, keep_up=True, ws=ws["agg"] if ws else None)

    def fwdbwd(ws=None):
        agg, up = fwd(ws)
        return hdp.aggregate_backward(f, cost, agg, g, 0.1, up=up, want_w=True,
                                      ws=ws["agg"] if ws else None)
    a = hdp.CapturedStep(fwd)
    ta = timed(a.replay, max(3, args.steps // 2), 2)
    del a
    b = hdp.CapturedStep(fwdbwd)
    tb = timed(b.replay, max(3, args.steps // 2), 2)
    del b
    entries = f.n * f.width
    return {"workload": "8 pairs 640x480, labels 0..127, full range", "entries": int(entries),
            "fwd_ms": ta * 1e3, "fwd_bwd_ms": tb * 1e3, "fwd_bwd_over_fwd": tb / ta,
            "fwd_GBs_at_16B_per_entry": 16.0 * entries / ta / 1e9}


if __name__ == "__main__":
    main()
