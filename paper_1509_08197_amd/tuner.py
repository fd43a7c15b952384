"""Autotuner of the aggregation tile schedule.

For a row width (labels per row) the aggregation passes can map 1, 2 or 4
consecutive labels to a thread and 4, 8 or 16 rows to a thread group; the best
choice depends on the width, on the forest (chain lengths, phase sizes) and on
the device.  ``tune`` times every valid schedule on a real forest and cost
volume of that width (HIP events around the whole aggregation) and keeps the
fastest; results are cached in a JSON file keyed by device name, width and
size class (log2 of the row count), and ``apply_cache`` installs them.
``tune_step`` instead times a whole captured step (HIP graph replays) for
each candidate, one width at a time, which also accounts for the schedule's
effect on the kernels around the aggregation.
"""

from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional

import torch

from . import hdp

CANDIDATES = [(4, 4), (4, 8), (2, 4), (2, 8), (2, 16), (1, 4), (1, 8)]


def cache_path() -> str:
    return os.environ.get("HDP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hdp_mi355x",
                                       "schedule.json"))


def _device_key() -> str:
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace(" ", "_")


def size_class(n: int) -> int:
    return int(math.log2(max(1, n)))


def valid(width: int, cpt: int, rpg: int) -> bool:
    return width % cpt == 0 and (rpg != 16 or cpt == 2)


def load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(cache: Dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    with open(p + ".tmp", "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(p + ".tmp", p)


def tune(forest: "hdp.Forest", cost: torch.Tensor, sigma: float = 0.1, reps: int = 3,
         cache: Optional[Dict] = None) -> Dict:
    """Time every valid schedule for forest.width on this forest; returns the
    entry {cpt, rpg, us, all} and records it in the cache (not saved)."""
    width = forest.width
    ws = hdp.Workspace()
    out = torch.empty_like(cost)
    times = {}
    for cpt, rpg in CANDIDATES:
        if not valid(width, cpt, rpg):
            continue
        hdp.set_schedule(width, cpt, rpg)
        hdp.aggregate(forest, cost, sigma, out=out, ws=ws)  # warm-up
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            hdp.aggregate(forest, cost, sigma, out=out, ws=ws)
        ev1.record()
        torch.cuda.synchronize()
        times[f"{cpt}x{rpg}"] = ev0.elapsed_time(ev1) * 1e3 / reps
    best = min(times, key=times.get)
    cpt, rpg = (int(x) for x in best.split("x"))
    hdp.set_schedule(width, cpt, rpg)
    entry = {"cpt": cpt, "rpg": rpg, "us": times[best], "all": times}
    if cache is not None:
        cache.setdefault(_device_key(), {})[f"{width}:{size_class(forest.n)}"] = entry
    return entry


def tune_step(step, widths, replays: int = 10, rounds: int = 3) -> Dict[int, str]:
    """Coordinate search over the schedules of the given widths (in order),
    timing graph replays of ``step`` (a function of a workspace dict, as for
    ``hdp.CapturedStep``).  Leaves the best schedules installed; returns
    {width: "CPTxRPG"}."""
    chosen: Dict[int, str] = {}
    for width in widths:
        times = {}
        for cpt, rpg in CANDIDATES:
            if not valid(width, cpt, rpg):
                continue
            hdp.set_schedule(width, cpt, rpg)
            g = hdp.CapturedStep(step)
            best = float("inf")
            for _ in range(rounds):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record()
                for _ in range(replays):
                    g.replay()
                ev1.record()
                torch.cuda.synchronize()
                best = min(best, ev0.elapsed_time(ev1) / replays)
            times[f"{cpt}x{rpg}"] = best
            del g
        pick = min(times, key=times.get)
        cpt, rpg = (int(x) for x in pick.split("x"))
        hdp.set_schedule(width, cpt, rpg)
        chosen[width] = pick
    return chosen


def apply_cache(cache: Optional[Dict] = None) -> int:
    """Install cached schedules for this device (largest size class per width).
    Returns the number of widths set."""
    cache = load() if cache is None else cache
    dev = cache.get(_device_key(), {})
    best: Dict[int, tuple] = {}
    for key, e in dev.items():
        w, sc = (int(x) for x in key.split(":"))
        if w not in best or sc > best[w][0]:
            best[w] = (sc, e["cpt"], e["rpg"])
    for w, (_, cpt, rpg) in best.items():
        hdp.set_schedule(w, cpt, rpg)
    return len(best)
