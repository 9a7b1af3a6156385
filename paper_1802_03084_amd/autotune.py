"""Autotuner for the fused search's schedule.

The fused search's results do not depend on its schedule (the same arithmetic
runs per image), but its speed does: how many lane streams run batches
concurrently, and how large the row-transformed batches of all lanes are
(image pairs per batch).  `tune` times a set of candidate schedules on a plan
of the same shape over the first few DM trials (every DM trial costs the
same), applies the fastest to the plan with rf_plan_set_tuning, and caches the
choice per device and shape in a JSON file.

    from paper_1802_03084_amd import autotune
    lanes, budget, info = autotune.tune(plan, dvis, cache_path="tuning.json")
"""
import json
import os
import time

from . import RF_OP_SEGMENT

# (lanes, budget of all lanes' row-transformed batches in MB)
CANDIDATES = [(1, 240), (2, 120), (2, 240), (2, 320), (3, 240), (4, 240)]
# 2048^2 batches hold few image pairs at 240 MB: larger budgets are tried too
LARGE_IMAGE_CANDIDATES = [(2, 960), (2, 1920), (3, 1920)]


def shape_key(plan):
    return (f"N{plan.npix}-T{plan.nint}-B{plan.nbl}-C{plan.nchan}-P{plan.npol}-"
            f"D{plan.vis_dtype}-W{'.'.join(str(w) for w in plan.widths)}")


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _time(plan, vis, reps):
    import torch
    ws = plan.workspace(RF_OP_SEGMENT)
    plan.search_segment(vis, cap=4096, ws=ws, collect=False)  # warm: first use of the tuning
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        plan.search_segment(vis, cap=4096, ws=ws, collect=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    del ws
    return dt


def tune(plan, vis, ndm=8, candidates=None, cache_path=None, reps=2):
    """Picks and applies the fastest schedule for `plan` (segment `vis` on the
    device).  Returns (lanes, m_budget_mb, info) with info["cached"] True when
    the choice came from the cache, else the per-candidate seconds per DM.
    candidates: (lanes, budget MB) pairs; default CANDIDATES, plus
    LARGE_IMAGE_CANDIDATES for 2048^2 images."""
    if candidates is None:
        candidates = CANDIDATES + (LARGE_IMAGE_CANDIDATES if plan.npix >= 2048 else [])
    key = f"{_device_name()}|{shape_key(plan)}"
    cache = _load(cache_path)
    if key in cache:
        lanes, budget = cache[key]["lanes"], cache[key]["m_budget_mb"]
        plan.set_tuning(lanes, budget)
        return lanes, budget, {"cached": True}
    sub = plan.subplan(min(ndm, plan.ndm))
    per_dm = {}
    for lanes, budget in candidates:
        sub.set_tuning(lanes, budget)
        per_dm[(lanes, budget)] = _time(sub, vis, reps) / sub.ndm
    lanes, budget = min(per_dm, key=per_dm.get)
    plan.set_tuning(lanes, budget)
    if cache_path:
        cache[key] = {"lanes": lanes, "m_budget_mb": budget,
                      "seconds_per_dm": {f"{l}x{b}": round(v, 6) for (l, b), v in per_dm.items()}}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return lanes, budget, {"cached": False,
                           "seconds_per_dm": {f"{l}x{b}": v for (l, b), v in per_dm.items()}}
