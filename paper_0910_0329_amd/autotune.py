"""Autotuner of the regrouped launch.  For a workload it times short batched
runs on the device and picks, in three stages:

1. the regrouping schedule, block shape, table placement (LDS or device
   memory, wave-stack schedule only) and chunk size (queues only; it also
   sizes them: 3 x lanes x chunk_per_lane records);
2. the occupancy of the winner: workgroups per CU (and so waves per CU) from
   one up to the number the device holds at once, as grid_blocks;
3. the wave-schedule thresholds.

The choice is cached per device and workload shape in a JSON file.  The
search times a scaled-down copy of the workload (every item's history count
divided by `scale`, at least `min_hist`), so a tuning pass costs a few
seconds; the result depends only on timing, never on the dose, because every
option runs the same histories.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

DEFAULT_SPACE = {
    "regroup": (1, 2, 3),
    "chunk_per_lane": (8, 16, 32, 64),
    "block_size": (256, 512),
    "table_placement": (1, 2),          # MCD_TABLES_LDS, MCD_TABLES_GLOBAL
}
# third stage, searched around the best launch options: the wave-stack
# schedule's thresholds (regroup 3: fetch_div holds in electron mode,
# fetch_photon_div in photon mode, photon_div sets the mode switch)
SCHED_SPACE = {
    "sched_fetch_div": (8, 16),
    "sched_fetch_photon_div": (2, 3),
    "sched_hard_div": (24, 64),
    "sched_photon_div": (1,),
}
CACHE_ENV = "MCDOSE_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "mcdose_autotune.json")


def workload_key(device_name: str, n_vox: int, items) -> str:
    """Device, phantom size and the mix of sources (particle kinds and the
    order of magnitude of the history counts)."""
    kinds = sorted({(int(s.particle), int(s.energy_kind)) for s, _, _ in items})
    tot = sum(int(n) for _, n, _ in items)
    mag = len(str(max(tot, 1)))
    raw = json.dumps([device_name, int(n_vox), kinds, len(items), mag])
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: str | None = None):
    path = path or cache_path()
    d = load_cache(path)
    d[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(space=None):
    """Every combination of the values in `space`, except that chunk_per_lane
    only matters with queues (regroup 1) and table_placement only with wave
    stacks (regroup 3): other schedules keep their first value."""
    space = space or DEFAULT_SPACE
    names = sorted(space)
    for combo in itertools.product(*(space[n] for n in names)):
        d = dict(zip(names, combo))
        if d.get("regroup") in (2, 3) and "chunk_per_lane" in space and \
                d["chunk_per_lane"] != space["chunk_per_lane"][0]:
            continue
        if d.get("regroup") in (1, 2) and "table_placement" in space and \
                d["table_placement"] != space["table_placement"][0]:
            continue
        yield d


def occupancy_candidates(shape: dict):
    """grid_blocks for one up to one fewer than the workgroups a CU holds at
    once (the default grid fills the device, so it is already timed), from
    the launch shape of mcd_launch_shape; none for kernels without the
    occupancy figure."""
    per_cu = int(shape.get("resident_per_cu", 0))
    return [{"grid_blocks": shape["cu_count"] * k} for k in range(1, per_cu)]


def scaled(items, scale: int, min_hist: int):
    return [(s, max(min_hist, int(n) // scale), k) for s, n, k in items]


def tune(eng, phantom: int, n_vox: int, items, seed: int, *, space=None, sched_space=None,
         occupancy: bool = True, scale: int = 8, min_hist: int = 2000, reps: int = 2,
         use_cache: bool = True, path: str | None = None, device_name: str | None = None, log=None) -> dict:
    """Returns the fastest launch options for `items` (sequence of (source,
    n_histories, request_key)) on `phantom`, from the cache when present.
    Stage 1 searches `space` (regrouping, block shape, table placement);
    stage 2 the workgroups per CU of the stage-1 winner (`occupancy`);
    stage 3 `sched_space` (wave-schedule thresholds) around the best so far;
    an empty `sched_space` ({}) skips stage 3."""
    import torch

    if device_name is None:
        p = torch.cuda.get_device_properties(eng.device)
        device_name = f"{p.name}/{getattr(p, 'gcnArchName', '')}/{p.multi_processor_count}"
    key = workload_key(device_name, n_vox, items)
    if use_cache:
        hit = load_cache(path).get(key)
        if hit and "opts" in hit:
            return dict(hit["opts"])
    probe = scaled(items, scale, min_hist)
    n_probe = sum(n for _, n, _ in probe)
    results = []
    stage2 = SCHED_SPACE if sched_space is None else sched_space
    trials = list(candidates(space))
    for opts in trials:
        results.append(_time(eng, phantom, n_vox, probe, n_probe, seed, opts, reps, log))
    results = [r for r in results if r]
    if not results:
        raise RuntimeError("autotune: no candidate ran")
    results.sort(key=lambda t: t[0])
    if occupancy:
        base = results[0][1]
        for extra in occupancy_candidates(eng.launch_shape(phantom, **base)):
            r = _time(eng, phantom, n_vox, probe, n_probe, seed, {**base, **extra}, reps, log)
            if r:
                results.append(r)
        results.sort(key=lambda t: t[0])
    if stage2:
        base = results[0][1]
        for extra in candidates(stage2):
            r = _time(eng, phantom, n_vox, probe, n_probe, seed, {**base, **extra}, reps, log)
            if r:
                results.append(r)
        results.sort(key=lambda t: t[0])
    best_t, best_opts = results[0]
    entry = {"opts": best_opts, "hist_per_s": n_probe / best_t, "probe_histories": n_probe,
             "device": device_name, "n_vox": int(n_vox), "n_items": len(items),
             "table": [{"opts": o, "hist_per_s": n_probe / t} for t, o in results]}
    store_cache(key, entry, path)
    return dict(best_opts)


def _time(eng, phantom, n_vox, probe, n_probe, seed, opts, reps, log):
    """Best of `reps` timed batched runs after a warm-up; None if it fails."""
    import torch
    try:
        eng.simulate_batch(phantom, probe, seed, n_vox=n_vox, want_dose=False, **opts)   # warm-up
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eng.simulate_batch(phantom, probe, seed, n_vox=n_vox, want_dose=False, **opts)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
    except RuntimeError as e:          # e.g. over the HBM budget: not a candidate
        if log:
            log(f"autotune: {opts} failed: {e}")
        return None
    if log:
        log(f"autotune: {opts} {n_probe / best:.3e} hist/s")
    return best, dict(opts)
