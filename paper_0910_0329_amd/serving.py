"""Request-stream replay for the serving loop: calibrates history counts for a
target uncertainty, replays timed arrivals against an Engine's mcd_submit /
mcd_wait, and summarises latency and throughput.

Only orchestration lives here; admission, scheduling, transport and
finalisation run in libmcdose's worker thread and kernels.
"""
from __future__ import annotations

import math
import queue
import threading
import time

import numpy as np

from .inputs import configs
from .inputs.sources import ELECTRON, PHOTON

CAL_SIDES = (1.0, 3.0, 10.0)
CAL_ELECTRON_MEV = 13.0
CAL_PILOT = {PHOTON: 2_000_000, ELECTRON: 500_000}


def calibrate(eng, pool_ids, pool, sides=CAL_SIDES, pilot=None, seed=5, log=None):
    """N_cal per (phantom, particle, field side): histories that bring sigma-bar
    (mean sigma/D over voxels above Dmax/2, history-by-history estimator of the
    plain kernel) to 1%, from one pilot run each: N_cal = N_p (sigma_p / 1%)^2."""
    from .mcdose import KERNEL_PLAIN
    pilot = pilot or CAL_PILOT
    cal = {}
    for i, (pid, ph) in enumerate(zip(pool_ids, pool)):
        for particle in (PHOTON, ELECTRON):
            pts = []
            for side in sides:
                src = configs.serving_source(ph, particle, CAL_ELECTRON_MEV, side)
                n = pilot[particle]
                r = eng.simulate(pid, src, n, seed, 0xC0000000 + len(cal) * 16 + len(pts), n_vox=ph.n_vox,
                                 kernel=KERNEL_PLAIN)
                sb = r["sigma_bar"]
                pts.append((side, n * (sb / 0.01) ** 2 if sb > 0 else float("inf")))
            cal[(i, particle)] = pts
            if log:
                log(f"calibration phantom {i} particle {particle}: " +
                    ", ".join(f"{s:g} cm -> {v:.3g}" for s, v in pts))
    return cal


def n_histories(cal, req, clip=(100_000, 50_000_000)) -> int:
    """History count of a request: N_cal interpolated in log(side) and
    log(N), scaled by (1% / target)^2 and clipped."""
    pts = cal[(req.phantom, req.particle)]
    xs = np.log([p[0] for p in pts])
    ys = np.log([p[1] for p in pts])
    ncal = float(np.exp(np.interp(math.log(req.side), xs, ys)))
    n = ncal * (0.01 / req.target) ** 2
    return int(min(max(n, clip[0]), clip[1]))


def replay(eng, pool_ids, pool, reqs, cal, seed=5, clip=(100_000, 50_000_000), collectors=8,
           adaptive=False, log=None) -> dict:
    """Submits every request at its arrival time (relative to the start of the
    replay) and collects the results on `collectors` threads.  adaptive: each
    request runs until its own sigma-bar reaches the target (at most the
    clipped upper bound), instead of the calibrated history count."""
    tickets = queue.Queue()
    done = []
    failures = []
    lock = threading.Lock()
    plan = [(r, clip[1] if adaptive else n_histories(cal, r, clip)) for r in reqs]

    def collect():
        while True:
            item = tickets.get()
            if item is None:
                return
            r, n, t, t_sub = item
            try:
                out = eng.wait(t, want_dose=False)
                n = out["n_histories"]
            except RuntimeError as e:
                with lock:
                    failures.append((r.index, str(e)))
                continue
            with lock:
                done.append({"index": r.index, "n": n, "latency_ms": out["latency_ms"],
                             "done_s": t_sub + out["latency_ms"] * 1e-3, "sigma_bar": out["sigma_bar"],
                             "target": r.target, "kernel_ms": out["kernel_ms"], "phantom": r.phantom,
                             "particle": r.particle})

    workers = [threading.Thread(target=collect, daemon=True) for _ in range(collectors)]
    for w in workers:
        w.start()
    s0 = eng.serve_stats()
    t0 = time.perf_counter()
    for r, n in plan:
        delay = t0 + r.t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        src = configs.serving_source(pool[r.phantom], r.particle, r.energy, r.side)
        t_sub = time.perf_counter() - t0
        t = eng.submit(pool_ids[r.phantom], src, n, seed, r.index, sigma_target=r.target if adaptive else None)
        tickets.put((r, n, t, t_sub))
    t_last_submit = time.perf_counter() - t0
    if log:
        log(f"serving: {len(plan)} requests submitted in {t_last_submit:.1f} s")
    for _ in workers:
        tickets.put(None)
    for w in workers:
        w.join()
    s1 = eng.serve_stats()
    lat = np.array([d["latency_ms"] for d in done]) if done else np.zeros(1)
    makespan = max([d["done_s"] for d in done] + [t_last_submit])
    hist = sum(d["n"] for d in done)
    offered = sum(n for _, n in plan) if not adaptive else sum(d["n"] for d in done)
    duration = max(r.t for r in reqs) if reqs else 0.0
    ach = np.array([d["sigma_bar"] / d["target"] for d in done if d["sigma_bar"] > 0])
    busy = s1["busy_ms"] - s0["busy_ms"]
    return {
        "requests": len(plan), "completed": len(done), "failed": len(failures),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
        "histories": int(hist), "makespan_s": makespan,
        "hist_per_s": hist / makespan if makespan > 0 else 0.0,
        "offered_hist_per_s": offered / duration if duration > 0 else None,
        "arrival_window_s": duration,
        "gpu_busy_frac": busy * 1e-3 / makespan if makespan > 0 else None,
        "epochs": s1["epochs"] - s0["epochs"],
        "sigma_bar_over_target_median": float(np.median(ach)) if len(ach) else None,
        "failures": failures[:5],
    }
