#!/usr/bin/env python3
"""Throughput benchmark of the dose engine on one MI355X.

Workload (the headline configuration): 6 MV synthetic photon spectrum from a
point source at SSD 100 cm with a 10x10 cm field on a 61x61x60 water-bone-water
phantom of 0.5 cm voxels, seed 2.  A pilot run of 1e7 histories measures
sigma-bar (mean sigma/D over voxels above Dmax/2); one step then transports
N_1% = 1e7 (sigma-bar / 1%)^2 histories, the count that reaches 1% sigma-bar.
The reported value is histories per second of whole steps (tally clear,
transport, finalisation) with phantom and tables already resident in HBM.

Alongside: 20 MeV electron pencil beam on the 32x32x30 water-lung-water
phantom (1e7 histories per run), the ALU roofline of the transport kernel and
the FP64 CPU reference timed on a bounded sample on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the transport kernel: VALU instructions on the converged
# instruction path of one history (all 64 lanes of a wave replaying the same
# history, `lockstep` launch), per history, from rocprofv3 SQ_INSTS_VALU over
# 2e5 histories (profiles/transport_lockstep_insts.txt).  Each is one lane-op
# of the history's own work.
PATH_LANE_OPS = {
    "g6mv_wbw_61x61x60": 3239419221 / 200_000,     # 16197
    "e20_wlw_32x32x30": 12571416380 / 200_000,     # 62857
}
# Plain VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 3.93e13 lane-ops/s (one non-packed FP32/INT32 op per lane per cycle).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# HBM bytes per history of the transport kernel (rocprofv3 FETCH_SIZE +
# WRITE_SIZE scaled by a 1 GiB copy; profiles/transport_g6mv_hbm_traffic.txt).
TRAFFIC_BYTES_PER_HIST = {
    "g6mv_wbw_61x61x60": None,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="histories of the CPU reference sample (0: skip)")
    ap.add_argument("--lockstep-probe", action="store_true",
                    help="run one lockstep launch per workload (for SQ_INSTS_VALU) and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy (calibrates FETCH_SIZE/WRITE_SIZE) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this engine has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_0910_0329_amd.inputs import configs, tables
    from paper_0910_0329_amd.mcdose import Engine

    if args.copy_probe:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return

    blob = tables.standard_blob()
    eng = Engine(0)
    th = eng.load_materials(blob)
    wg = configs.photon_6mv_wbw(10_000_000)
    we = configs.electron_20mev_wlw(10_000_000)
    pg = eng.load_phantom(wg.phantom, th)
    pe = eng.load_phantom(we.phantom, th)

    if args.lockstep_probe:
        for w, p in ((wg, pg), (we, pe)):
            n = 200_000
            r = eng.simulate(p, w.source, n, w.seed, n_vox=w.phantom.n_vox, want_dose=False, lockstep=1)
            print(json.dumps({"workload": w.name, "lockstep_histories": n, "kernel_ms": r["kernel_ms"]}),
                  flush=True)
        return

    def run(w, p, n):
        return eng.simulate(p, w.source, n, w.seed, w.request_key, n_vox=w.phantom.n_vox)

    # pilot: sigma-bar after the configured 1e7 histories fixes N_1%
    pilot = run(wg, pg, wg.n_histories)
    n1 = int(math.ceil(wg.n_histories * (pilot["sigma_bar"] / 0.01) ** 2))
    for _ in range(args.warmup):
        run(wg, pg, n1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms, sbar = [], []
    for _ in range(args.steps):
        r = run(wg, pg, n1)
        kms.append(r["kernel_ms"])
        sbar.append(r["sigma_bar"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n1 * args.steps / (t1 - t0)
    k_ms = sum(kms) / len(kms)
    b = r["bal"]
    closure = abs(b["E_csda"] + b["E_local"] + b["E_esc"] + b["E_miss"] - b["E_src"]) / b["E_src"]

    # electron workload: fixed 1e7 histories per run (its N_1% is too small to fill the GPU)
    run(we, pe, we.n_histories)
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    re_ = run(we, pe, we.n_histories)
    torch.cuda.synchronize()
    te1 = time.perf_counter()
    n1e = int(math.ceil(we.n_histories * (re_["sigma_bar"] / 0.01) ** 2))
    electron = {
        "workload": we.name, "histories": we.n_histories,
        "hist_per_s": we.n_histories / (te1 - te0),
        "kernel_hist_per_s": we.n_histories / (re_["kernel_ms"] * 1e-3),
        "sigma_bar": re_["sigma_bar"], "n_at_1pct": n1e,
    }
    path = PATH_LANE_OPS.get(wg.name)
    if path:
        achieved = path * n1 / (k_ms * 1e-3)
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                    "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS}
        tb = TRAFFIC_BYTES_PER_HIST.get(wg.name)
        roofline["traffic"] = tb * n1 if tb else None
        pe_path = PATH_LANE_OPS.get(we.name)
        if pe_path:
            electron["alu_frac"] = pe_path * we.n_histories / (re_["kernel_ms"] * 1e-3) / PEAK_LANE_OPS
    else:
        roofline = {"bound": "alu", "achieved": None, "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                    "frac": None, "traffic": None}

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        n_cpu = args.cpu_sample
        c0 = time.perf_counter()
        oracle.simulate(blob, wg.phantom, wg.source, n_cpu, wg.seed, wg.request_key)
        c1 = time.perf_counter()
        cpu = {"value": n_cpu / (c1 - c0), "unit": "histories/s", "cores": 1, "kind": "oracle",
               "sample": f"histories [0, {n_cpu}) of the same workload and keys, FP64, one thread"}

    line = {
        "metric": "histories/s (6 MV photon, 20 MeV e-) at 1% sigma; p50/p99 dose-request latency",
        "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wg.name, "source": "6 MV spectrum, point source SSD 100 cm, 10x10 cm field",
                   "histories_per_step": n1, "sigma_bar": sum(sbar) / len(sbar),
                   "pilot_histories": wg.n_histories, "pilot_sigma_bar": pilot["sigma_bar"],
                   "kernel_ms": k_ms, "kernel_hist_per_s": n1 / (k_ms * 1e-3),
                   "energy_balance_rel": closure, "tally": "fp64", "transport": "fp32"},
        "electron_20MeV": electron,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
