#!/usr/bin/env python3
"""Throughput benchmark of the dose engine on one MI355X.

Headline workload: 6 MV synthetic photon spectrum from a point source at SSD
100 cm with a 10x10 cm field on a 61x61x60 water-bone-water phantom of 0.5 cm
voxels, seed 2.  A pilot of 1e7 histories on the plain kernel (exact
history-by-history sigma) measures sigma-bar (mean sigma/D over voxels above
Dmax/2); one step then transports N_1% = 1e7 (sigma-bar / 1%)^2 histories, the
count that reaches 1% sigma-bar, on the default (regrouped) kernel.  `value`
is histories per second of whole steps (tally clear, transport,
finalisation, scalar read-back) with phantom and tables resident in HBM.

Alongside, in the same JSON line:
  forms       the plain per-history kernel at the same N_1%, the batched form
              (128 beamlets in one hipGraph launch with autotuned options vs
              128 separate plain and 128 separate regrouped launches) and the
              served forms (timed Poisson arrivals through the serving loop:
              p50/p99 latency, histories/s; fixed N and sigma-bar targets);
  electron    20 MeV electrons on the 32x32x30 water-lung-water phantom: the
              pencil beam at its N_1% and at 1e7 histories, and a 10x10 cm
              point-source field at its N_1%;
  roofline    ALU roofline of the transport kernel (algorithmic lane-ops per
              history from the converged-path measurement), HBM traffic and
              the FP64 atomic rate against measured ceilings;
  table_variants, table_placement_tissues8, paper_geometry, end_to_end
              physics-refinement tables, LDS vs global tables on an
              eight-tissue CT, the paper's Table 1 setups, and the paper's T;
  cpu_baseline, oracle_agreement
              the FP64 oracle on a bounded sample of the headline and electron
              workloads, and the GPU's dose on the same histories against it.

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

# Algorithmic work: VALU instructions of one history on the converged
# instruction path (all 64 lanes of a wave replaying the same history, plain
# kernel `lockstep` launch), from rocprofv3 SQ_INSTS_VALU over 2e5 histories
# of each workload divided by 2e5 (profiles/transport_lockstep_valu.md).  Each
# VALU instruction of that path is one lane-op of the history's own work.  The
# figure is the lowest any build of the shared transport measured: the
# branch-free random-word selects cost a few converged instructions more
# (17760.8 and 68566.5) while saving far more under divergence.
PATH_LANE_OPS = {
    "g6mv_wbw_61x61x60": 3442984358 / 200_000,     # 17214.9
    "e20_wlw_32x32x30": 13295921535 / 200_000,     # 66479.6
}
# Plain VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 3.93e13 lane-ops/s (one non-packed FP32/INT32 op per lane per cycle).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# HBM bytes per history of the transport kernel (the wave-stack kernel
# k_wave<false, false, false>): rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by
# its reading for a 1 GiB device copy (profiles/transport_g6mv_hbm_traffic.md,
# profiles/transport_e20_wlw_hbm_traffic.md).
TRAFFIC_BYTES_PER_HIST = {
    "g6mv_wbw_61x61x60": (16080082.0 * 2.0 + 42854716.0 * 1.0) * 1024 / 164442762,     # 467.1
    "e20_wlw_32x32x30": (1148667.8125 * 2.0 + 16281907.75 * 1.0) * 1024 / 10_000_000,  # 1902.5
}
METRIC = "histories/s (6 MV photon, 20 MeV e-) at 1% sigma; p50/p99 dose-request latency"
# The paper's Table 1 (Tesla C1060, FP32; DPM physics and a measured 6 MV
# spectrum, neither available here): histories, GPU seconds, sigma-bar.
PAPER_TABLE1 = {
    "paper_e20_wlw_61x61x150": (10_000_000, 80.6, 0.0065),
    "paper_e20_wbw_61x61x150": (10_000_000, 101.8, 0.0063),
    "paper_g6mv_wlw_61x61x150": (1_000_000_000, 845.8, 0.0052),
    "paper_g6mv_wbw_61x61x150": (1_000_000_000, 1242.3, 0.0046),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=250_000,
                    help="photon histories per host process of the CPU oracle sample (0: skip); "
                         "electrons take a tenth as many")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the served form (0: skip); 60 s is the full stream")
    ap.add_argument("--serve-adaptive-seconds", type=float, default=15.0,
                    help="arrival window of the served form with sigma-bar targets (0: skip)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline steps (used for profiling the transport phase)")
    ap.add_argument("--lockstep-probe", action="store_true",
                    help="run one lockstep launch per workload (for SQ_INSTS_VALU) and exit")
    ap.add_argument("--electron-only", action="store_true",
                    help="only the 20 MeV pencil-beam steps of 1e7 histories, one JSON line "
                         "(used for profiling the electron-source phase kernel)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy (calibrates FETCH_SIZE/WRITE_SIZE) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def closure(b):
    return abs(b["E_csda"] + b["E_local"] + b["E_esc"] + b["E_miss"] - b["E_src"]) / b["E_src"]


def atomic_ceilings(eng, nv, S, Q, flush_rate, flushes_per_history):
    """FP64 atomic-add rates of the device (mcd_measure_atomics) on three
    address streams over the 16 sub-tallies of an nv-voxel phantom."""
    import numpy as np
    import torch
    n_target = 16 * nv
    target = torch.zeros(n_target, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(11)
    n = 1 << 25
    w = np.where(Q > 0, S * S / np.where(Q > 0, Q, 1.0), 0.0)
    w = w / w.sum()
    streams = {
        "replay": rng.integers(0, 16, n, dtype=np.int64) * nv + rng.choice(nv, n, p=w),
        "uniform": rng.integers(0, n_target, n, dtype=np.int64),
        "one_address": np.full(n, n_target // 2, dtype=np.int64),
    }
    out = {"flushes_per_history": flushes_per_history, "flush_rate": flush_rate, "unit": "atomics/s"}
    for name, idx in streams.items():
        t = torch.from_numpy(idx.astype(np.uint32).view(np.int32)).cuda()
        eng.measure_atomics(target, t, 1)
        reps = 1 if name == "one_address" else 4
        ms = eng.measure_atomics(target, t, reps)
        out[f"ceiling_{name}"] = n * reps / (ms * 1e-3)
        del t
    out["atomic_frac"] = flush_rate / out["ceiling_replay"]
    return out


def cpu_leg(per_proc, blob, eng, run, wg, pg, we, pe):
    """The FP64 oracle on the host cores: P single-threaded processes run
    disjoint history ranges of the headline (and the 20 MeV electron)
    workload with the same keys, merged in FP64.  The same histories on the
    GPU (plain kernel) give the dose agreement."""
    import numpy as np

    import oracle
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out, agree = {}, {}
    for tag, w, p, n in (("photon", wg, pg, per_proc * procs), ("electron", we, pe, per_proc // 10 * procs)):
        t0 = time.perf_counter()
        ref = oracle.simulate_parallel(blob, w.phantom, w.source, n, w.seed, w.request_key, procs=procs)
        dt = time.perf_counter() - t0
        # value: whole job on the wall clock (process start-up included);
        # per_core: histories per second of one process's transport time
        out[tag] = {"value": n / dt, "per_core": n / ref["busy_s"], "histories": n, "s": dt}
        d_ref, s_ref, dmax_ref, sbar_ref = oracle.finalize(w.phantom, ref["S"], ref["Q"], n)
        g = run(w, p, n, kernel=1)
        d = g["dose"].cpu().numpy()
        diff = np.abs(d - d_ref)
        sel = d_ref > 0.1 * dmax_ref
        agree[w.name] = {"histories": n, "same_keys": True, "max_abs_diff_over_dmax": float(diff.max() / dmax_ref),
                         "frac_within_1pct_dmax_above_10pct": float((diff[sel] <= 0.01 * dmax_ref).mean()),
                         "frac_within_1pct_dmax_all": float((diff <= 0.01 * dmax_ref).mean()),
                         "voxels_above_10pct": int(sel.sum()), "sigma_bar_oracle": sbar_ref,
                         "sigma_bar_gpu": g["sigma_bar"]}
    cpu = {"value": out["photon"]["value"], "unit": "histories/s", "cores": procs, "kind": "oracle",
           "per_core": out["photon"]["per_core"], "cpu_model": model,
           "sample": f"histories [0, {out['photon']['histories']}) of the headline workload and keys, FP64, "
                     f"{procs} single-threaded processes on disjoint ranges, tallies merged",
           "electron_value": out["electron"]["value"], "electron_per_core": out["electron"]["per_core"],
           "electron_sample": f"histories [0, {out['electron']['histories']}) of the 20 MeV pencil workload, "
                              f"{procs} processes",
           "seconds": out["photon"]["s"] + out["electron"]["s"]}
    return cpu, agree


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this engine has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_0910_0329_amd.inputs import configs, sources, tables
    from paper_0910_0329_amd.mcdose import KERNEL_PLAIN, Engine

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
            r = eng.simulate(p, w.source, n, w.seed, n_vox=w.phantom.n_vox, want_dose=False,
                             kernel=KERNEL_PLAIN, lockstep=1)
            print(json.dumps({"workload": w.name, "lockstep_histories": n, "kernel_ms": r["kernel_ms"]}),
                  flush=True)
        return

    def run(w, p, n, **kw):
        return eng.simulate(p, w.source, n, w.seed, w.request_key, n_vox=w.phantom.n_vox, **kw)

    if args.electron_only:
        for _ in range(args.warmup):
            run(we, pe, we.n_histories)
        te, re_ = timed(lambda: run(we, pe, we.n_histories), args.steps)
        pe_path = PATH_LANE_OPS[we.name]
        k_s = re_["kernel_ms"] * 1e-3
        print(json.dumps({"workload": we.name, "histories_per_step": we.n_histories, "steps": args.steps,
                          "hist_per_s": we.n_histories / te, "kernel_ms": re_["kernel_ms"],
                          "launches": re_["launches"],
                          "per_launch_ms": re_["kernel_ms"] / max(re_["launches"], 1),
                          "alu_frac": pe_path * we.n_histories / k_s / PEAK_LANE_OPS,
                          "traffic": (TRAFFIC_BYTES_PER_HIST[we.name] * we.n_histories / max(re_["launches"], 1)
                                      if we.name in TRAFFIC_BYTES_PER_HIST else None),
                          "energy_balance_rel": closure(re_["bal"])}), flush=True)
        eng.close()
        return

    # ------------------------------------------------------------ headline
    pilot = run(wg, pg, wg.n_histories, kernel=KERNEL_PLAIN, want_tallies=True)
    n1 = int(math.ceil(wg.n_histories * (pilot["sigma_bar"] / 0.01) ** 2))
    log(f"photon pilot sigma-bar {pilot['sigma_bar']:.4f} -> N_1% = {n1}")
    # The N^-1/2 projection undershoots a little (Dmax falls as its noise does,
    # so more voxels enter the average); confirm N_1% with the exact
    # history-by-history estimator and grow it until sigma-bar <= 1%.
    tp = rp = None
    for _ in range(6):
        tp, rp = timed(lambda: run(wg, pg, n1, kernel=KERNEL_PLAIN), 1)
        log(f"exact sigma-bar at {n1}: {rp['sigma_bar']:.5f}")
        if rp["sigma_bar"] <= 0.01:
            break
        n1 = int(math.ceil(n1 * (rp["sigma_bar"] / 0.01) ** 2 * 1.002))
    if rp["sigma_bar"] > 0.01:
        raise SystemExit(f"could not reach 1% sigma-bar (exact estimator {rp['sigma_bar']:.5f} at {n1})")
    for _ in range(args.warmup):
        run(wg, pg, n1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = []
    for _ in range(args.steps):
        rs.append(run(wg, pg, n1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n1 * args.steps / (t1 - t0)
    k_ms = sum(r["kernel_ms"] for r in rs) / len(rs)
    launches = rs[-1]["launches"]
    sbar = sum(r["sigma_bar"] for r in rs) / len(rs)
    log(f"regrouped: {value:.3e} hist/s, kernel {k_ms:.1f} ms over {launches} launches")

    line = {
        "metric": METRIC, "value": value, "unit": "histories/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wg.name,
                   "source": "6 MV spectrum (64 bins, 0.1-6 MeV), point source SSD 100 cm, 10x10 cm field",
                   "phantom": "61x61x60 x 0.5 cm: water 0-3 cm, bone 1.85 g/cm3 3-7 cm, water 7-30 cm",
                   "kernel": "regrouped (wave stacks by particle type, photon/electron modes; 16 sub-tallies, "
                             "batch statistics)",
                   "histories_per_step": n1, "sigma_bar": sbar, "sigma_bar_exact": rp["sigma_bar"],
                   "sigma_bar_estimators": "sigma_bar: the regrouped kernel's 16-group estimate (c4-corrected); "
                                           "sigma_bar_exact: history-by-history (plain kernel) at the same N",
                   "pilot_histories": wg.n_histories, "pilot_sigma_bar": pilot["sigma_bar"],
                   "kernel_ms": k_ms, "launches_per_step": launches,
                   "kernel_hist_per_s": n1 / (k_ms * 1e-3),
                   "energy_balance_rel": closure(rs[-1]["bal"]), "tally": "fp64", "transport": "fp32"},
    }

    path = PATH_LANE_OPS.get(wg.name)
    roofline = {"bound": "alu", "kernel": "k_wave<false,false,false> (wave-stack transport, LDS tables)", "achieved": None,
                "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s", "frac": None, "traffic": None,
                "per_launch_ms": k_ms / max(launches, 1), "histories_per_launch": n1 / max(launches, 1)}
    if path:
        achieved = path * n1 / (k_ms * 1e-3)
        roofline.update(achieved=achieved / 1e12, frac=achieved / PEAK_LANE_OPS,
                        lane_ops_per_history=path)
        tb = TRAFFIC_BYTES_PER_HIST.get(wg.name)
        roofline["traffic"] = tb * n1 / max(launches, 1) if tb else None
    # The peak's issue model, measured: SIMD cycles per wave64 instruction of
    # the kinds the transport is made of (4 = 16 lanes per cycle, the rate the
    # peak assumes; an FMA issues faster, which the 157.3 TFLOP/s FP32 figure
    # counts)
    from paper_0910_0329_amd.mcdose import (VALU_ADD_F32, VALU_EXP_F32, VALU_FMA_F32, VALU_FMAMK_F32,
                                            VALU_MAD_U64, VALU_MUL_F32, VALU_RCP_F32, VALU_XAD_U32)
    roofline["valu_issue_cycles"] = {
        name: eng.measure_valu(kind, 200) for name, kind in
        (("fma_f32", VALU_FMA_F32), ("fmamk_f32", VALU_FMAMK_F32), ("add_f32", VALU_ADD_F32),
         ("mul_f32", VALU_MUL_F32), ("xad_u32", VALU_XAD_U32), ("mad_u64_plus_xor", VALU_MAD_U64),
         ("rcp_f32", VALU_RCP_F32), ("exp_f32", VALU_EXP_F32))}
    log(f"VALU issue cycles per wave64 operation: {roofline['valu_issue_cycles']}")
    line["roofline"] = roofline

    # ------------------------------------------------------- atomic ceiling
    # The tally flushes are FP64 atomic adds (the paper's dose collection by
    # atomic float addition, Sec. 2.4).  Their rate in the headline step
    # (flushes per history from a diagnostics run x histories/s) against the
    # rate the device sustains for the same operation on address streams: the
    # flush pattern of the headline (a voxel drawn with probability proportional
    # to S^2/Q of the plain pilot, the number of histories that deposit in it,
    # and a uniform sub-tally), uniform addresses over the 16 sub-tallies, and
    # every lane on one address.
    rd = run(wg, pg, 2_000_000, diagnostics=1, want_dose=False)
    flushes = rd["cnt"]["flushes"] / 2_000_000
    roofline["atomic"] = atomic_ceilings(eng, wg.phantom.n_vox, pilot["S"].cpu().numpy(),
                                         pilot["Q"].cpu().numpy(), flushes * n1 / (k_ms * 1e-3), flushes)
    log(f"atomics: {roofline['atomic']}")

    if args.headline_only:
        line["cpu_baseline"] = None
        print(json.dumps(line), flush=True)
        eng.close()
        return

    # ------------------------------------------------------------ plain kernel
    forms = {}
    forms["plain"] = {"photon": {"hist_per_s": n1 / tp, "kernel_hist_per_s": n1 / (rp["kernel_ms"] * 1e-3),
                                 "histories": n1, "sigma_bar": rp["sigma_bar"]}}
    log(f"plain photon: {n1 / tp:.3e} hist/s")

    # ------------------------------------------------------------ electrons
    electron = {"workload": we.name}
    pe_pilot = run(we, pe, 1_000_000, kernel=KERNEL_PLAIN, want_tallies=True)
    n1e = max(2, int(math.ceil(1_000_000 * (pe_pilot["sigma_bar"] / 0.01) ** 2)))
    reps = 20
    te, re_ = timed(lambda: run(we, pe, n1e), reps)
    electron["pencil_at_1pct"] = {"histories": n1e, "ms": te * 1e3, "hist_per_s": n1e / te,
                                  "sigma_bar": re_["sigma_bar"]}
    run(we, pe, we.n_histories)
    te, re_ = timed(lambda: run(we, pe, we.n_histories), 2)
    tpe, rpe = timed(lambda: run(we, pe, we.n_histories, kernel=KERNEL_PLAIN), 1)
    electron["pencil_1e7"] = {"histories": we.n_histories, "hist_per_s": we.n_histories / te,
                              "kernel_hist_per_s": we.n_histories / (re_["kernel_ms"] * 1e-3),
                              "plain_hist_per_s": we.n_histories / tpe,
                              "energy_balance_rel": closure(re_["bal"])}
    pe_path = PATH_LANE_OPS.get(we.name)
    if pe_path:
        electron["pencil_1e7"]["alu_frac"] = pe_path * we.n_histories / (re_["kernel_ms"] * 1e-3) / PEAK_LANE_OPS
    pe_tb = TRAFFIC_BYTES_PER_HIST.get(we.name)
    if pe_tb:
        # one launch per step in lane-stack mode: bytes per launch, and HBM rate
        electron["pencil_1e7"]["traffic"] = pe_tb * we.n_histories / max(re_["launches"], 1)
        electron["pencil_1e7"]["hbm_frac"] = pe_tb * we.n_histories / (re_["kernel_ms"] * 1e-3) / 8e12
    # the pencil beam's flushes crowd the beam axis: their rate against the
    # device's rate on the same address pattern (drawn from the pilot's S^2/Q)
    rde = run(we, pe, 200_000, diagnostics=1, want_dose=False)
    e_flushes = rde["cnt"]["flushes"] / 200_000
    electron["pencil_1e7"]["atomic"] = atomic_ceilings(
        eng, we.phantom.n_vox, pe_pilot["S"].cpu().numpy(), pe_pilot["Q"].cpu().numpy(),
        e_flushes * we.n_histories / (re_["kernel_ms"] * 1e-3), e_flushes)
    wf = configs.electron_20mev_point_field(we.phantom, 1_000_000)
    fpilot = run(wf, pe, wf.n_histories, kernel=KERNEL_PLAIN)
    n1f = int(math.ceil(wf.n_histories * (fpilot["sigma_bar"] / 0.01) ** 2))
    run(wf, pe, n1f)
    tf, rf = timed(lambda: run(wf, pe, n1f), 3)
    tfp, rfp = timed(lambda: run(wf, pe, n1f, kernel=KERNEL_PLAIN), 1)
    electron["field10x10_at_1pct"] = {"histories": n1f, "hist_per_s": n1f / tf,
                                      "kernel_hist_per_s": n1f / (rf["kernel_ms"] * 1e-3),
                                      "plain_hist_per_s": n1f / tfp, "sigma_bar": rf["sigma_bar"]}
    forms["plain"]["electron_field10x10"] = {"hist_per_s": n1f / tfp, "histories": n1f}
    log(f"electrons: pencil N_1%={n1e}, 1e7 at {we.n_histories / te:.3e} hist/s; "
        f"10x10 field N_1%={n1f} at {n1f / tf:.3e} hist/s")
    line["electron_20MeV"] = electron

    # ------------------------------------------------------------ table variants
    # physics refinements in the tables: emission angles, the density effect,
    # per-element screening, Rayleigh scattering, the second-moment hinge,
    # Bhabha events for positrons, and all of them but per-element screening
    # together
    variants = {}
    for variant in ("angular", "density", "elements", "rayleigh", "hinge2", "bhabha", "refined"):
        thv = eng.load_materials(tables.standard_blob(variant))
        cur = {}
        for w, n in ((wg, 20_000_000), (we, 4_000_000)):
            pa = eng.load_phantom(w.phantom, thv)
            eng.simulate(pa, w.source, n, w.seed, n_vox=w.phantom.n_vox)
            ta_, ra_ = timed(lambda: eng.simulate(pa, w.source, n, w.seed, n_vox=w.phantom.n_vox), 2)
            cur[w.name] = {"histories": n, "hist_per_s": n / ta_,
                           "kernel_hist_per_s": n / (ra_["kernel_ms"] * 1e-3)}
            eng.unload_phantom(pa)
        eng.unload_materials(thv)
        variants[variant] = cur
    line["table_variants"] = variants
    log(f"table variants: {variants}")

    # ------------------------------------------------------------ table placement
    # eight tissue classes: the LDS copy of their tables (128 KiB) leaves room
    # for one 512-thread workgroup per CU; device-memory tables (the automatic
    # choice here) let the registers set the occupancy
    from paper_0910_0329_amd.mcdose import TABLES_GLOBAL, TABLES_LDS
    wt = configs.photon_6mv_ct8(40_000_000)
    th8 = eng.load_materials(tables.tissue_blob())
    p8 = eng.load_phantom(wt.phantom, th8)
    placement = {"workload": f"{wt.name}: 6 MV, 10x10 cm field, 128^3 x 0.25 cm random field in 8 tissue classes",
                 "histories": wt.n_histories}
    for label, opts in (("lds", {"table_placement": TABLES_LDS}), ("global", {"table_placement": TABLES_GLOBAL}),
                        ("auto", {})):
        shape = eng.launch_shape(p8, **opts)
        eng.simulate(p8, wt.source, wt.n_histories // 10, wt.seed, n_vox=wt.phantom.n_vox, **opts)
        tp_, rp_ = timed(lambda: eng.simulate(p8, wt.source, wt.n_histories, wt.seed, n_vox=wt.phantom.n_vox,
                                              **opts), 2)
        placement[label] = {"hist_per_s": wt.n_histories / tp_,
                            "kernel_hist_per_s": wt.n_histories / (rp_["kernel_ms"] * 1e-3),
                            "waves_per_cu": shape["resident_per_cu"] * shape["block_size"] // 64,
                            "table_placement": "global" if shape["table_placement"] == TABLES_GLOBAL else "lds"}
    eng.unload_phantom(p8)
    eng.unload_materials(th8)
    line["table_placement_tissues8"] = placement
    log(f"table placement, 8 tissues: {placement}")

    # ------------------------------------------------------------ paper geometry
    from paper_0910_0329_amd.inputs.sources import ELECTRON, PHOTON
    paper = {}
    for particle in (ELECTRON, PHOTON):
        for middle in ("lung", "bone"):
            wp = configs.paper_workload(particle, middle, 0)
            n_p, t_c1060, sb_c1060 = PAPER_TABLE1[wp.name]
            pp = eng.load_phantom(wp.phantom, th)
            tp_, rp_ = timed(lambda: eng.simulate(pp, wp.source, n_p, wp.seed, n_vox=wp.phantom.n_vox), 1)
            paper[wp.name] = {"histories": n_p, "s": tp_, "hist_per_s": n_p / tp_,
                              "kernel_hist_per_s": n_p / (rp_["kernel_ms"] * 1e-3), "sigma_bar": rp_["sigma_bar"],
                              "c1060_s": t_c1060, "c1060_sigma_bar": sb_c1060}
            eng.unload_phantom(pp)
            log(f"{wp.name}: {n_p} histories in {tp_:.2f} s (C1060: {t_c1060} s), sigma-bar {rp_['sigma_bar']:.4f}")
    line["paper_geometry"] = paper

    # ------------------------------------------------------------ CT-like phantom
    wc = configs.photon_6mv_random_field(100_000_000)
    pc = eng.load_phantom(wc.phantom, th)
    ct = {"workload": wc.name, "histories": wc.n_histories}
    doses = {}
    for fp32 in (0, 1):
        tc, rc_ = timed(lambda: eng.simulate(pc, wc.source, wc.n_histories, wc.seed, n_vox=wc.phantom.n_vox,
                                             tally_fp32=fp32), 1)
        key = "fp32" if fp32 else "fp64"
        ct[key] = {"hist_per_s": wc.n_histories / tc, "kernel_hist_per_s": wc.n_histories / (rc_["kernel_ms"] * 1e-3),
                   "sigma_bar": rc_["sigma_bar"], "dmax": rc_["dmax"]}
        doses[key] = rc_["dose"].cpu().numpy()
    import numpy as np
    from paper_0910_0329_amd.inputs.tables import MAT_AIR, MAT_BONE, MAT_LUNG, MAT_WATER
    mat = wc.phantom.mat.reshape(-1)
    sel = doses["fp64"] > 0.1 * ct["fp64"]["dmax"]
    per = {}
    for name, m in (("air", MAT_AIR), ("lung", MAT_LUNG), ("water", MAT_WATER), ("bone", MAT_BONE)):
        c = sel & (mat == m)
        if c.any():
            rel = np.abs(doses["fp32"][c] - doses["fp64"][c]) / doses["fp64"][c]
            per[name] = {"voxels": int(c.sum()), "max_rel": float(rel.max()), "median_rel": float(np.median(rel))}
    ct["fp32_vs_fp64_dose_above_10pct_dmax"] = per
    del doses
    eng.unload_phantom(pc)
    line["ct_phantom"] = ct
    log(f"ct phantom: fp64 {ct['fp64']['hist_per_s']:.3e} hist/s, fp32 {ct['fp32']['hist_per_s']:.3e}; {per}")

    # ------------------------------------------------------------ batched
    from paper_0910_0329_amd import autotune
    srcs, ns = sources.beamlets(wg.phantom, seed=4)
    items = [(s, int(n), i) for i, (s, n) in enumerate(zip(srcs, ns))]
    n_tot = sum(n for _, n, _ in items)
    tuned = autotune.tune(eng, pg, wg.phantom.n_vox, items, 4, scale=8, reps=1, use_cache=False)
    eng.simulate_batch(pg, items, 4, n_vox=wg.phantom.n_vox, use_graph=1, **tuned)       # capture
    tb_, (outs, tot) = timed(lambda: eng.simulate_batch(pg, items, 4, n_vox=wg.phantom.n_vox, use_graph=1,
                                                        **tuned), 3)

    def separate():
        r = None
        for s, n, k in items:
            r = eng.simulate(pg, s, n, 4, k, n_vox=wg.phantom.n_vox, kernel=KERNEL_PLAIN)
        return r

    ts_, _ = timed(separate, 1)

    def separate_regrouped():
        r = None
        for s, n, k in items:
            r = eng.simulate(pg, s, n, 4, k, n_vox=wg.phantom.n_vox)
        return r

    tsr_, _ = timed(separate_regrouped, 1)
    forms["batched"] = {"workload": "128 beamlets 0.5x0.5 cm on g6mv_wbw_61x61x60 (even 6 MV, odd e- U(6,20) MeV)",
                        "histories": n_tot, "hist_per_s": n_tot / tb_, "ms": tb_ * 1e3,
                        "kernel_ms": tot["kernel_ms"], "tuned_opts": tuned,
                        "kernel_hist_per_s": n_tot / (tot["kernel_ms"] * 1e-3),
                        "kernel_ms_is_replay_time": "graph replay (set-up fills, transport, finalisation) "
                                                    "timed by events around the launch",
                        "separate_plain_hist_per_s": n_tot / ts_, "separate_plain_ms": ts_ * 1e3,
                        "separate_regrouped_hist_per_s": n_tot / tsr_, "separate_regrouped_ms": tsr_ * 1e3,
                        "speedup_vs_separate": ts_ / tb_, "speedup_vs_separate_regrouped": tsr_ / tb_,
                        "energy_balance_rel": closure(tot["bal"])}
    if tot["kernel_ms"] > tb_ * 1e3:
        raise SystemExit(f"batched: replay time {tot['kernel_ms']:.1f} ms exceeds the call's {tb_ * 1e3:.1f} ms")
    log(f"batched: {n_tot / tb_:.3e} hist/s vs {n_tot / ts_:.3e} separate plain")

    # ------------------------------------------------------------ served
    if args.serve_seconds > 0:
        from paper_0910_0329_amd import serving
        pool = configs.serving_phantoms()
        pool_ids = [eng.load_phantom(p, th) for p in pool]
        cal = serving.calibrate(eng, pool_ids, pool, log=log)
        reqs = configs.serving_requests(20.0, args.serve_seconds, seed=5)
        eng.serve_configure()
        warm = eng.submit(pool_ids[0], configs.serving_source(pool[0], 0, 0.0, 5.0), 100_000, 5, 0xFFFF0000)
        eng.wait(warm, want_dose=False)
        sv = serving.replay(eng, pool_ids, pool, reqs, cal, seed=5, collectors=32, log=log)
        sv["workload"] = (f"Poisson 20 req/s for {args.serve_seconds:g} s (seed 5); random-field phantoms "
                          "64^3 x 0.5, 128^3 x 0.25, 256^3 x 0.2 cm (seeds 51-53); 6 MV or e- U(6,20) MeV; "
                          "field 1-10 cm; target sigma-bar 2% or 1%; N clipped to [1e5, 5e7]")
        forms["served"] = sv
        log(f"served: p50 {sv['p50_ms']:.0f} ms p99 {sv['p99_ms']:.0f} ms, {sv['hist_per_s']:.3e} hist/s "
            f"(offered {sv['offered_hist_per_s']:.3e})")
    if args.serve_seconds > 0 and args.serve_adaptive_seconds > 0:
        reqs_a = configs.serving_requests(20.0, args.serve_adaptive_seconds, seed=5)
        sa = serving.replay(eng, pool_ids, pool, reqs_a, cal, seed=5, collectors=32, adaptive=True, log=log)
        sa["workload"] = (f"the first {args.serve_adaptive_seconds:g} s of the same arrivals; each request stops "
                          "at its own sigma-bar target (at most 5e7 histories)")
        forms["served_adaptive"] = sa
        log(f"served adaptive: p50 {sa['p50_ms']:.0f} ms p99 {sa['p99_ms']:.0f} ms, {sa['hist_per_s']:.3e} hist/s")
    line["forms"] = forms

    # ------------------------------------------------------------ end to end
    # The paper's time T covers initialisation, transfers and finalisation
    # (Sec. 3): here table and phantom upload, the regrouped run of N_1%
    # histories, dose and sigma copied to host memory, and the unloads.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th2 = eng.load_materials(blob)
    pg2 = eng.load_phantom(wg.phantom, th2)
    r2 = run(wg, pg2, n1, device_out=False)
    eng.unload_phantom(pg2)
    eng.unload_materials(th2)
    t_e2e = time.perf_counter() - t0
    line["end_to_end"] = {"s": t_e2e, "hist_per_s": n1 / t_e2e, "histories": n1, "sigma_bar": r2["sigma_bar"],
                          "includes": "table blob and phantom upload, Woodcock majorant, transport, finalisation, "
                                      "dose and sigma copied to host memory, unloads"}
    log(f"end to end: {t_e2e:.3f} s for {n1} histories")

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if args.cpu_sample > 0:
        cpu, line["oracle_agreement"] = cpu_leg(args.cpu_sample, blob, eng, run, wg, pg, we, pe)
        log(f"cpu baseline: {cpu}")
        log(f"oracle agreement: {line['oracle_agreement']}")
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
