#!/usr/bin/env python3
"""Benchmark: population annealing of a 3D +-J Edwards-Anderson instance on one
MI355X, reported as spin-flip attempts per nanosecond.

One benchmark step is one complete anneal of the workload (every row of the
hot path: N_S checkerboard Metropolis sweeps of every replica at each of the
n_temps temperatures, energy histogram, FP64 weight normalisation, copy
counts, prefix sum and gather of the surviving replicas, family and overlap
statistics).  Inputs (couplings, initial population) are resident on the GPU
before the timed region; each timed anneal runs on its own, freshly created
run handle.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel (the sweep) against the chip's integer
                VALU peak, timed live with HIP events on the run's stream;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload;
  extra         the other single-GPU workloads (L = 4 latency-bound case,
                L = 16 throughput case).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import pamc_inputs as pi  # noqa: E402

METRIC = "spin-flip attempts/ns + HBM GB/s fraction; instances/sec batched vs plain"

# int32 VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic int32 operations per spin-flip attempt of the sweep: per
# Philox block of four attempts, Philox4x32-10 = 10 rounds x (2 widening
# multiplies + 2 three-input XORs) = 40, the local fields of the four sites
# packed one byte per site = 6 XORs + 5 adds + 1 byte-align = 12, and the
# acceptance = 4 x (extract + compare + select) + 2 (downhill mask) + 1
# (apply) = 15; 67 / 4 = 16.75.
ALU_OPS_PER_ATTEMPT = 16.75

COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_counters.json")
SWEEP_SOURCE = os.path.join(ROOT, "paper_1710_09025_amd", "csrc", "sweep.hip")


def source_hash() -> str:
    return hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()[:16]


def workload_inputs(name):
    cfg = pi.WORKLOADS[name]
    J = pi.pm_j_couplings(cfg["L"], cfg["disorder_seed"])
    beta = pi.linear_beta(cfg["beta_max"], cfg["n_temps"])
    return cfg, J, beta


def attempts_of(obs, N, sweeps):
    return float(np.sum(obs["R"][obs["measured"] == 1])) * N * sweeps


def time_anneals(name, steps, warmup, timing=True):
    """Creates warmup + steps run handles up front, anneals them one after
    another; returns wall time of the timed anneals and per-phase device
    times."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name)
    N = cfg["L"] ** 3
    runs = [Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], timing=timing)
            for _ in range(warmup + steps)]
    for r in runs[:warmup]:
        assert r.anneal() == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs[warmup:]:
        st = r.anneal()
        assert st == 0, st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms = other_ms = 0.0
    nsteps = 0
    if timing:
        for r in runs[warmup:]:
            a, b, n = r.phase_times()
            sweep_ms += a
            other_ms += b
            nsteps += n
    obs = runs[-1].observables()
    att = attempts_of(obs, N, cfg["sweeps"])
    Rbar = float(np.mean(obs["R"]))
    for r in runs:
        r.close()
    del runs
    torch.cuda.empty_cache()
    return dict(cfg=cfg, wall_s=t1 - t0, sweep_ms=sweep_ms, other_ms=other_ms, nsteps=nsteps,
                attempts_per_anneal=att, mean_R=Rbar, N=N)


def roofline(res):
    K = res["nsteps"] / res["cfg"]["n_temps"]
    sweep_s = res["sweep_ms"] / 1e3
    ops = ALU_OPS_PER_ATTEMPT * res["attempts_per_anneal"] * K
    achieved = ops / sweep_s / 1e12
    traffic = None
    if os.path.exists(COUNTERS_FILE):
        try:
            c = json.load(open(COUNTERS_FILE))
            w = c.get("workloads", {}).get(res["cfg"].get("name", ""), None)
            if c.get("sweep_source_sha256_16") == source_hash() and w:
                traffic = w["hbm_bytes_per_launch"]
        except Exception:
            traffic = None
    rb = ((res["N"] + 15) // 16) * 16
    alg_bytes = 2.0 * res["mean_R"] * rb + 16.0 * res["mean_R"]  # tile in + out, map/E/family
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 3),
            "unit": "Tops/s (int32 VALU)", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
            "kernel": "k_sweep_eo (N_S sweeps of every replica at one temperature)",
            "ops_per_attempt": ALU_OPS_PER_ATTEMPT,
            "avg_launch_ms": round(res["sweep_ms"] / max(1, res["nsteps"]), 4),
            "hbm_gbs_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9, 1),
            "hbm_frac_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9
                                          / HBM_PEAK_GBS, 4)}


def cpu_baseline(name, n_steps):
    import oracle

    cfg, J, beta = workload_inputs(name)
    threads = min(16, os.cpu_count() or 1)
    o = oracle.Oracle(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], threads=threads)
    t0 = time.perf_counter()
    st = o.run(n_steps)
    t1 = time.perf_counter()
    assert st == 0
    rec = o.records()
    att = float(np.sum(rec["R"][:n_steps])) * cfg["L"] ** 3 * cfg["sweeps"]
    return {"value": round(att / ((t1 - t0) * 1e9), 4), "unit": "attempts/ns", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n_steps} of {cfg['n_temps']} temperature steps of the same workload "
                      f"(full population R={cfg['R']}, L={cfg['L']}), {t1 - t0:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed anneals")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="L8_R100000", choices=sorted(pi.WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=16, help="temperature steps of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    res = time_anneals(args.workload, args.steps, args.warmup)
    res["cfg"]["name"] = args.workload
    total_attempts = res["attempts_per_anneal"] * args.steps
    value = total_attempts / (res["wall_s"] * 1e9)
    cfg = res["cfg"]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["wall_s"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: +-J couplings and Philox-initialised replicas from fixed seeds",
        "config": {"workload": f"3D EA +-J L={cfg['L']} periodic, R={cfg['R']}, n_temps={cfg['n_temps']} "
                               f"beta linear 0->{cfg['beta_max']}, N_S={cfg['sweeps']}, one instance",
                   "L": cfg["L"], "R": cfg["R"], "n_temps": cfg["n_temps"], "sweeps": cfg["sweeps"],
                   "step": "one complete anneal", "spins": "int8"},
        "sweep_attempts_per_ns": round(res["attempts_per_anneal"] * args.steps / (res["sweep_ms"] * 1e6), 3),
        "sweep_share": round(res["sweep_ms"] / (res["sweep_ms"] + res["other_ms"]), 4),
        "roofline": roofline(res),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps)
    if not args.no_extra:
        extra = {}
        for name, k, w in (("L4_R1000", 5, 1), ("L16_R500000", 1, 0)):
            if name == args.workload:
                continue
            r = time_anneals(name, k, w)
            extra[name] = {
                "attempts_per_ns": round(r["attempts_per_anneal"] * k / (r["wall_s"] * 1e9), 3),
                "sweep_attempts_per_ns": round(r["attempts_per_anneal"] * k / (r["sweep_ms"] * 1e6), 3),
                "ms_per_anneal": round(r["wall_s"] / k * 1e3, 3),
                "sweep_share": round(r["sweep_ms"] / (r["sweep_ms"] + r["other_ms"]), 4),
            }
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
