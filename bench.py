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
# The same with real (Gaussian, fixed-point) couplings, per attempt: Philox
# 40 / 4 = 10; the local field over six neighbours, each an XOR shared by the
# four replicas of a word (1/4) + extract + 24-bit multiply-add, and dE from
# it = 6 x 2.25 + 1 = 14.5; the acceptance: binary32 conversion and product
# (2), the exp recipe (scale, round, 2 reduction FMAs, 7 Horner FMAs,
# convert, ldexp = 13), the threshold (scale, convert = 2) and four compares
# (dE <= 0, x >= -23, e >= 1, u < T) = 21; applying the flip = 2: 47.5.
ALU_OPS_PER_ATTEMPT_REAL = 47.5

COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_counters.json")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_1710_09025_amd", "csrc", f)
                 for f in ("sweep.hip", "step_common.h", "pamc_dev.h")]


def log(msg: str):
    """Progress of the legs on stderr (the JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the sources that define the sweep kernel; the committed HBM
    counters apply only while it is unchanged."""
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def workload_inputs(name, real=False):
    """Configuration, couplings and schedule of a named workload; square
    lattice workloads (dim = 2) always take Gaussian couplings."""
    cfg = pi.WORKLOADS[name]
    dim = cfg.get("dim", 3)
    if dim == 2:
        J = pi.gaussian_couplings(cfg["L"], cfg["disorder_seed"], dim=2)
    else:
        gen = pi.gaussian_couplings if real else pi.pm_j_couplings
        J = gen(cfg["L"], cfg["disorder_seed"])
    beta = pi.linear_beta(cfg["beta_max"], cfg["n_temps"])
    return cfg, J, beta


def attempts_of(obs, N, sweeps):
    return float(np.sum(obs["R"][obs["measured"] == 1])) * N * sweeps


def time_anneals(name, steps, warmup, autotune=True, packed=False, real=False, icm_rounds=0):
    """Creates warmup + steps run handles up front (each temperature step a
    replayed hipGraph; sweep shapes chosen by the autotuner at creation,
    outside the timed region) and anneals them one after another for the
    wall time; one more anneal with HIP events around every step's kernels
    gives the per-kernel device time."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name, real)
    N = cfg["L"] ** cfg.get("dim", 3)
    runs = [Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], autotune=autotune, packed=packed,
                 icm_rounds=icm_rounds) for _ in range(warmup + steps)]
    shape = runs[0].sweep_shape()
    for r in runs[:warmup]:
        assert r.anneal() == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs[warmup:]:
        st = r.anneal()
        assert st == 0, st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = runs[-1].observables()
    for r in runs:
        r.close()
    del runs
    timed = Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], timing=True, autotune=autotune,
                 packed=packed, icm_rounds=icm_rounds)
    assert timed.sweep_shape() == shape
    assert timed.anneal() == 0
    sweep_ms, other_ms, _, nsteps = timed.phase_times()
    obs_t = timed.observables()
    for key in ("R", "sum_E", "sum_E2"):
        assert np.array_equal(obs[key], obs_t[key]), "timed and graph runs differ"
    timed.close()
    torch.cuda.empty_cache()
    att = attempts_of(obs, N, cfg["sweeps"])
    Rbar = float(np.mean(obs["R"]))
    return dict(cfg=cfg, wall_s=t1 - t0, sweep_ms=sweep_ms, other_ms=other_ms, nsteps=nsteps,
                attempts_per_anneal=att, mean_R=Rbar, N=N, shape=shape, real=real)


def footprint_gb(name, packed):
    import ctypes

    from paper_1710_09025_amd import _capi

    cfg = pi.WORKLOADS[name]
    lib = _capi.load()
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    opt.spin_format = _capi.SPINS_PACKED if packed else _capi.SPINS_INT8
    return round(lib.pamc_footprint(cfg["L"], cfg["R"], cfg["n_temps"], ctypes.byref(opt)) / 1e9, 3)


def gather_bench(name, n_steps, packed=False):
    """The stand-alone gather of surviving replicas (fuse_gather off) over the
    first n_steps temperature steps of a workload, timed with HIP events:
    algorithmic bytes per output replica = row read + row write + energy and
    family read and write + the copy-map read."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name)
    p = Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], timing=True, fuse_gather=False,
             autotune=True, packed=packed)
    assert p.anneal(n_steps) == 0
    sweep_ms, resample_ms, gather_ms, nsteps = p.phase_times()
    obs = p.observables()
    k_now, R_now = p.shape()
    assert k_now == n_steps
    p.close()
    torch.cuda.empty_cache()
    rb = ((cfg["L"] ** 3 + 15) // 16) * 16
    if packed:
        rb = (rb + 127) // 128 * 16
    # the gather after step k writes the R_{k+1} replicas of step k + 1
    rows = float(np.sum(obs["R"][1:n_steps])) + R_now
    per_row = 2 * rb + 2 * 8 + 4
    gbs = rows * per_row / (gather_ms / 1e3) / 1e9
    return {"kernel": "k_gather", "spins": "packed" if packed else "int8", "steps": int(nsteps),
            "bytes_per_replica": per_row,
            "avg_launch_ms": round(gather_ms / nsteps, 4), "achieved_gbs": round(gbs, 1),
            "peak_gbs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
            "resample_ms_per_step": round(resample_ms / nsteps, 4),
            "sweep_ms_per_step": round(sweep_ms / nsteps, 4)}


def sweep_kernel_name(L, real):
    if real:
        return f"k_sweep_cq<{2 if L % 2 == 0 else 3}, 512>"
    return f"k_sweep_eo<{L}>" if L in (8, 16) else "k_sweep_cm / k_sweep_lex"


def roofline(res):
    sweep_s = res["sweep_ms"] / 1e3
    real = res.get("real", False)
    opa = ALU_OPS_PER_ATTEMPT_REAL if real else ALU_OPS_PER_ATTEMPT
    ops = opa * res["attempts_per_anneal"]
    achieved = ops / sweep_s / 1e12
    traffic = None
    key = res["cfg"].get("name", "") + ("_gaussian" if real else "")
    if os.path.exists(COUNTERS_FILE):
        try:
            c = json.load(open(COUNTERS_FILE))
            w = c.get("workloads", {}).get(key, None)
            if c.get("sweep_source_sha256_16") == source_hash() and w:
                traffic = w["hbm_bytes_per_launch"]
        except Exception:
            traffic = None
    rb = ((res["N"] + 15) // 16) * 16
    # tile in + out, map / energy / family
    alg_bytes = 2.0 * res["mean_R"] * rb + (20.0 if real else 16.0) * res["mean_R"]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 3),
            "unit": "Tops/s (int32 VALU)", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
            "kernel": sweep_kernel_name(res["cfg"]["L"], real) + " (N_S sweeps of every replica at one temperature)",
            "ops_per_attempt": opa,
            "sweep_shape": {"tile_rows": res["shape"][0], "group_replicas": res["shape"][1]},
            "avg_launch_ms": round(res["sweep_ms"] / max(1, res["nsteps"]), 4),
            "hbm_gbs_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9, 1),
            "hbm_frac_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9
                                          / HBM_PEAK_GBS, 4)}


def cpu_baseline(name, n_steps, real=False):
    import oracle

    cfg, J, beta = workload_inputs(name, real)
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


def batch_bench(n_inst, plain_per_L):
    """Mixed-size batch: all instances annealed together (graph-replayed
    steps) against separate per-instance runs on a stratified sample."""
    import torch

    from paper_1710_09025_amd import Pamc, PamcBatch, autotune

    insts = pi.batch_instances(n_inst)
    t0 = time.perf_counter()
    b = PamcBatch(insts, autotune=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = b.anneal()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert st == 0, st
    # attempts actually run: sum_k R_k N N_S over every instance
    att_run = 0.0
    for i in range(0, n_inst):
        o = b.observables(i)
        att_run += float(np.sum(o["R"])) * insts[i]["L"] ** 3 * insts[i]["sweeps"]
    b.close()
    del b
    torch.cuda.empty_cache()
    # per-instance runs: plain_per_L instances of each size, one after another
    per_L = {}
    for L in sorted({d["L"] for d in insts}):
        sample = [d for d in insts if d["L"] == L][:plain_per_L]
        ts, tc = [], []
        for d in sample:
            c0 = time.perf_counter()
            p = Pamc(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"], autotune=True)
            torch.cuda.synchronize()
            c1 = time.perf_counter()
            assert p.anneal() == 0
            torch.cuda.synchronize()
            c2 = time.perf_counter()
            p.close()
            ts.append(c2 - c1)
            tc.append(c2 - c0)
        per_L[L] = (float(np.mean(ts)), float(np.mean(tc)), len(sample))
    count = {L: sum(1 for d in insts if d["L"] == L) for L in per_L}
    shapes = {}
    for L in per_L:
        d = next(d for d in insts if d["L"] == L)
        t, g, ns = autotune(L, d["R"], d["sweeps"])  # cached: the shapes both sides used
        shapes[str(L)] = {"tile_rows": t, "group_replicas": g, "sweep_ns_per_attempt": round(ns, 6)}
    plain_anneal = sum(count[L] * per_L[L][0] for L in per_L)
    plain_total = sum(count[L] * per_L[L][1] for L in per_L)
    return {
        "instances": n_inst,
        "batched_instances_per_s": round(n_inst / (t2 - t1), 3),
        "batched_instances_per_s_incl_create": round(n_inst / (t2 - t0), 3),
        "batched_attempts_per_ns": round(att_run / ((t2 - t1) * 1e9), 3),
        "batched_anneal_s": round(t2 - t1, 3),
        "plain_instances_per_s": round(n_inst / plain_anneal, 3),
        "plain_instances_per_s_incl_create": round(n_inst / plain_total, 3),
        "plain_sample": f"{plain_per_L} per L, extrapolated by instance count",
        "speedup": round(plain_anneal / (t2 - t1), 3),
        "sweep_shapes_autotuned": shapes,
    }


def schedule_bench(name, kind):
    """One anneal of a workload under the paper's LBLT or TSPL schedule
    (Sec. III.B), or TSPL with the clipped exponential population schedule
    (Sec. III.D; same mean population), timed like the main line."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, _ = workload_inputs(name)
    nT = cfg["n_temps"]
    beta = pi.lblt_beta(cfg["beta_max"], nT) if kind == "lblt" else pi.tspl_beta(cfg["beta_max"], nT)
    pop = pi.clipped_exponential_population(beta, cfg["R"]) if kind == "tspl_dynamic_R" else None
    R = int(pop[0]) if pop is not None else cfg["R"]
    p = Pamc(cfg["L"], J, R, beta, cfg["sweeps"], cfg["seed"], autotune=True, pop_schedule=pop)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert p.anneal() == 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = p.observables()
    p.close()
    torch.cuda.empty_cache()
    att = attempts_of(obs, cfg["L"] ** 3, cfg["sweeps"])
    return {"schedule": kind, "attempts_per_ns": round(att / ((t1 - t0) * 1e9), 3),
            "ms_per_anneal": round((t1 - t0) * 1e3, 3), "final_rho_s": round(float(obs["rho_s"][-1]), 3),
            "final_S_f": round(float(obs["S_f"][-1]), 4), "peak_R": int(np.max(obs["R"]))}


def rho_f_bench(L=8, R=20000, n_temps=201, runs=128, icm_rounds=0, icm_beta_min=0.0):
    """rho_f = R var(beta F) from independent runs of one instance (Eq. (4)),
    annealed together as one batch (with cluster moves when icm_rounds > 0)."""
    import torch

    from paper_1710_09025_amd import free_energy_variance

    J = pi.pm_j_couplings(L, 2)
    beta = pi.linear_beta(5.0, n_temps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = free_energy_variance(L, J, R, beta, 10, [7000 + i for i in range(runs)], autotune=True,
                               icm_rounds=icm_rounds, icm_beta_min=icm_beta_min)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return {"L": L, "R": R, "n_temps": n_temps, "runs": runs, "icm_rounds": icm_rounds, "icm_beta_min": icm_beta_min,
            "rho_f_final": round(float(res["rho_f"][-1]), 4), "rho_f_max": round(float(np.max(res["rho_f"])), 4),
            "seconds": round(t1 - t0, 3)}


def rho_f_square_bench(L=8, R=50000, n_temps=101, runs=64, instances=(1, 2, 3, 4), icm_rounds=2):
    """The paper's 2D cluster-move comparison: rho_f = R var(beta F) of each
    Gaussian square-lattice instance from `runs` independent runs, without
    and with icm_rounds x floor(R_k/2) pair updates at every step."""
    import torch

    from paper_1710_09025_amd import free_energy_variance

    beta = pi.linear_beta(5.0, n_temps)
    out = {"L": L, "R": R, "n_temps": n_temps, "runs": runs, "icm_rounds": icm_rounds, "instances": {}}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in instances:
        J = pi.gaussian_couplings(L, 9000 + d, dim=2)
        row = {}
        for rounds in (0, icm_rounds):
            res = free_energy_variance(L, J, R, beta, 10, [11000 + 100 * d + i for i in range(runs)],
                                       autotune=True, icm_rounds=rounds)
            row["rho_f_icm" if rounds else "rho_f"] = round(float(res["rho_f"][-1]), 3)
        out["instances"][str(d)] = row
    torch.cuda.synchronize()
    out["seconds"] = round(time.perf_counter() - t0, 3)
    ratios = [v["rho_f"] / v["rho_f_icm"] for v in out["instances"].values()]
    out["geomean_ratio_without_over_with"] = round(float(np.exp(np.mean(np.log(ratios)))), 3)
    return out


def icm_bench(name, rounds=2):
    """One anneal of a workload with isoenergetic cluster moves (Sec. IV):
    rounds x floor(R_k/2) pair updates per step between the two halves of
    the sweeps, timed like the main line; the attempts counted are the
    Metropolis ones, so the rate shows the cost of the cluster moves."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name)
    p = Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], autotune=True, icm_rounds=rounds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assert p.anneal() == 0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    obs = p.observables()
    p.close()
    torch.cuda.empty_cache()
    att = attempts_of(obs, cfg["L"] ** cfg.get("dim", 3), cfg["sweeps"])
    pairs = rounds * int(np.sum(obs["R"][1:] // 2))
    return {"icm_rounds": rounds, "attempts_per_ns": round(att / ((t1 - t0) * 1e9), 3),
            "ms_per_anneal": round((t1 - t0) * 1e3, 3), "pair_updates": pairs,
            "pair_updates_per_us": round(pairs / ((t1 - t0) * 1e6), 3)}


def warm_serving_shapes(sweeps=10):
    """Tunes the sweep shapes of the serving size classes before the stream
    (as a deployment would ship a tuning cache): every L of the request mix
    and a grid of populations covering its capacity classes."""
    from paper_1710_09025_amd import autotune

    t0 = time.perf_counter()
    for L in range(4, 15):
        for R in (5000, 8000, 12000, 16000, 24000, 32000, 40000, 50000):
            autotune(L, R, sweeps)
    return time.perf_counter() - t0


def serve_bench(n_req, rate, budget_gb):
    """Poisson request stream replayed in real time against the serving loop."""
    from paper_1710_09025_amd import PamcServer

    reqs = pi.serving_requests(n_req, rate=rate)
    srv = PamcServer(int(budget_gb * (1 << 30)), max_active=256, autotune=True)
    ids = []
    t0 = time.perf_counter()
    for d in reqs:
        now = time.perf_counter() - t0
        if d["arrival"] > now:
            time.sleep(d["arrival"] - now)
        ids.append(srv.submit(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"]))
    lat = []
    last = 0.0
    first = None
    for rid in ids:
        st, _, tm = srv.wait(rid, timeout=1200)
        assert st == 0, st
        lat.append(tm["finish"] - tm["submit"])
        last = max(last, tm["finish"])
        first = tm["submit"] if first is None else min(first, tm["submit"])
    srv.close()
    lat = np.array(lat)
    att = sum(float(d["R"]) * d["L"] ** 3 * d["sweeps"] * len(d["beta"]) for d in reqs)
    span = last - first
    return {"requests": n_req, "offered_rate_per_s": round(rate, 3), "hbm_budget_gb": budget_gb,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "instances_per_s": round(n_req / span, 3),
            "attempts_per_ns": round(att / (span * 1e9), 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed anneals")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="L8_R100000",
                    choices=sorted(k for k, v in pi.WORKLOADS.items() if v.get("dim", 3) == 3))
    ap.add_argument("--couplings", default="pm1", choices=("pm1", "gaussian"),
                    help="couplings of the benchmark instance: +-1, or Gaussian in fixed point")
    ap.add_argument("--icm-rounds", type=int, default=0,
                    help="isoenergetic cluster-move rounds per step in the main line (0: none)")
    ap.add_argument("--cpu-steps", type=int, default=16, help="temperature steps of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--batch", type=int, default=2000, help="instances of the mixed-size batch (0: skip)")
    ap.add_argument("--batch-plain", type=int, default=5, help="per-instance runs per L for the comparison")
    ap.add_argument("--serve", type=int, default=300, help="requests of the serving stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-light", type=int, default=150,
                    help="requests of the second stream at 0.8x the measured saturation rate (0: skip)")
    ap.add_argument("--gather-steps", type=int, default=20,
                    help="temperature steps of the stand-alone gather measurement (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    real = args.couplings == "gaussian"
    res = time_anneals(args.workload, args.steps, args.warmup, real=real, icm_rounds=args.icm_rounds)
    res["cfg"]["name"] = args.workload
    log(f"{args.workload} ({args.couplings}) timed")
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
        "data": f"synthetic: {'Gaussian' if real else '+-J'} couplings and Philox-initialised replicas from "
                "fixed seeds",
        "config": {"workload": f"3D EA {'Gaussian' if real else '+-J'} L={cfg['L']} periodic, R={cfg['R']}, n_temps={cfg['n_temps']} "
                               f"beta linear 0->{cfg['beta_max']}, N_S={cfg['sweeps']}, one instance",
                   "L": cfg["L"], "R": cfg["R"], "n_temps": cfg["n_temps"], "sweeps": cfg["sweeps"],
                   "step": "one complete anneal", "spins": "int8", "icm_rounds": args.icm_rounds},
        "sweep_attempts_per_ns": round(res["attempts_per_anneal"] / (res["sweep_ms"] * 1e6), 3),
        "sweep_share": round(res["sweep_ms"] / (res["sweep_ms"] + res["other_ms"]), 4),
        "roofline": roofline(res),
    }
    if args.gather_steps and not real:
        line["gather"] = {name: gather_bench(name, args.gather_steps) for name in (args.workload, "L16_R500000")}
        line["gather"]["L16_R500000_packed"] = gather_bench("L16_R500000", args.gather_steps, packed=True)
        log("gather legs done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_steps if not real else max(1, args.cpu_steps // 4),
                                            real)
        log("cpu baseline done")
    if not args.no_extra:
        extra = {}
        for name, k, w, packed in (("L4_R1000", 5, 1, False), ("L16_R500000", 1, 0, False),
                                   ("L16_R500000", 1, 0, True)):
            if name == args.workload and not packed:
                continue
            r = time_anneals(name, k, w, packed=packed)
            log(f"{name}{' packed' if packed else ''} done")
            extra[name + ("_packed" if packed else "")] = {
                "attempts_per_ns": round(r["attempts_per_anneal"] * k / (r["wall_s"] * 1e9), 3),
                "sweep_attempts_per_ns": round(r["attempts_per_anneal"] / (r["sweep_ms"] * 1e6), 3),
                "ms_per_anneal": round(r["wall_s"] / k * 1e3, 3),
                "sweep_share": round(r["sweep_ms"] / (r["sweep_ms"] + r["other_ms"]), 4),
                "spins": "packed" if packed else "int8",
                "footprint_gb": footprint_gb(name, packed),
                "sweep_shape": {"tile_rows": r["shape"][0], "group_replicas": r["shape"][1]},
            }
        if not real:
            # the paper's own case study: Gaussian couplings, same workload
            g = time_anneals(args.workload, 3, 1, real=True)
            g["cfg"]["name"] = args.workload
            extra[args.workload + "_gaussian"] = {
                "attempts_per_ns": round(g["attempts_per_anneal"] * 3 / (g["wall_s"] * 1e9), 3),
                "sweep_attempts_per_ns": round(g["attempts_per_anneal"] / (g["sweep_ms"] * 1e6), 3),
                "ms_per_anneal": round(g["wall_s"] / 3 * 1e3, 3),
                "sweep_share": round(g["sweep_ms"] / (g["sweep_ms"] + g["other_ms"]), 4),
                "roofline": roofline(g),
                "cpu_baseline": cpu_baseline(args.workload, 3, real=True),
            }
            log("gaussian leg done")
        for kind in ("lblt", "tspl", "tspl_dynamic_R"):
            extra[f"{args.workload}_{kind}"] = schedule_bench(args.workload, kind)
            log(f"schedule {kind} done")
        extra["rho_f"] = rho_f_bench()
        extra[f"{args.workload}_icm"] = icm_bench(args.workload)
        extra["rho_f_icm"] = rho_f_bench(icm_rounds=2)
        # only below T = 1, around and below the spin-glass transition
        extra["rho_f_icm_low_T"] = rho_f_bench(icm_rounds=2, icm_beta_min=1.0)
        log("rho_f and cluster moves done")
        # the square lattice (Sec. II.A): throughput at the paper's largest
        # 2D size, and its cluster-move comparison of rho_f
        s = time_anneals("L32_2D_R1000000", 1, 0)
        extra["L32_2D_R1000000"] = {
            "attempts_per_ns": round(s["attempts_per_anneal"] / (s["wall_s"] * 1e9), 3),
            "sweep_attempts_per_ns": round(s["attempts_per_anneal"] / (s["sweep_ms"] * 1e6), 3),
            "ms_per_anneal": round(s["wall_s"] * 1e3, 3),
            "sweep_share": round(s["sweep_ms"] / (s["sweep_ms"] + s["other_ms"]), 4),
            "sweep_shape": {"tile_rows": s["shape"][0], "group_replicas": s["shape"][1]},
        }
        # the same with two cluster-move rounds per step, the paper's 2D setting
        extra["L32_2D_R1000000_icm"] = icm_bench("L32_2D_R1000000")
        # rho_f is intensive (independent of R once R >> rho_f), so the larger
        # lattices use R = 5 10^4 to afford more runs and instances
        extra["rho_f_2D_L8"] = rho_f_square_bench()
        extra["rho_f_2D_L16"] = rho_f_square_bench(L=16, R=50000, runs=64)
        extra["rho_f_2D_L32"] = rho_f_square_bench(L=32, R=50000, n_temps=301, runs=32, instances=(1, 2))
        log("square lattice done")
        if args.batch:
            extra["batch_mixed_L"] = batch_bench(args.batch, args.batch_plain)
            log("batch done")
        if args.serve:
            warm = warm_serving_shapes()
            sat = serve_bench(args.serve, args.serve_rate, args.serve_budget_gb)
            sat["shape_tuning_before_stream_s"] = round(warm, 2)
            extra["serving"] = sat
            log("serving done")
            if args.serve_light:
                extra["serving_at_0.8x_saturation"] = serve_bench(
                    args.serve_light, 0.8 * sat["instances_per_s"], args.serve_budget_gb)
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
