#!/usr/bin/env python3
"""Benchmark: population annealing of a 3D +-J Edwards-Anderson instance on one
MI355X, reported as spin-flip attempts per nanosecond.

One benchmark step is one complete anneal of the workload (every row of the
hot path: N_S checkerboard Metropolis sweeps of every replica at each of the
n_temps temperatures, energy histogram, FP64 weight normalisation, copy
counts, prefix sum and gather of the surviving replicas, family and overlap
statistics).  The default workload is the largest one a single GPU runs: L =
16, R = 5 10^5, 301 temperatures, one byte per spin.  Inputs (couplings,
initial population) are resident on the GPU before the timed region; each
timed anneal runs on its own, freshly created run handle.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel (the sweep) against the chip's integer
                VALU peak, timed live with HIP events on the run's stream;
  cpu_baseline  the CPU oracle on a row sample of the same anneal, timed
                at one thread and at the host's threads and extrapolated;
  gather        the HBM-bound kernel of the path (stand-alone gather of the
                surviving replicas) against the HBM peak;
  extra         the other workloads (bit-packed spins, L = 8 and L = 4
                instances, Gaussian couplings, schedules, rho_f, cluster
                moves, the square lattice, the 2000-instance batch against
                2000 separate runs with a result check, the serving loop,
                and the calibration kernels of the roofline).
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

# int32 VALU peak of MI355X: 256 CUs x 4 SIMDs, each issuing a plain 32-bit
# wave64 instruction every two cycles (128 lanes per CU per cycle; the fp32
# vector rate of 157.3 TFLOP/s counts an FMA as two), at 2.4 GHz: 78.6 T
# operations per second.  The calibration kernels confirm the lane rate
# (plain chains issue 1.6 wave instructions per CU per cycle, more than a
# 16-lane SIMD could).
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic int32 operations per spin-flip attempt of the sweep, per Philox
# block of four attempts (one Philox4x32-10 call):
#   Philox: 10 rounds x (2 widening multiplies + 2 three-input XORs) = 40,
#     of which the first round's products, its XOR with the replica word and
#     the second round's product and XOR of words fixed for the step are the
#     same in every sweep of a step (5), leaving 35;
#   local fields of the four sites packed one byte per site: 6 three-input
#     XORs + 3 adds (two three-input) + 1 byte-align = 10;
#   acceptance: 4 x (threshold index + compare + select into the flip mask)
#     + downhill mask (add, shift, and) + 2 merges of the partial masks = 17;
#   the flip applied to the word: 1;
# 63 / 4 = 15.75.  The compiled kernels issue 16.5 lane instructions per
# attempt (profiles/sweep_L16_R500000_valu_counters.md).
ALU_OPS_PER_ATTEMPT = 15.75
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


def time_anneals(name, steps, warmup, autotune=True, packed=False, real=False, icm_rounds=0, tile_rows=0,
                 group_replicas=0):
    """Creates warmup + steps run handles up front (each temperature step a
    replayed hipGraph; sweep shapes chosen by the autotuner at creation,
    outside the timed region) and anneals them one after another for the
    wall time; one more anneal with HIP events around every step's kernels
    gives the per-kernel device time."""
    import torch

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name, real)
    N = cfg["L"] ** cfg.get("dim", 3)
    shape_kw = dict(tile_rows=tile_rows, group_replicas=group_replicas)
    runs = [Pamc(cfg["L"], J, cfg["R"], beta, cfg["sweeps"], cfg["seed"], autotune=autotune, packed=packed,
                 icm_rounds=icm_rounds, **shape_kw) for _ in range(warmup + steps)]
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
                 packed=packed, icm_rounds=icm_rounds, **shape_kw)
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
                attempts_per_anneal=att, mean_R=Rbar, N=N, shape=shape, real=real, packed=packed,
                R_steps=np.array(obs["R"], dtype=np.float64))


def size_run(L, R, n_temps, tile_rows=0, group_replicas=0):
    """One timed anneal of a +-J instance of side L (R replicas, n_temps
    temperatures linear in beta up to 5, N_S = 10): the sweep rate of the
    kernel that size selects, for profiling one lattice size at a time.
    Without a tile the shape comes from the autotuner (whose trial launches
    then precede the anneal)."""
    from paper_1710_09025_amd import Pamc

    J = pi.pm_j_couplings(L, 7)
    beta = pi.linear_beta(5.0, n_temps)
    p = Pamc(L, J, R, beta, 10, 11, timing=True, autotune=tile_rows == 0, tile_rows=tile_rows,
             group_replicas=group_replicas)
    shape = p.sweep_shape()
    assert p.anneal() == 0
    sweep_ms, other_ms, _, nsteps = p.phase_times()
    obs = p.observables()
    p.close()
    att = attempts_of(obs, L ** 3, 10)
    return {"L": L, "R": R, "n_temps": n_temps, "shape": list(shape), "sweep_ms": round(sweep_ms, 3),
            "other_ms": round(other_ms, 3), "sweep_attempts_per_ns": round(att / (sweep_ms * 1e6), 1),
            "sum_E_last": int(obs["sum_E"][-1])}


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


def roofline(res, calib=None):
    sweep_s = res["sweep_ms"] / 1e3
    real = res.get("real", False)
    opa = ALU_OPS_PER_ATTEMPT_REAL if real else ALU_OPS_PER_ATTEMPT
    ops = opa * res["attempts_per_anneal"]
    achieved = ops / sweep_s / 1e12
    traffic = None
    key = res["cfg"].get("name", "") + ("_gaussian" if real else "") + ("_packed" if res.get("packed") else "")
    if os.path.exists(COUNTERS_FILE):
        try:
            c = json.load(open(COUNTERS_FILE))
            w = c.get("workloads", {}).get(key, None)
            if c.get("sweep_source_sha256_16") == source_hash() and w:
                traffic = w["hbm_bytes_per_launch"]
        except Exception:
            traffic = None
    rb = ((res["N"] + 15) // 16) * 16
    if res.get("packed"):
        rb = (rb + 127) // 128 * 16
    # tile in + out, map / energy / family
    alg_bytes = 2.0 * res["mean_R"] * rb + (20.0 if real else 16.0) * res["mean_R"]
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 3),
            "unit": "Tops/s (int32 VALU)", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
            "kernel": sweep_kernel_name(res["cfg"]["L"], real) + " (N_S sweeps of every replica at one temperature)",
            "ops_per_attempt": opa,
            "sweep_shape": {"tile_rows": res["shape"][0], "group_replicas": res["shape"][1]},
            "avg_launch_ms": round(res["sweep_ms"] / max(1, res["nsteps"]), 4),
            "hbm_gbs_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9, 1),
            "hbm_frac_algorithmic": round(alg_bytes / (res["sweep_ms"] / max(1, res["nsteps"]) / 1e3) / 1e9
                                          / HBM_PEAK_GBS, 4)}
    if calib and not real and "philox_words_per_ns" in calib:
        # one 32-bit Philox word per attempt: the draws alone, measured,
        # bound the attempts per ns of any sweep that makes them
        sweep_rate = res["attempts_per_anneal"] / (res["sweep_ms"] * 1e6)
        out["philox_only_words_per_ns"] = calib["philox_words_per_ns"]
        out["frac_of_philox_only_ceiling"] = round(sweep_rate / calib["philox_words_per_ns"], 4)
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, n_steps, real=False):
    """The oracle on the first n_steps temperature steps of a workload at its
    full population (small workloads)."""
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
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {n_steps} of {cfg['n_temps']} temperature steps of the same workload "
                      f"(full population R={cfg['R']}, L={cfg['L']}), {t1 - t0:.1f} s"}


def cpu_baseline_sampled(name, R_steps, rows_1t=448, rows_nt=6144, rows_resample=20000):
    """The oracle on a row sample of the workload's anneal, extrapolated to
    the whole anneal (the full run takes hours on the host).

    Sweeps: the first 10 temperature steps of the first rows of the initial
    population (the oracle's own, which equals the run's), and the last 10
    steps of rows sampled evenly from the population the GPU exported at
    step n_temps - 10; each sample is swept step after step by the oracle's
    sweep_rows (the same per-replica sweep its run uses), timed.  The time
    per row and step is interpolated linearly in k between the two samples.
    Resampling and measurement: the oracle's measure_resample of the first
    rows_resample rows of the exported population, timed, per row.  The
    whole anneal is then sum_k R_k (sweep + resampling time per row) with
    the GPU run's R_k.  Timed at one thread and at the host's threads."""
    import oracle

    from paper_1710_09025_amd import Pamc

    cfg, J, beta = workload_inputs(name)
    L, NS, nT = cfg["L"], cfg["sweeps"], cfg["n_temps"]
    N = L ** 3
    k_late = nT - 10
    p = Pamc(L, J, cfg["R"], beta, NS, cfg["seed"], autotune=True)
    assert p.anneal(k_late) == 0
    late = p.get_state()
    p.close()
    del p
    threads = min(16, os.cpu_count() or 1)
    o = oracle.Oracle(L, J, rows_nt, beta, NS, cfg["seed"], threads=threads)
    first = o.get_state()["spins"]
    Rs = min(rows_resample, late["R"])
    o2 = oracle.Oracle(L, J, Rs, beta, NS, cfg["seed"], threads=threads)
    out = {}
    t_all0 = time.perf_counter()
    for thr, rows in ((1, rows_1t), (threads, rows_nt)):
        o.set_threads(thr)
        o2.set_threads(thr)
        sp = first[:rows]
        idx = np.arange(rows, dtype=np.int64)
        t0 = time.perf_counter()
        for k in range(10):
            sp, _ = o.sweep_rows(k, idx, sp)
        early = (time.perf_counter() - t0) / (10 * rows)
        idx = np.linspace(0, late["R"] - 1, rows).astype(np.int64)
        sp = late["spins"][idx]
        t0 = time.perf_counter()
        for k in range(k_late, nT):
            sp, _ = o.sweep_rows(k, idx, sp)
        late_t = (time.perf_counter() - t0) / (10 * rows)
        o2.set_state(k_late, late["spins"][:Rs], np.arange(Rs, dtype=np.uint32), late["lnZ"])
        t0 = time.perf_counter()
        assert o2.measure_resample() == 0
        res_t = (time.perf_counter() - t0) / Rs
        ks = np.arange(nT, dtype=np.float64)
        per_row = np.interp(ks, [4.5, k_late + 4.5], [early, late_t]) + res_t
        total_s = float(np.sum(R_steps * per_row))
        att = float(np.sum(R_steps)) * N * NS
        out[thr] = (att / (total_s * 1e9), total_s, early, late_t, res_t)
    cpu_s = time.perf_counter() - t_all0
    v, total_s, early, late_t, res_t = out[threads]
    return {"value": round(v, 4), "unit": "attempts/ns", "cores": threads, "kind": "oracle",
            "extrapolated": True, "value_1_thread": round(out[1][0], 5),
            "full_anneal_s_extrapolated": round(total_s, 1),
            "full_anneal_s_extrapolated_1_thread": round(out[1][1], 1),
            "cpu_model": cpu_model(),
            "sample": f"{name}: sweeps of {rows_nt} rows ({rows_1t} at one thread) over the first 10 and the "
                      f"last 10 of {nT} temperature steps (late rows from the GPU's exported population at step "
                      f"{k_late}), and one measurement and resampling of {Rs} exported rows, timed and "
                      f"extrapolated to the whole anneal by the GPU run's population sizes; {cpu_s:.1f} s of "
                      f"timing",
            "ms_per_row_step": {"first_steps": round(early * 1e3, 4), "last_steps": round(late_t * 1e3, 4),
                                "resampling": round(res_t * 1e3, 6)}}


def batch_bench(n_inst, plain_n):
    """Mixed-size batch: all instances annealed together (graph-replayed
    steps) against plain_n separate runs, one after another on one stream
    (plain_n = n_inst runs every instance).  Every separate run's per-step
    records must equal its batched twin's; a mismatch fails the leg."""
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
    keys = ("R", "sum_E", "sum_E2", "E_min", "E_max", "lnZ", "S_f")
    batched = []
    for i in range(n_inst):
        o = b.observables(i)
        att_run += float(np.sum(o["R"])) * insts[i]["L"] ** 3 * insts[i]["sweeps"]
        batched.append({k: np.array(o[k]) for k in keys})
    b.close()
    del b
    torch.cuda.empty_cache()
    log(f"batch of {n_inst} annealed in {t2 - t1:.2f} s")
    # separate runs: the first plain_n instances (all of them by default)
    t_anneal, t_total, mismatches = 0.0, 0.0, []
    att_plain = 0.0
    for i, d in enumerate(insts[:plain_n]):
        c0 = time.perf_counter()
        p = Pamc(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"], autotune=True)
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        assert p.anneal() == 0
        torch.cuda.synchronize()
        c2 = time.perf_counter()
        o = p.observables()
        p.close()
        t_anneal += c2 - c1
        t_total += c2 - c0
        att_plain += float(np.sum(o["R"])) * d["L"] ** 3 * d["sweeps"]
        if any(list(np.asarray(o[k])) != list(batched[i][k]) for k in keys):
            mismatches.append(i)
    count = {}
    for d in insts:
        count[d["L"]] = count.get(d["L"], 0) + 1
    shapes = {}
    for L in sorted(count):
        d = next(d for d in insts if d["L"] == L)
        # cached: the separate runs tune for their own population, the batch
        # for the population of its launch of that size (at most 2e5 rows)
        t, g, ns = autotune(L, d["R"], d["sweeps"])
        tb, gb, nsb = autotune(L, min(count[L] * d["R"], 200_000), d["sweeps"])
        shapes[str(L)] = {"separate": {"tile_rows": t, "group_replicas": g, "sweep_ns_per_attempt": round(ns, 6)},
                          "batched": {"tile_rows": tb, "group_replicas": gb,
                                      "sweep_ns_per_attempt": round(nsb, 6)}}
    if mismatches:
        raise AssertionError(f"batched and separate runs differ for instances {mismatches[:10]}")
    full = plain_n >= n_inst
    plain_rate = plain_n / t_anneal
    return {
        "instances": n_inst,
        "batched_instances_per_s": round(n_inst / (t2 - t1), 3),
        "batched_instances_per_s_incl_create": round(n_inst / (t2 - t0), 3),
        "batched_attempts_per_ns": round(att_run / ((t2 - t1) * 1e9), 3),
        "batched_anneal_s": round(t2 - t1, 3),
        "plain_instances_per_s": round(plain_rate, 3),
        "plain_instances_per_s_incl_create": round(plain_n / t_total, 3),
        "plain_attempts_per_ns": round(att_plain / (t_anneal * 1e9), 3),
        "plain_anneal_s": round(t_anneal, 3),
        "plain_runs": plain_n,
        "plain_sample": "every instance, one run after another" if full else
                        f"the first {plain_n} of {n_inst} instances (a sample)",
        "batched_equals_plain": f"per-step R, sum E, sum E^2, E_min, E_max, ln Z, S_f identical for all "
                                f"{plain_n} separate runs",
        "speedup": round((n_inst / (t2 - t1)) / plain_rate, 3),
        "sweep_shapes_autotuned": shapes,
    }


def calibration():
    """Philox-only and plain-VALU rates of the device (pamc_calibrate)."""
    from paper_1710_09025_amd import calibrate

    words, valu = calibrate()
    return {"philox_words_per_ns": round(words, 1), "valu_int32_ops_per_ns": round(valu, 1),
            "valu_peak_ops_per_ns": round(ALU_PEAK_TOPS * 1e3, 1),
            "valu_frac_of_peak": round(valu / (ALU_PEAK_TOPS * 1e3), 4)}


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
    (found in the shipped tuning cache, so normally instant): every L of the
    request mix at the population the server tunes requests for."""
    from paper_1710_09025_amd import autotune

    t0 = time.perf_counter()
    for L in range(4, 15):
        # the server tunes every request for a population of 10^5 rows
        autotune(L, 100_000, sweeps)
    return time.perf_counter() - t0


def serve_bench(n_req, rate, budget_gb):
    """Poisson request stream replayed in real time against the serving loop;
    latency = completion - submission; GPU busy = device time of the step
    batches over the span from the first submission to the last completion."""
    from paper_1710_09025_amd import PamcServer

    reqs = pi.serving_requests(n_req, rate=rate)
    srv = PamcServer(int(budget_gb * (1 << 30)), max_active=256, autotune=True)
    ids = []
    busy0 = srv.usage()["busy_s"]
    t0 = time.perf_counter()
    for d in reqs:
        now = time.perf_counter() - t0
        if d["arrival"] > now:
            time.sleep(d["arrival"] - now)
        ids.append(srv.submit(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"]))
    lat = []
    last = 0.0
    first = None
    att = 0.0
    for rid, d in zip(ids, reqs):
        st, obs, tm = srv.wait(rid, timeout=1200)
        assert st == 0, st
        lat.append(tm["finish"] - tm["submit"])
        last = max(last, tm["finish"])
        first = tm["submit"] if first is None else min(first, tm["submit"])
        att += float(np.sum(obs["R"])) * d["L"] ** 3 * d["sweeps"]
    busy = srv.usage()["busy_s"] - busy0
    srv.close()
    lat = np.array(lat)
    span = last - first
    return {"requests": n_req, "offered_rate_per_s": round(rate, 3), "hbm_budget_gb": budget_gb,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "instances_per_s": round(n_req / span, 3),
            "attempts_per_ns": round(att / (span * 1e9), 3),
            "gpu_busy_frac": round(busy / span, 4)}


def line_for(res, steps):
    """Rate figures of one timed workload."""
    return {"attempts_per_ns": round(res["attempts_per_anneal"] * steps / (res["wall_s"] * 1e9), 3),
            "sweep_attempts_per_ns": round(res["attempts_per_anneal"] / (res["sweep_ms"] * 1e6), 3),
            "ms_per_anneal": round(res["wall_s"] / steps * 1e3, 3),
            "sweep_share": round(res["sweep_ms"] / (res["sweep_ms"] + res["other_ms"]), 4),
            "spins": "packed" if res.get("packed") else "int8",
            "sweep_shape": {"tile_rows": res["shape"][0], "group_replicas": res["shape"][1]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed anneals")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="L16_R500000",
                    choices=sorted(k for k, v in pi.WORKLOADS.items() if v.get("dim", 3) == 3))
    ap.add_argument("--couplings", default="pm1", choices=("pm1", "gaussian"),
                    help="couplings of the benchmark instance: +-1, or Gaussian in fixed point")
    ap.add_argument("--icm-rounds", type=int, default=0,
                    help="isoenergetic cluster-move rounds per step in the main line (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--batch", type=int, default=2000, help="instances of the mixed-size batch (0: skip)")
    ap.add_argument("--batch-plain", type=int, default=2000,
                    help="separate runs compared with the batch (the first this many instances)")
    ap.add_argument("--serve", type=int, default=300, help="requests of the serving stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-light", type=int, default=150,
                    help="requests of the second stream at 0.8x the measured saturation rate (0: skip)")
    ap.add_argument("--gather-steps", type=int, default=20,
                    help="temperature steps of the stand-alone gather measurement (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run the calibration kernels (Philox-only and plain VALU) and print their rates")
    ap.add_argument("--legs", default="",
                    help="comma-separated subset of the extra legs to run (default: all)")
    ap.add_argument("--packed", action="store_true", help="main line with bit-packed spin rows")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="main line with this sweep tile instead of the autotuned one (profiling)")
    ap.add_argument("--group-replicas", type=int, default=0,
                    help="main line with this colour-major replica group (with --tile-rows)")
    ap.add_argument("--size", type=int, default=0, metavar="L",
                    help="only anneal one +-J instance of side L (--size-replicas replicas, 201 temperatures) "
                         "and print its sweep rate (with --tile-rows / --group-replicas: that shape)")
    ap.add_argument("--size-replicas", type=int, default=200_000)
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

    if args.calibrate:
        print(json.dumps(calibration()), flush=True)
        return

    if args.size:
        print(json.dumps(size_run(args.size, args.size_replicas, 201, args.tile_rows, args.group_replicas)),
              flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs an instance on one device and has no "
              "multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    legs = set(x for x in args.legs.split(",") if x)

    def want(leg):
        return not legs or leg in legs

    real = args.couplings == "gaussian"
    fixed = args.tile_rows > 0
    res = time_anneals(args.workload, args.steps, args.warmup, real=real, icm_rounds=args.icm_rounds,
                       packed=args.packed, autotune=not fixed, tile_rows=args.tile_rows,
                       group_replicas=args.group_replicas)
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
        "config": {"workload": f"3D EA {'Gaussian' if real else '+-J'} L={cfg['L']} periodic, R={cfg['R']}, "
                               f"n_temps={cfg['n_temps']} beta linear 0->{cfg['beta_max']}, N_S={cfg['sweeps']}, "
                               "one instance, " + ("one bit per spin" if args.packed else "one byte per spin"),
                   "L": cfg["L"], "R": cfg["R"], "n_temps": cfg["n_temps"], "sweeps": cfg["sweeps"],
                   "step": "one complete anneal", "spins": "packed" if args.packed else "int8",
                   "icm_rounds": args.icm_rounds},
        "sweep_attempts_per_ns": round(res["attempts_per_anneal"] / (res["sweep_ms"] * 1e6), 3),
        "sweep_share": round(res["sweep_ms"] / (res["sweep_ms"] + res["other_ms"]), 4),
    }
    calib = calibration()
    line["roofline"] = roofline(res, calib)
    if args.gather_steps and not real:
        line["gather"] = {name: gather_bench(name, args.gather_steps) for name in ("L16_R500000", "L8_R100000")}
        line["gather"]["L16_R500000_packed"] = gather_bench("L16_R500000", args.gather_steps, packed=True)
        log("gather legs done")
    if not args.no_cpu_baseline:
        if real or args.workload == "L4_R1000":
            line["cpu_baseline"] = cpu_baseline(args.workload, 3 if real else 20, real)
        else:
            line["cpu_baseline"] = cpu_baseline_sampled(args.workload, res["R_steps"])
        log("cpu baseline done")
    if not args.no_extra:
        extra = {}
        line["extra"] = extra

        def leg(key, fn):
            """Runs one extra leg; a failure is recorded in its place."""
            if not want(key.split(":")[0]):
                return
            try:
                extra[key.split(":")[-1]] = fn()
            except Exception as e:  # noqa: BLE001
                extra[key.split(":")[-1]] = {"error": f"{type(e).__name__}: {e}"}
            log(f"{key} done")

        extra["calibration"] = calib
        if args.workload == "L16_R500000" and not real:
            def packed_leg():
                r = time_anneals("L16_R500000", max(1, args.steps - 1), 1, packed=True)
                r["cfg"]["name"] = "L16_R500000"
                out = line_for(r, max(1, args.steps - 1))
                out["footprint_gb"] = footprint_gb("L16_R500000", True)
                out["roofline"] = roofline(r, calib)
                return out
            leg("packed:L16_R500000_packed", packed_leg)

        def small_leg(name, k, w):
            def f():
                r = time_anneals(name, k, w)
                r["cfg"]["name"] = name
                out = line_for(r, k)
                out["footprint_gb"] = footprint_gb(name, False)
                out["roofline"] = roofline(r, calib)
                out["cpu_baseline"] = cpu_baseline(name, 16 if name == "L8_R100000" else 101)
                return out
            return f
        for name, k, w in (("L8_R100000", 5, 1), ("L4_R1000", 5, 1)):
            if name != args.workload:
                leg(f"small:{name}", small_leg(name, k, w))
        if not real:
            def gaussian_leg():
                g = time_anneals("L8_R100000", 3, 1, real=True)
                g["cfg"]["name"] = "L8_R100000"
                out = line_for(g, 3)
                out["roofline"] = roofline(g)
                out["cpu_baseline"] = cpu_baseline("L8_R100000", 3, real=True)
                return out
            leg("gaussian:L8_R100000_gaussian", gaussian_leg)
        for kind in ("lblt", "tspl", "tspl_dynamic_R"):
            leg(f"schedules:L8_R100000_{kind}", lambda kind=kind: schedule_bench("L8_R100000", kind))
        leg("rho_f:rho_f", rho_f_bench)
        leg("icm:L8_R100000_icm", lambda: icm_bench("L8_R100000"))
        leg("icm:rho_f_icm", lambda: rho_f_bench(icm_rounds=2))
        # only below T = 1, around and below the spin-glass transition
        leg("icm:rho_f_icm_low_T", lambda: rho_f_bench(icm_rounds=2, icm_beta_min=1.0))

        # the square lattice (Sec. II.A): throughput at the paper's largest
        # 2D size, and its cluster-move comparison of rho_f
        def square_leg():
            r = time_anneals("L32_2D_R1000000", 1, 0)
            return line_for(r, 1)
        leg("square:L32_2D_R1000000", square_leg)
        leg("square:L32_2D_R1000000_icm", lambda: icm_bench("L32_2D_R1000000"))
        # rho_f is intensive (independent of R once R >> rho_f), so the larger
        # lattices use R = 5 10^4 to afford more runs and instances
        leg("square:rho_f_2D_L8", rho_f_square_bench)
        leg("square:rho_f_2D_L16", lambda: rho_f_square_bench(L=16, R=50000, runs=64))
        leg("square:rho_f_2D_L32", lambda: rho_f_square_bench(L=32, R=50000, n_temps=301, runs=32,
                                                               instances=(1, 2)))
        if args.batch:
            leg("batch:batch_mixed_L", lambda: batch_bench(args.batch, min(args.batch, args.batch_plain)))
        if args.serve and want("serving"):
            t0 = time.perf_counter()
            warm_serving_shapes()
            warm = time.perf_counter() - t0
            leg("serving:serving", lambda: serve_bench(args.serve, args.serve_rate, args.serve_budget_gb))
            sat = extra.get("serving", {})
            if "instances_per_s" in sat:
                sat["shape_tuning_before_stream_s"] = round(warm, 2)
                if args.serve_light:
                    leg("serving:serving_at_0.8x_saturation",
                        lambda: serve_bench(args.serve_light, 0.8 * sat["instances_per_s"], args.serve_budget_gb))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
