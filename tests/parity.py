"""Helpers comparing the GPU library with the CPU oracle."""
import math
import os

import numpy as np

import oracle
import pamc_inputs as pi

REL_TOL = 1e-12  # floating-point observables; integers must match exactly
THREADS = min(16, os.cpu_count() or 1)


def rel_close(a, b, tol=REL_TOL):
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    b = np.atleast_1d(np.asarray(b, dtype=np.float64))
    both_nan = np.isnan(a) & np.isnan(b)
    diff = np.abs(a - b)
    scale = np.maximum(np.maximum(np.abs(a), np.abs(b)), 1e-300)
    ok = both_nan | (diff <= tol * scale) | (diff == 0)
    return bool(np.all(ok)), np.nonzero(~ok)[0]


def compare_run(gpu_obs, gpu_sums, orc, steps=None, what=""):
    """Per-step integer records bit-exact, normalisers bitwise, derived
    observables within REL_TOL."""
    rec = orc.records()
    oobs = orc.observables()
    n = orc.nT if steps is None else steps
    sl = slice(0, n)
    np.testing.assert_array_equal(gpu_obs["R"][sl], rec["R"][sl], err_msg=f"{what} R_k")
    np.testing.assert_array_equal(gpu_obs["sum_E"][sl], rec["sumE"][sl], err_msg=f"{what} sum E")
    np.testing.assert_array_equal(gpu_obs["sum_E2"][sl], rec["sumE2"][sl], err_msg=f"{what} sum E^2")
    np.testing.assert_array_equal(gpu_obs["E_min"][sl], rec["Emin"][sl], err_msg=f"{what} E_min")
    np.testing.assert_array_equal(gpu_obs["E_max"][sl], rec["Emax"][sl], err_msg=f"{what} E_max")
    S, T = gpu_sums
    # the oracle stores 0 where the GPU stores NaN (no resampling after the last step)
    last = orc.nT - 1
    idx = [k for k in range(n) if k != last]
    np.testing.assert_array_equal(S[idx], rec["S"][idx], err_msg=f"{what} normaliser S (bitwise)")
    np.testing.assert_array_equal(T[sl], rec["T"][sl], err_msg=f"{what} family term (bitwise)")
    for key in ("mean_E", "e", "C_V", "lnQ", "lnZ", "betaF", "f", "S_f", "rho_s", "q_abs", "q2", "q4",
                "g_SG"):
        ok, bad = rel_close(gpu_obs[key][sl], oobs[key][sl])
        assert ok, (what, key, bad[:5], gpu_obs[key][sl][bad[:5]], oobs[key][sl][bad[:5]])


def compare_state(gs, os_, what=""):
    assert gs["R"] == os_["R"], (what, gs["R"], os_["R"])
    np.testing.assert_array_equal(gs["family"], os_["family"], err_msg=f"{what} family")
    np.testing.assert_array_equal(gs["E"], os_["E"], err_msg=f"{what} energies")
    np.testing.assert_array_equal(gs["spins"], os_["spins"], err_msg=f"{what} spins")


def instance(L, R, nT, sweeps=10, beta_max=5.0, disorder_seed=1, seed=1):
    return dict(L=L, couplings=pi.pm_j_couplings(L, disorder_seed), R=R,
                beta=pi.linear_beta(beta_max, nT), sweeps=sweeps, seed=seed)


def run_oracle(inst, overlap_steps=None, capacity=None, steps=-1):
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      capacity=capacity, overlap_steps=overlap_steps, threads=THREADS)
    st = o.run(steps)
    return o, st


INT_KEYS = (("R", "R"), ("sum_E", "sumE"), ("sum_E2", "sumE2"), ("E_min", "Emin"), ("E_max", "Emax"))
FLOAT_KEYS = ("mean_E", "e", "C_V", "lnQ", "lnZ", "betaF", "f", "S_f", "rho_s", "q_abs", "q2", "q4", "g_SG")


def compare_obs(gpu_obs, orc, steps=None, what=""):
    """Per-step records of a run whose normalisers are not exported (batch
    members, served requests): integers bit-exact, derived observables
    within REL_TOL, over the first `steps` steps (all by default)."""
    rec = orc.records()
    oobs = orc.observables()
    sl = slice(0, orc.nT if steps is None else steps)
    for g, o in INT_KEYS:
        np.testing.assert_array_equal(gpu_obs[g][sl], rec[o][sl], err_msg=f"{what} {g}")
    for key in FLOAT_KEYS:
        ok, bad = rel_close(gpu_obs[key][sl], oobs[key][sl])
        assert ok, (what, key, bad[:5], gpu_obs[key][sl][bad[:5]], oobs[key][sl][bad[:5]])


def same_obs(a, b, what=""):
    """Two GPU runs of the same request: every observable identical."""
    for key in ("R", "sum_E", "sum_E2", "E_min", "E_max") + FLOAT_KEYS + ("measured",):
        x, y = np.asarray(a[key]), np.asarray(b[key])
        if x.dtype == object or np.issubdtype(x.dtype, np.integer):
            assert list(x) == list(y), (what, key)
        else:
            np.testing.assert_array_equal(x, y, err_msg=f"{what} {key}")
