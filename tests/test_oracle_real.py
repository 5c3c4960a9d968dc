"""Pins of the oracle's real-coupling mode (the paper's Gaussian case study,
Sec. II.A) against facts it does not compute itself: libm's exp, an
independent enumeration of every configuration, the +-1 coupling mode run on
the same couplings, direct numpy reweighting, closed forms and exact
symmetries of the dynamics.  A wrong scale, sign, index or rounding step in
the fixed-point energies, the binary32 acceptance or the per-replica weights
fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import pamc_inputs as pi

SCALE = 2.0 ** -20


# --------------------------------------------------------------------------
# The binary32 exponential and the acceptance rule
# --------------------------------------------------------------------------
def test_exp_f32_against_libm():
    xs = np.concatenate([np.linspace(-23.0, 0.0, 40001), -np.logspace(-9, math.log10(23.0), 4000),
                         -np.arange(0, 34) * math.log(2.0)])
    worst = 0.0
    for x in xs.astype(np.float32):
        if x < -23.0:
            continue
        got = oracle.exp_f32(float(x))
        ref = math.exp(float(x))
        worst = max(worst, abs(got - ref) / ref)
    # a few binary32 ulps (2^-24 relative each)
    assert worst < 4 * 2.0 ** -24, worst
    assert oracle.exp_f32(0.0) == 1.0
    assert oracle.exp_f32(-0.0) == 1.0


def test_exp_f32_is_monotone_on_a_fine_grid():
    xs = np.linspace(-23.0, 0.0, 20001).astype(np.float32)
    ys = np.array([oracle.exp_f32(float(x)) for x in xs])
    assert np.all(np.diff(ys) >= 0.0)


def _acceptance_threshold(bq, dE):
    """Smallest u that is rejected (every smaller u is accepted), by bisection
    over the decision function."""
    if oracle.real_accept(bq, dE, 0xFFFFFFFF):
        return 1 << 32
    lo, hi = 0, 0xFFFFFFFF  # accept(lo) unknown, reject(hi)
    if not oracle.real_accept(bq, dE, 0):
        return 0
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if oracle.real_accept(bq, dE, mid):
            lo = mid
        else:
            hi = mid
    return hi


def test_acceptance_probability_is_boltzmann_factor():
    """The fraction of uniform 32-bit draws accepted is exp(-beta dE) up to
    binary32 rounding: of beta 2^-20, dE and their product (each a relative
    2^-24 on x, so |x| 2^-24 on exp(x)) and of exp itself (a few 2^-24)."""
    rng = np.random.default_rng(5)
    for _ in range(150):
        beta = float(rng.uniform(0.05, 5.0))
        dE = int(rng.integers(1, 12 * (1 << 23)))
        bq = oracle.real_beta(beta)
        T = _acceptance_threshold(bq, dE)
        p = math.exp(-beta * dE * SCALE)
        if p * 2.0 ** 32 < 1.0:
            assert T <= 1
            continue
        x = beta * dE * SCALE
        assert abs(T / 2.0 ** 32 - p) <= (8 + 3 * x) * 2.0 ** -24 * p + 2.0 ** -32, (beta, dE, T, p)


def test_acceptance_extremes():
    bq = oracle.real_beta(1.0)
    # exp(x) 2^32 < 1 for x < -23: never accepted
    assert not oracle.real_accept(bq, int(24 * 2 ** 20), 0)
    # |x| below 2^-25: e rounds to 1, every draw accepted
    assert oracle.real_accept(oracle.real_beta(0.01), 1, 0xFFFFFFFF)
    # |x| = 2^-20 still rejects the largest draws
    assert not oracle.real_accept(bq, 1, 0xFFFFFFFF)
    # exactly at the Boltzmann factor of ln 2: half of the draws
    dE = int(round(math.log(2.0) / SCALE))
    T = _acceptance_threshold(bq, dE)
    assert abs(T - 2 ** 31) < 2 ** 31 * 4e-6


# --------------------------------------------------------------------------
# Energies
# --------------------------------------------------------------------------
def test_real_couplings_generator_is_gaussian():
    J = pi.gaussian_couplings(12, 3).astype(np.float64) * SCALE
    assert J.shape == (3, 12 ** 3)
    assert abs(J.mean()) < 0.05 and abs(J.var() - 1.0) < 0.05
    assert np.all(np.abs(J) < 8.0)


def test_energy_equals_enumeration_L2():
    L, N = 2, 8
    J = pi.gaussian_couplings(L, 11)
    E_all = oracle.all_energies_real(L, J)
    idx = np.arange(2 ** N)
    spins = np.where((idx[:, None] >> np.arange(N)[None, :]) & 1, 1, -1).astype(np.int8)
    o = oracle.Oracle(L, J, 4, [0.0], 1, 1)
    np.testing.assert_array_equal(o.energies(spins), E_all)
    # global flip symmetry and the Eq. (1) sum written out in numpy
    np.testing.assert_array_equal(E_all, E_all[::-1])
    x, y, z = idx[:N] % L, (idx[:N] // L) % L, idx[:N] // (L * L)
    nb = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z), x + L * (y + L * ((z + 1) % L))]
    E_np = np.zeros(2 ** N, dtype=np.int64)
    for d in range(3):
        E_np -= (spins.astype(np.int64) * J[d][None, :] * spins[:, nb[d]]).sum(axis=1)
    np.testing.assert_array_equal(E_all, E_np)


def test_energy_scales_with_pm1_couplings():
    """Real couplings j = +-2^20 (J = +-1 exactly): every energy is 2^20 times
    the +-1 mode's energy of the same spins."""
    L = 4
    Jpm = pi.pm_j_couplings(L, 12)
    Jq = Jpm.astype(np.int32) * (1 << 20)
    a = oracle.Oracle(L, Jpm, 50, [0.0], 1, 3)
    b = oracle.Oracle(L, Jq, 50, [0.0], 1, 3)
    s = a.get_state()["spins"]
    np.testing.assert_array_equal(b.energies(s), a.energies(s).astype(np.int64) << 20)


@pytest.mark.parametrize("L", [3, 4])
def test_incremental_energy_equals_recomputed(L):
    J = pi.gaussian_couplings(L, 41)
    o = oracle.Oracle(L, J, 200, pi.linear_beta(3.0, 12), 5, 6)
    for _ in range(12):
        assert o.run(1) == oracle.OK
        st = o.get_state()
        assert st["E"].dtype == np.int64
        np.testing.assert_array_equal(st["E"], o.energies(st["spins"]))
        assert np.all(np.diff(st["family"].astype(np.int64)) >= 0)


# --------------------------------------------------------------------------
# Dynamics against exact results
# --------------------------------------------------------------------------
def _gtest_pooled(counts, p, min_expected=5.0):
    """G statistic with bins of small expectation pooled into one."""
    n = counts.sum()
    e = p * n
    big = e >= min_expected
    c = np.append(counts[big], counts[~big].sum())
    ee = np.append(e[big], e[~big].sum())
    keep = ee > 0
    c, ee = c[keep], ee[keep]
    m = c > 0
    G = 2.0 * np.sum(c[m] * np.log(c[m] / ee[m]))
    return G, len(c) - 1


@pytest.mark.parametrize("beta,seed", [(0.4, 1), (1.2, 2)])
def test_fixed_beta_population_is_boltzmann(beta, seed):
    """From beta = 0, one resampling to beta, then constant beta: later
    resamplings weight every replica equally, so the replicas evolve as
    Metropolis chains whose configurations must follow the exact Boltzmann
    law over all 2^N configurations."""
    L, N, R = 2, 8, 6000
    J = pi.gaussian_couplings(L, 100 + seed)
    o = oracle.Oracle(L, J, R, [0.0] + [beta] * 24, 10, seed, threads=8)
    assert o.run() == oracle.OK
    st = o.get_state()
    assert np.all(np.diff(st["family"].astype(np.int64)) >= 0)
    E_all = oracle.all_energies_real(L, J).astype(np.float64) * SCALE
    w = np.exp(-beta * (E_all - E_all.min()))
    p = w / w.sum()
    code = ((st["spins"] > 0).astype(np.int64) << np.arange(N)[None, :]).sum(axis=1)
    counts = np.bincount(code, minlength=2 ** N).astype(np.float64)
    G, dof = _gtest_pooled(counts, p)
    assert G < dof + 10 * math.sqrt(2 * dof) + 20, (G, dof)
    # the test is not vacuous: the law at -beta is rejected
    q = np.exp(beta * (E_all - E_all.max()))
    q /= q.sum()
    G2, dof2 = _gtest_pooled(counts, q)
    assert G2 > dof2 + 10 * math.sqrt(2 * dof2) + 20


@pytest.mark.slow
def test_pamc_matches_exact_thermodynamics():
    L, N = 2, 8
    J = pi.gaussian_couplings(L, 203)
    E_all = oracle.all_energies_real(L, J)
    beta = pi.linear_beta(2.0, 31)
    ex = oracle.exact_thermo_real(E_all, N, beta)
    R, M = 3000, 10
    runs = []
    for seed in range(M):
        o = oracle.Oracle(L, J, R, beta, 10, 2000 + seed, threads=8)
        assert o.run() == oracle.OK
        runs.append(o.observables())
    for key in ("lnZ", "mean_E", "C_V"):
        vals = np.array([r[key] for r in runs])
        mean = vals.mean(axis=0)
        se = vals.std(axis=0, ddof=1) / math.sqrt(M)
        for k in (5, 10, 20, 30):
            tol = 5 * se[k] + 1e-3 * abs(ex[key][k]) + 1e-9
            assert abs(mean[k] - ex[key][k]) < tol, (key, k, mean[k], ex[key][k], se[k])
    assert runs[0]["lnZ"][0] == N * math.log(2.0)


# --------------------------------------------------------------------------
# Resampling
# --------------------------------------------------------------------------
def _post_sweep_energies(L, J, R, beta, k, st, seed):
    probe = oracle.Oracle(L, J, R, beta[: k + 1], 10, seed)
    probe.set_state(k, st["spins"], st["family"], st["lnZ"])
    assert probe.run(1) == oracle.OK
    return probe.get_state()["E"]


def test_normaliser_and_free_energy_step_match_direct_reweighting():
    """S_k = sum_i exp(-dbeta (E_i - E_min)) and ln Q_k =
    ln[(1/R_k) sum_i exp(-dbeta E_i)], evaluated with numpy's exp on the
    post-sweep energies (not the oracle's products of powers)."""
    L = 4
    J = pi.gaussian_couplings(L, 7)
    beta = pi.linear_beta(3.0, 12)
    o = oracle.Oracle(L, J, 400, beta, 10, 9)
    for k in range(len(beta) - 1):
        st = o.get_state()
        E = _post_sweep_energies(L, J, 400, beta, k, st, 9).astype(np.float64) * SCALE
        assert o.run(1) == oracle.OK
        rec = o.records()
        db = beta[k + 1] - beta[k]
        S = np.exp(-db * (E - E.min())).sum()
        assert abs(rec["S"][k] - S) <= 1e-12 * S, (k, rec["S"][k], S)
        a = -db * E
        lnQ = a.max() + math.log(np.exp(a - a.max()).sum()) - math.log(len(E))
        assert abs(rec["lnQ"][k] - lnQ) <= 1e-11 * max(1.0, abs(lnQ)), (k, rec["lnQ"][k], lnQ)
        assert rec["Emin"][k] * SCALE == E.min() and rec["Emax"][k] * SCALE == E.max()


def test_copy_numbers_are_floor_or_ceil_of_tau():
    L, R = 3, 500
    J = pi.gaussian_couplings(L, 8)
    beta = [0.0, 0.9]
    o = oracle.Oracle(L, J, R, beta, 10, 4)
    st0 = o.get_state()
    E = _post_sweep_energies(L, J, R, beta, 0, st0, 4).astype(np.float64) * SCALE
    assert o.run() == oracle.OK
    st = o.get_state()
    w = np.exp(-0.9 * (E - E.min()))
    tau = R * w / w.sum()
    n = np.bincount(st["family"].astype(np.int64), minlength=R)
    lo, hi = np.floor(tau), np.ceil(tau)
    assert np.all((n == lo) | (n == hi)), np.nonzero((n != lo) & (n != hi))[0][:5]
    assert abs(n.sum() - R) < 6 * math.sqrt(R)


def test_pm1_couplings_in_real_mode_follow_the_pm1_run():
    """Real couplings j = +-2^20 describe the same model as +-1 couplings.
    The two modes round differently (binary32 acceptance, per-replica
    weights), which changes a decision only when a draw falls within a few
    parts in 2^24 of its threshold; for this seed none does, so the runs
    coincide replica by replica and their energies differ by the scale."""
    L, R = 4, 300
    Jpm = pi.pm_j_couplings(L, 13)
    Jq = Jpm.astype(np.int32) * (1 << 20)
    beta = pi.linear_beta(2.5, 9)
    a = oracle.Oracle(L, Jpm, R, beta, 5, 21)
    b = oracle.Oracle(L, Jq, R, beta, 5, 21)
    assert a.run() == oracle.OK and b.run() == oracle.OK
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sb["spins"], sa["spins"])
    np.testing.assert_array_equal(sb["family"], sa["family"])
    np.testing.assert_array_equal(sb["E"], sa["E"].astype(np.int64) << 20)
    oa, ob = a.observables(), b.observables()
    for key in ("mean_E", "C_V", "lnZ", "S_f"):
        np.testing.assert_allclose(ob[key], oa[key], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("L", [3, 4])
def test_gauge_transform_gives_gauge_image_trajectory(L):
    N, R = L ** 3, 150
    J = pi.gaussian_couplings(L, 51)
    eps = (2 * np.random.default_rng(4).integers(0, 2, N) - 1).astype(np.int8)
    Jg = pi.gauge_transform(L, J, eps)
    assert Jg.dtype == np.int32
    beta = pi.linear_beta(3.0, 10)
    a = oracle.Oracle(L, J, R, beta, 4, 8)
    b = oracle.Oracle(L, Jg, R, beta, 4, 8)
    s0 = a.get_state()
    b.set_state(0, s0["spins"] * eps[None, :], s0["family"], s0["lnZ"])
    assert a.run() == oracle.OK and b.run() == oracle.OK
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sb["spins"], sa["spins"] * eps[None, :])
    np.testing.assert_array_equal(sb["E"], sa["E"])
    np.testing.assert_array_equal(sb["family"], sa["family"])


def test_invalid_real_couplings_are_rejected():
    L = 3
    J = pi.gaussian_couplings(L, 1)
    J[1, 5] = 1 << 23  # |J| = 8
    with pytest.raises(ValueError):
        oracle.Oracle(L, J, 10, [0.0], 1, 1)
