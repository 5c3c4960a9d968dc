"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Every check compares the oracle with something it does not compute: an
independent Philox implementation (rocRAND), exact enumeration of all
configurations, an independently built hypercube graph, closed forms, or
exact symmetries of the dynamics.  A dropped term, wrong sign, wrong
neighbour or coupling index, or wrong resampling rule fails at least one.
"""
import itertools
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import pamc_inputs as pi

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND (an independent implementation)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_tool():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp(prefix="rocrand_philox_")
    exe = os.path.join(d, "rocrand_philox")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "helpers", "rocrand_philox.cpp"), "-o", exe],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_tool):
    rng = np.random.default_rng(123)
    cases = rng.integers(0, 2**32, size=(400, 6), dtype=np.uint64)
    cases[0] = 0
    cases[1] = 2**32 - 1
    cases[2, :4] = [0, 5, 7, 0x20000003]  # shaped like a sweep counter
    text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([rocrand_tool], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(w, 16) for w in line.split()] for line in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    mine = np.array([oracle.philox4x32_10(c[:4], c[4:]) for c in cases], dtype=np.uint64)
    assert ref.shape == mine.shape
    np.testing.assert_array_equal(mine, ref)
    # the input module's vectorised Philox (it draws the +-J instances)
    for key in ((0, 0), (1, 0), (0xDEADBEEF, 0x12345678)):
        c = cases.copy()
        c[:, 4], c[:, 5] = key
        text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in c) + "\n"
        out = subprocess.run([rocrand_tool], input=text, capture_output=True, text=True, check=True)
        ref = np.array([[int(w, 16) for w in line.split()] for line in out.stdout.strip().splitlines()],
                       dtype=np.uint64)
        got = pi.philox4x32_10(c[:, :4], key[0] | (key[1] << 32)).astype(np.uint64)
        np.testing.assert_array_equal(got, ref)


# --------------------------------------------------------------------------
# Lattice, colouring, thresholds
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", list(range(2, 17)))
def test_colouring_is_proper_and_ranks_are_bijective(L):
    J = pi.pm_j_couplings(L, 11)
    o = oracle.Oracle(L, J, 1, [0.0], 1, 1)
    ncol, col, rank = o.colouring()
    assert ncol == (2 if L % 2 == 0 else 3)
    nb = o.neighbours()
    for d in range(6):
        assert np.all(col != col[nb[:, d]]), "neighbouring sites share a colour"
    for c in range(ncol):
        r = np.sort(rank[col == c])
        np.testing.assert_array_equal(r, np.arange(len(r)))
        # ranks follow lexicographic site order
        sites = np.nonzero(col == c)[0]
        np.testing.assert_array_equal(rank[sites], np.arange(len(sites)))


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_neighbours_are_periodic_unit_steps(L):
    o = oracle.Oracle(L, pi.pm_j_couplings(L, 3), 1, [0.0], 1, 1)
    nb = o.neighbours()
    s = np.arange(L ** 3)
    x, y, z = s % L, (s // L) % L, s // (L * L)
    want = np.stack([(x + 1) % L + L * (y + L * z), (x - 1) % L + L * (y + L * z),
                     x + L * ((y + 1) % L + L * z), x + L * ((y - 1) % L + L * z),
                     x + L * (y + L * ((z + 1) % L)), x + L * (y + L * ((z - 1) % L))], axis=1)
    np.testing.assert_array_equal(nb, want)


def test_thresholds_golden():
    # tests/golden/thresholds.txt: hand-derived values (see the file header).
    path = os.path.join(HERE, "golden", "thresholds.txt")
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        b, t4, t8, t12, flag = line.split()
        T, all_ = oracle.thresholds(float(b))
        assert all_ == bool(int(flag))
        if not all_:
            assert list(T) == [int(t4), int(t8), int(t12)], (b, T)


def test_thresholds_monotone_and_bounded():
    prev = None
    for b in np.linspace(1e-6, 6, 200):
        T, all_ = oracle.thresholds(float(b))
        assert not all_
        assert T[0] >= T[1] >= T[2]
        # floor(p 2^32) within one unit of the exact probability
        for j, dE in enumerate((4, 8, 12)):
            p = math.exp(-b * dE)
            assert abs(int(T[j]) - p * 2**32) <= 1.0 + 1e-6 * p * 2**32
        if prev is not None:
            assert np.all(T <= prev)
        prev = T


# --------------------------------------------------------------------------
# Enumeration against independent brute force
# --------------------------------------------------------------------------
def _hypercube_ferro_energies():
    """L = 2 periodic lattice = 3-cube whose 12 edges each carry two bonds.
    Vertex v = x + 2y + 4z, neighbours v ^ (1 << d).  Built without the
    lattice code of the oracle."""
    E = []
    for conf in range(256):
        S = [1 if (conf >> v) & 1 else -1 for v in range(8)]
        e = 0
        for v in range(8):
            for d in range(3):
                w = v ^ (1 << d)
                if v < w:
                    e -= 2 * S[v] * S[w]  # two parallel bonds of J = +1
        E.append(e)
    return np.array(E)


def test_enumeration_L2_ferro_matches_hypercube():
    J = pi.ferro_couplings(2)
    g = oracle.density_of_states(2, J)
    E = _hypercube_ferro_energies()
    want = np.bincount((E + 24) // 2, minlength=25)
    np.testing.assert_array_equal(g, want)
    np.testing.assert_array_equal(np.sort(oracle.all_energies(2, J)), np.sort(E))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_enumeration_L2_random_matches_numpy(seed):
    L, N = 2, 8
    J = pi.pm_j_couplings(L, seed)
    # numpy brute force over all 256 configurations from explicit bonds
    confs = np.array([[1 if (c >> s) & 1 else -1 for s in range(N)] for c in range(2 ** N)])
    s = np.arange(N)
    x, y, z = s % L, (s // L) % L, s // (L * L)
    nbs = [(x + 1) % L + L * (y + L * z), x + L * ((y + 1) % L + L * z),
           x + L * (y + L * ((z + 1) % L))]
    E = np.zeros(2 ** N, dtype=np.int64)
    for d in range(3):
        E -= (confs * J[d][None, :] * confs[:, nbs[d]]).sum(axis=1)
    np.testing.assert_array_equal(oracle.all_energies(L, J), E)
    g = oracle.density_of_states(L, J)
    np.testing.assert_array_equal(g, np.bincount((E + 3 * N) // 2, minlength=3 * N + 1))


@pytest.mark.slow
def test_enumeration_L3_sums_and_gauge_invariance():
    L, N = 3, 27
    J = pi.pm_j_couplings(L, 5)
    g = oracle.density_of_states(L, J)
    assert g.sum() == 2 ** N
    # a gauge transformation only relabels configurations
    eps = (2 * np.random.default_rng(9).integers(0, 2, N) - 1).astype(np.int8)
    g2 = oracle.density_of_states(L, pi.gauge_transform(L, J, eps))
    np.testing.assert_array_equal(g, g2)
    # ferromagnet: two ground states at E = -3N; odd L frustrates E = +3N
    gf = oracle.density_of_states(L, pi.ferro_couplings(L))
    assert gf[0] == 2 and gf[-1] == 0 and gf.sum() == 2 ** N


def test_oracle_energy_equals_enumeration_L2():
    L, N = 2, 8
    J = pi.pm_j_couplings(L, 21)
    o = oracle.Oracle(L, J, 1, [0.0], 1, 1)
    confs = np.array([[1 if (c >> s) & 1 else -1 for s in range(N)] for c in range(2 ** N)],
                     dtype=np.int8)
    np.testing.assert_array_equal(o.energies(confs), oracle.all_energies(L, J))


@pytest.mark.parametrize("L", [3, 4, 5])
def test_mattis_ground_state_energy(L):
    J, eps = pi.mattis_couplings(L, 17)
    o = oracle.Oracle(L, J, 1, [0.0], 1, 1)
    E = o.energies(np.stack([eps, -eps]).astype(np.int8))
    assert list(E) == [-3 * L ** 3, -3 * L ** 3]


# --------------------------------------------------------------------------
# Metropolis dynamics: detailed balance against exact Boltzmann weights
# --------------------------------------------------------------------------
def _gtest(counts, probs):
    """G statistic and degrees of freedom, merging bins with expectation < 5."""
    n = counts.sum()
    exp_ = probs * n
    order = np.argsort(exp_)
    c_m, e_m, acc_c, acc_e = [], [], 0.0, 0.0
    for i in order:
        acc_c += counts[i]
        acc_e += exp_[i]
        if acc_e >= 5:
            c_m.append(acc_c)
            e_m.append(acc_e)
            acc_c = acc_e = 0.0
    if acc_e > 0 and c_m:
        c_m[-1] += acc_c
        e_m[-1] += acc_e
    c_m, e_m = np.array(c_m), np.array(e_m)
    m = c_m > 0
    G = 2 * np.sum(c_m[m] * np.log(c_m[m] / e_m[m]))
    return G, len(c_m) - 1


def _boltzmann(g, N, beta):
    E = np.arange(len(g)) * 2 - 3 * N
    lw = np.where(g > 0, np.log(np.maximum(g, 1)) - beta * E, -np.inf)
    w = np.exp(lw - lw.max())
    return w / w.sum()


@pytest.mark.parametrize("L,beta,R,seed", [(2, 0.3, 6000, 1), (2, 1.0, 6000, 2), (3, 0.5, 12000, 3),
                                           (4, 0.35, 3000, 4)])
def test_fixed_beta_population_is_boltzmann(L, beta, R, seed):
    """Every run starts at beta = 0; after the first resampling the
    temperature stays at beta, so every later weight is 1 (tau = R / R_k,
    copies independent of the state) and the replicas evolve as Metropolis
    chains at beta.  After burn-in their energies must follow the exact
    Boltzmann distribution g(E) e^{-beta E} / Z."""
    N = L ** 3
    J = pi.pm_j_couplings(L, 100 + L)
    nT = 25
    o = oracle.Oracle(L, J, R, [0.0] + [beta] * (nT - 1), 10, seed, threads=8)
    assert o.run() == oracle.OK
    st = o.get_state()
    assert abs(st["R"] - R) < 8 * math.sqrt(R)
    assert np.all(np.diff(st["family"].astype(np.int64)) >= 0)
    if N <= 27:
        g = oracle.density_of_states(L, J)
        p = _boltzmann(g, N, beta)
        counts = np.bincount((st["E"] + 3 * N) // 2, minlength=3 * N + 1).astype(float)
        G, dof = _gtest(counts, p)
        # chi-square(dof) upper tail p ~ 1e-6
        assert G < dof + 10 * math.sqrt(2 * dof) + 20, (G, dof)
    else:
        # L = 4: no enumeration; check the mean energy is stationary instead
        obs = o.observables()
        late = obs["mean_E"][10:]
        assert np.std(late) < 0.05 * abs(np.mean(late)) + 1.0


def test_sweep_sign_matters():
    """Planting the wrong sign of dE makes the fixed-beta test fail; the
    comparison itself must not be vacuous.  (Checked on the exact law: an
    anti-Boltzmann distribution differs from the Boltzmann one.)"""
    L, N = 2, 8
    J = pi.pm_j_couplings(L, 102)
    g = oracle.density_of_states(L, J)
    p = _boltzmann(g, N, 1.0)
    q = _boltzmann(g, N, -1.0)
    counts = np.round(q * 6000)
    G, dof = _gtest(counts, p)
    assert G > dof + 10 * math.sqrt(2 * dof) + 20


# --------------------------------------------------------------------------
# Annealing: free energy, <E>, C_V against exact enumeration
# --------------------------------------------------------------------------
@pytest.mark.slow
@pytest.mark.parametrize("L", [2, 3])
def test_pamc_matches_exact_thermodynamics(L):
    N = L ** 3
    J = pi.pm_j_couplings(L, 200 + L)
    g = oracle.density_of_states(L, J)
    beta = pi.linear_beta(2.0, 41)
    ex = oracle.exact_thermo(g, N, beta)
    R, M = 3000, 12
    runs = []
    for seed in range(M):
        o = oracle.Oracle(L, J, R, beta, 10, 1000 + seed, threads=8)
        assert o.run() == oracle.OK
        runs.append(o.observables())
    for key in ("lnZ", "mean_E", "C_V"):
        vals = np.array([r[key] for r in runs])
        mean = vals.mean(axis=0)
        se = vals.std(axis=0, ddof=1) / math.sqrt(M)
        for k in (5, 10, 20, 30, 40):
            tol = 5 * se[k] + 1e-3 * abs(ex[key][k]) + 1e-9
            assert abs(mean[k] - ex[key][k]) < tol, (key, k, mean[k], ex[key][k], se[k])
    # beta = 0 anchor is exact
    assert runs[0]["lnZ"][0] == N * math.log(2.0)


def test_free_energy_step_matches_direct_reweighting():
    """ln Q_k = ln[(1/R_k) sum_i exp(-(beta_{k+1}-beta_k) E_i)] over the
    population measured at step k, evaluated here with a direct log-sum-exp
    of the energies (not the oracle's power-product weights)."""
    L = 4
    J = pi.pm_j_couplings(L, 7)
    beta = pi.linear_beta(3.0, 16)
    o = oracle.Oracle(L, J, 500, beta, 10, 9)
    for k in range(len(beta) - 1):
        st = o.get_state()
        # a copy whose last step is k sees the same post-sweep population
        probe = oracle.Oracle(L, J, 500, beta[: k + 1], 10, 9)
        probe.set_state(k, st["spins"], st["family"], st["lnZ"])
        assert probe.run(1) == oracle.OK
        E = probe.get_state()["E"].astype(np.float64)
        assert o.run(1) == oracle.OK
        lnQ_oracle = o.records()["lnQ"][k]
        a = -(beta[k + 1] - beta[k]) * E
        lnQ = a.max() + math.log(np.exp(a - a.max()).sum()) - math.log(len(E))
        assert abs(lnQ_oracle - lnQ) <= 1e-12 * max(1.0, abs(lnQ)), (k, lnQ_oracle, lnQ)


# --------------------------------------------------------------------------
# Resampling rule
# --------------------------------------------------------------------------
def test_resampling_copy_numbers_are_floor_or_ceil_of_tau():
    """Import a population, let beta_0 = 0 sweeps (even N_S) leave it
    unchanged, resample to beta_1: every source r gets floor(tau_r) or
    ceil(tau_r) copies, tau_r = R e^{-beta_1 E_r} / sum_j e^{-beta_1 E_j},
    and copies stay in source order."""
    L, N, R = 3, 27, 400
    J = pi.pm_j_couplings(L, 8)
    beta = [0.0, 0.7]
    spins = pi.random_spins(R, N, 5)
    totals = np.zeros(R)
    nseed = 60
    for seed in range(nseed):
        o = oracle.Oracle(L, J, R, beta, 2, 500 + seed)
        o.set_state(0, spins, np.arange(R, dtype=np.uint32), N * math.log(2))
        E = o.energies(spins).astype(np.float64)
        assert o.run(1) == oracle.OK
        st = o.get_state()
        fam = st["family"]
        assert np.all(np.diff(fam.astype(np.int64)) >= 0)
        n = np.bincount(fam, minlength=R)
        w = np.exp(-0.7 * (E - E.min()))
        tau = R * w / w.sum()
        assert np.all((n == np.floor(tau + 1e-9)) | (n == np.ceil(tau - 1e-9))), seed
        # copies are exact replicas of their source
        np.testing.assert_array_equal(st["spins"], spins[fam])
        totals += n
    mean = totals / nseed
    # E[n_r] = tau_r: frac part is a Bernoulli with p = frac(tau)
    frac = tau - np.floor(tau)
    se = np.sqrt(frac * (1 - frac) / nseed) + 1e-12
    z = (mean - tau) / se
    assert np.mean(np.abs(z) < 4) > 0.99


def test_resampling_targets_nominal_population():
    """tau_r = R w_r / sum w with the nominal R (Sec. II.B: the expected new
    population is R(beta')), also when the current R_k differs from R."""
    L, N, R, Rk = 3, 27, 400, 250
    J = pi.pm_j_couplings(L, 9)
    spins = pi.random_spins(Rk, N, 6)
    o = oracle.Oracle(L, J, R, [0.0, 0.4], 2, 11)
    o.set_state(0, spins, np.arange(Rk, dtype=np.uint32), N * math.log(2))
    E = o.energies(spins).astype(np.float64)
    assert o.run(1) == oracle.OK
    n = np.bincount(o.get_state()["family"], minlength=Rk)
    w = np.exp(-0.4 * (E - E.min()))
    tau = R * w / w.sum()
    assert np.all((n == np.floor(tau + 1e-9)) | (n == np.ceil(tau - 1e-9)))
    assert abs(n.sum() - R) < 6 * math.sqrt(R)


def test_population_stays_near_nominal():
    """Normalisation to the nominal R (not R_k): R_k does not random-walk."""
    L = 4
    J = pi.pm_j_couplings(L, 2)
    R = 2000
    o = oracle.Oracle(L, J, R, pi.linear_beta(4.0, 201), 1, 77, threads=8)
    assert o.run() == oracle.OK
    Rk = o.records()["R"]
    # std of R_{k+1} given R is at most sqrt(R)/2; no drift over 200 steps
    assert np.all(np.abs(Rk - R) < 6 * math.sqrt(R))


# --------------------------------------------------------------------------
# Exact invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [3, 4])
def test_beta_zero_leaves_population_unchanged(L):
    N, R = L ** 3, 300
    J = pi.pm_j_couplings(L, 31)
    o = oracle.Oracle(L, J, R, [0.0] * 5, 10, 3)
    st0 = o.get_state()
    assert o.run() == oracle.OK
    st = o.get_state()
    np.testing.assert_array_equal(st["spins"], st0["spins"])
    np.testing.assert_array_equal(st["family"], np.arange(R))
    obs = o.observables()
    assert np.all(obs["R"] == R)
    assert np.all(obs["lnZ"] == N * math.log(2.0))
    assert np.all(obs["S_f"] == math.log(R))


@pytest.mark.parametrize("L", [3, 4])
def test_odd_sweep_count_at_beta_zero_negates_spins(L):
    N, R = L ** 3, 50
    o = oracle.Oracle(L, pi.pm_j_couplings(L, 32), R, [0.0], 3, 3)
    st0 = o.get_state()
    o.run()
    st = o.get_state()
    np.testing.assert_array_equal(st["spins"], -st0["spins"])
    np.testing.assert_array_equal(st["E"], st0["E"])


@pytest.mark.parametrize("L", [3, 4])
def test_incremental_energy_equals_recomputed(L):
    J = pi.pm_j_couplings(L, 41)
    o = oracle.Oracle(L, J, 300, pi.linear_beta(3.0, 21), 10, 6)
    for _ in range(21):
        o.run(1)
        st = o.get_state()
        np.testing.assert_array_equal(st["E"], o.energies(st["spins"]))
        assert np.all(np.diff(st["family"].astype(np.int64)) >= 0)


@pytest.mark.parametrize("L", [3, 4])
def test_gauge_transform_gives_gauge_image_trajectory(L):
    """J_ij -> e_i J_ij e_j with initial state e S_0: every dE and every
    draw is unchanged, so energies, families and observables are identical
    and the spins are the gauge image."""
    N, R = L ** 3, 200
    J = pi.pm_j_couplings(L, 51)
    eps = (2 * np.random.default_rng(4).integers(0, 2, N) - 1).astype(np.int8)
    Jg = pi.gauge_transform(L, J, eps)
    beta = pi.linear_beta(3.0, 15)
    a = oracle.Oracle(L, J, R, beta, 4, 8)
    b = oracle.Oracle(L, Jg, R, beta, 4, 8)
    s0 = a.get_state()
    b.set_state(0, s0["spins"] * eps[None, :], s0["family"], s0["lnZ"])
    assert a.run() == oracle.OK and b.run() == oracle.OK
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sb["spins"], sa["spins"] * eps[None, :])
    np.testing.assert_array_equal(sb["E"], sa["E"])
    np.testing.assert_array_equal(sb["family"], sa["family"])
    oa, ob = a.observables(), b.observables()
    for key in ("R", "mean_E", "C_V", "lnZ", "S_f"):
        np.testing.assert_array_equal(oa[key], ob[key])


def test_global_flip_gives_negated_trajectory():
    L, N, R = 4, 64, 200
    J = pi.pm_j_couplings(L, 52)
    beta = pi.linear_beta(3.0, 12)
    a = oracle.Oracle(L, J, R, beta, 4, 8, overlap_steps=[11])
    b = oracle.Oracle(L, J, R, beta, 4, 8, overlap_steps=[11])
    s0 = a.get_state()
    b.set_state(0, -s0["spins"], s0["family"], s0["lnZ"])
    a.run()
    b.run()
    np.testing.assert_array_equal(b.get_state()["spins"], -a.get_state()["spins"])
    np.testing.assert_array_equal(b.records()["qhist"], a.records()["qhist"])


def test_zero_temperature_quench_never_raises_energy():
    """At beta = 30 every threshold is 0, so the sweeps of a step (applied
    to the same rows step after step) never raise a replica's energy."""
    L, R = 4, 200
    J = pi.pm_j_couplings(L, 61)
    o = oracle.Oracle(L, J, R, [0.0] + [30.0] * 12, 1, 2)
    T, _ = oracle.thresholds(30.0)
    assert list(T) == [0, 0, 0]
    st = o.get_state()
    spins, prev = st["spins"], st["E"]
    for k in range(1, 13):
        spins, E = o.sweep_rows(k, np.arange(R), spins)
        assert np.all(E <= prev)
        np.testing.assert_array_equal(E, o.energies(spins))
        prev = E
    assert np.mean(prev) < np.mean(st["E"]) - 1.0


def test_mattis_instance_reaches_ground_state():
    L = 4
    J, eps = pi.mattis_couplings(L, 3)
    o = oracle.Oracle(L, J, 500, pi.linear_beta(5.0, 51), 10, 4, threads=8)
    assert o.run() == oracle.OK
    E = o.get_state()["E"]
    assert np.mean(E == -3 * L ** 3) > 0.9


# --------------------------------------------------------------------------
# Observables from a crafted population
# --------------------------------------------------------------------------
def test_observables_of_crafted_population():
    L, N, R = 3, 27, 240
    J = pi.pm_j_couplings(L, 71)
    spins = pi.random_spins(R, N, 72)
    # families with known sizes: 1, 2, 3, ... (sorted ids)
    sizes = []
    while sum(sizes) < R:
        sizes.append(min(len(sizes) + 1, R - sum(sizes)))
    fam = np.repeat(np.arange(len(sizes)) * 3, sizes).astype(np.uint32)
    # beta = 0 with an even number of sweeps leaves the imported state as is
    o0 = oracle.Oracle(L, J, R, [0.0, 0.0], 2, 5, overlap_steps=[0])
    o0.set_state(0, spins, fam, 1.25)
    o0.run(1)
    E = o0.energies(spins).astype(np.int64)
    obs = o0.observables()
    rec = o0.records()
    assert rec["sumE"][0] == E.sum() and rec["sumE2"][0] == (E * E).sum()
    assert rec["Emin"][0] == E.min() and rec["Emax"][0] == E.max()
    nu = np.array(sizes) / R
    Sf = -(nu * np.log(nu)).sum()
    assert abs(obs["S_f"][0] - Sf) < 1e-12 * abs(Sf)
    assert abs(obs["rho_s"][0] - R / math.exp(Sf)) < 1e-11 * R
    assert obs["mean_E"][0] == E.sum() / R
    assert obs["C_V"][0] == 0.0  # beta = 0
    # overlap histogram: pair r with r + R/2
    h = R // 2
    Q = (spins[:h].astype(np.int64) * spins[h:2 * h]).sum(axis=1)
    want = np.bincount(Q + N, minlength=2 * N + 1)
    np.testing.assert_array_equal(rec["qhist"][0], want)
    q = Q / N
    assert abs(obs["q2"][0] - (q * q).mean()) < 1e-12
    g = 0.5 * (3 - (q ** 4).mean() / (q * q).mean() ** 2)
    assert abs(obs["g_SG"][0] - g) < 1e-12


def test_specific_heat_of_crafted_population():
    L, N, R = 3, 27, 100
    J = pi.pm_j_couplings(L, 81)
    spins = pi.random_spins(R, N, 82)
    o = oracle.Oracle(L, J, R, [0.0, 0.0], 2, 5)
    o.set_state(0, spins, np.arange(R, dtype=np.uint32), 0.0)
    o.run(1)
    E = o.energies(spins).astype(np.float64)
    # at beta = 0 C_V is 0 by definition; check the variance via records
    rec = o.records()
    var = (rec["sumE2"][0] * R - rec["sumE"][0] ** 2) / R**2
    assert abs(var - E.var()) < 1e-9 * max(1.0, E.var())


@pytest.mark.slow
def test_overlap_matches_exact_distribution_L2():
    """From beta = 0, one resampling to beta, then chains at fixed beta:
    pairs (r, r + R/2) lie in different families and are independent
    Boltzmann samples, so Q follows the exact P(Q)."""
    L, N, R, beta = 2, 8, 16000, 0.6
    J = pi.pm_j_couplings(L, 91)
    nT = 20
    o = oracle.Oracle(L, J, R, [0.0] + [beta] * (nT - 1), 10, 3, overlap_steps=[nT - 1], threads=8)
    assert o.run() == oracle.OK
    counts = o.records()["qhist"][nT - 1].astype(float)
    P = oracle.overlap_distribution(L, J, beta)
    G, dof = _gtest(counts, P)
    assert G < dof + 10 * math.sqrt(2 * dof) + 20, (G, dof)


def test_overlap_at_beta_zero_has_mean_q2_one_over_N():
    L, N, R = 4, 64, 20000
    o = oracle.Oracle(L, pi.pm_j_couplings(L, 92), R, [0.0], 2, 4, threads=8)
    o.run()
    q2 = o.observables()["q2"][0]
    # q^2 of two independent random configurations: mean 1/N, var ~ 2/N^2
    assert abs(q2 - 1 / N) < 5 * math.sqrt(2.0 / (R / 2)) / N


# --------------------------------------------------------------------------
# Annealing schedules and the population schedule (Sec. III.B, Eqs. (5)-(6))
# --------------------------------------------------------------------------
def test_lblt_schedule_is_linear_in_beta_then_in_T():
    b = pi.lblt_beta(5.0, 201, T_N=1.0)
    kN = 100
    assert b[0] == 0.0 and b[-1] == pytest.approx(5.0, rel=1e-15) and b[kN] == pytest.approx(1.0, rel=1e-15)
    assert np.allclose(np.diff(b[: kN + 1]), 1.0 / kN, rtol=1e-12)
    T = 1.0 / b[kN:]
    assert np.allclose(np.diff(T), (0.2 - 1.0) / 100, rtol=1e-9)
    assert np.all(np.diff(b) > 0)


def test_tspl_schedule_endpoints_and_switch_over():
    a1, a2, b0, bmax, nT = np.exp(-0.0734), np.exp(2.15), 1.63, 5.0, 301
    b = pi.tspl_beta(bmax, nT)
    assert b[0] == 0.0 and b[-1] == pytest.approx(bmax, rel=1e-15)
    assert np.all(np.diff(b) > 0)
    tau0 = (b0 / bmax) ** (1 / a2)
    # both branches give beta0 at tau0 (continuity), each is its power law
    a = b0 / tau0 ** a1
    tau = np.arange(nT) / (nT - 1)
    lo = tau < tau0
    assert np.allclose(b[lo], a * tau[lo] ** a1, rtol=1e-14)
    assert np.allclose(b[~lo], bmax * tau[~lo] ** a2, rtol=1e-14)
    assert a * tau0 ** a1 == pytest.approx(b0, rel=1e-14) and bmax * tau0 ** a2 == pytest.approx(b0, rel=1e-14)


def test_clipped_exponential_population():
    beta = pi.linear_beta(5.0, 201)
    R = pi.clipped_exponential_population(beta, 10000)
    R0 = R[0]
    assert np.all(R[beta <= 0.9] == R0)
    assert np.all(np.diff(R) <= 0)
    assert R[-1] == pytest.approx(R0 / 33.8, abs=1.0)
    assert R.mean() == pytest.approx(10000, rel=1e-3)


def test_resampling_targets_the_scheduled_population():
    """With a population schedule the resampling to beta_{k+1} targets
    R(beta_{k+1}): tau_r = R(beta') w_r / sum w."""
    L, N, R, R1 = 3, 27, 400, 250
    J = pi.pm_j_couplings(L, 9)
    spins = pi.random_spins(R, N, 6)
    o = oracle.Oracle(L, J, R, [0.0, 0.4], 2, 11, pop_schedule=[R, R1])
    o.set_state(0, spins, np.arange(R, dtype=np.uint32), N * math.log(2))
    E = o.energies(spins).astype(np.float64)  # beta_0 = 0: the sweeps flip every spin twice
    assert o.run(1) == oracle.OK
    n = np.bincount(o.get_state()["family"], minlength=R)
    w = np.exp(-0.4 * (E - E.min()))
    tau = R1 * w / w.sum()
    assert np.all((n == np.floor(tau + 1e-9)) | (n == np.ceil(tau - 1e-9)))
    assert abs(n.sum() - R1) < 6 * math.sqrt(R1)


def test_population_follows_its_schedule():
    L = 4
    J = pi.pm_j_couplings(L, 2)
    beta = pi.linear_beta(4.0, 101)
    pop = pi.clipped_exponential_population(beta, 2000)
    o = oracle.Oracle(L, J, int(pop[0]), beta, 1, 78, threads=8, pop_schedule=pop)
    assert o.run() == oracle.OK
    Rk = o.records()["R"]
    assert np.all(np.abs(Rk - pop) < 6 * np.sqrt(pop) + 1)
