"""Pins of the oracle on the square lattice (D = 2, Sec. II.A: N = L^2 spins,
four neighbours) against facts it does not compute itself: a proper
colouring checked bond by bond, every configuration's energy enumerated here
from Eq. (1), the exact Boltzmann law and thermodynamics of tiny instances,
closed forms at beta = 0 and at the ferromagnet's ground state, and the
cluster-move island as a connected component found by a search written here.
A 3D neighbour or bond left in the 2D path, a wrong colour or a wrong energy
offset fails at least one of them."""
import math

import numpy as np
import pytest

import oracle
import pamc_inputs as pi

SCALE = 2.0 ** -20
TAG_ICM = 0x40000000


def _all_energies(L, J):
    """Energy (units of 2^-20) of every configuration, bit s of the index
    being spin s up."""
    N = L * L
    codes = np.arange(2 ** N, dtype=np.int64)
    S = np.where((codes[:, None] >> np.arange(N)[None, :]) & 1, 1, -1).astype(np.int64)
    nb = pi.square_neighbours(L)
    E = np.zeros(2 ** N, dtype=np.int64)
    for d in range(2):
        E -= (S * S[:, nb[d]] * J[d].astype(np.int64)[None, :]).sum(axis=1)
    return E


def _codes(spins):
    N = spins.shape[1]
    return ((spins > 0).astype(np.int64) << np.arange(N)[None, :]).sum(axis=1)


def _gtest_pooled(counts, p, min_expected=5.0):
    n = counts.sum()
    e = p * n
    big = e >= min_expected
    c = np.append(counts[big], counts[~big].sum())
    ee = np.append(e[big], e[~big].sum())
    keep = ee > 0
    c, ee = c[keep], ee[keep]
    m = c > 0
    return 2.0 * np.sum(c[m] * np.log(c[m] / ee[m])), len(c) - 1


@pytest.mark.parametrize("L", [2, 3, 4, 5, 7, 8, 9])
def test_colouring_is_proper_and_ranked(L):
    J = pi.gaussian_couplings(L, 1, dim=2)
    o = oracle.Oracle(L, J, 4, [0.0], 1, 1)
    ncol, c, r = o.colouring()
    assert ncol == (2 if L % 2 == 0 else 3)
    for nb in pi.square_neighbours(L):
        assert np.all(c != c[nb])
    for col in range(ncol):
        sites = np.nonzero(c == col)[0]
        np.testing.assert_array_equal(r[sites], np.arange(len(sites)))


@pytest.mark.parametrize("L", [3, 4])
def test_energies_equal_enumeration(L):
    J = pi.gaussian_couplings(L, 11 + L, dim=2)
    E_all = _all_energies(L, J)
    o = oracle.Oracle(L, J, 4, [0.0], 1, 1)
    N = L * L
    rng = np.random.default_rng(L)
    codes = rng.integers(0, 2 ** N, size=500)
    spins = np.where((codes[:, None] >> np.arange(N)[None, :]) & 1, 1, -1).astype(np.int8)
    np.testing.assert_array_equal(o.energies(spins), E_all[codes])


@pytest.mark.parametrize("beta,icm", [(0.5, 0), (1.3, 0), (1.0, 2)])
def test_fixed_beta_population_is_boltzmann(beta, icm):
    """From beta = 0, one resampling to beta, then constant beta: later
    resamplings weight every replica equally, and the sweeps (and the pair
    updates, which keep the product of the pair's Boltzmann weights) leave
    the exact law over all 2^9 configurations invariant."""
    L, N, R = 3, 9, 8000
    J = pi.gaussian_couplings(L, 40, dim=2)
    o = oracle.Oracle(L, J, R, [0.0] + [beta] * 24, 6, 3 + icm, threads=8, icm_rounds=icm)
    assert o.run() == oracle.OK
    E_all = _all_energies(L, J).astype(np.float64) * SCALE
    w = np.exp(-beta * (E_all - E_all.min()))
    counts = np.bincount(_codes(o.get_state()["spins"]), minlength=2 ** N).astype(np.float64)
    G, dof = _gtest_pooled(counts, w / w.sum())
    assert G < dof + 10 * math.sqrt(2 * dof) + 20, (G, dof)
    # not vacuous: the law at -beta is rejected
    q = np.exp(beta * (E_all - E_all.max()))
    G2, dof2 = _gtest_pooled(counts, q / q.sum())
    assert G2 > dof2 + 10 * math.sqrt(2 * dof2) + 20


def test_annealing_matches_exact_thermodynamics():
    L, N = 4, 16
    J = pi.gaussian_couplings(L, 77, dim=2)
    E = _all_energies(L, J).astype(np.float64) * SCALE
    beta = pi.linear_beta(2.5, 26)
    ex = {"lnZ": [], "mean_E": [], "C_V": []}
    for b in beta:
        a = -b * E
        w = np.exp(a - a.max())
        Z = w.sum()
        m1, m2 = (w * E).sum() / Z, (w * E * E).sum() / Z
        ex["lnZ"].append(a.max() + math.log(Z))
        ex["mean_E"].append(m1)
        ex["C_V"].append(b * b * (m2 - m1 * m1) / N)
    runs = []
    for seed in range(8):
        o = oracle.Oracle(L, J, 3000, beta, 10, 500 + seed, threads=8)
        assert o.run() == oracle.OK
        runs.append(o.observables())
    for key in ("lnZ", "mean_E", "C_V"):
        vals = np.array([r[key] for r in runs])
        mean, se = vals.mean(axis=0), vals.std(axis=0, ddof=1) / math.sqrt(len(runs))
        for k in (5, 12, 25):
            tol = 5 * se[k] + 1e-3 * abs(ex[key][k]) + 1e-9
            assert abs(mean[k] - ex[key][k]) < tol, (key, k, mean[k], ex[key][k], se[k])
    assert runs[0]["lnZ"][0] == N * math.log(2.0)


def test_beta_zero_closed_forms():
    """Random configurations: <E> = 0 and <E^2> = sum_b J_b^2 over the 2N
    bonds (each bond product is an independent sign)."""
    L, R = 8, 20000
    J = pi.gaussian_couplings(L, 5, dim=2)
    o = oracle.Oracle(L, J, R, [0.0], 1, 8, threads=8)
    assert o.run() == oracle.OK
    rec = o.records()
    var = float(((J.astype(np.float64) * SCALE) ** 2).sum())
    mean = rec["sumE"][0] * SCALE / R
    second = float(rec["sumE2"][0]) * SCALE * SCALE / R
    assert abs(mean) < 5 * math.sqrt(var / R)
    assert abs(second - var) < 5 * var * math.sqrt(2.0 / R)


def test_ferromagnet_reaches_its_ground_state():
    """All couplings +1: the two uniform states have E = -2N, and the gap to
    the next level is 8 (one flipped spin breaks four bonds)."""
    L = 6
    N = L * L
    J = pi.pm_couplings_as_real(np.ones((2, N), dtype=np.int8))
    o = oracle.Oracle(L, J, 400, pi.linear_beta(5.0, 61), 10, 12)
    assert o.run() == oracle.OK
    st = o.get_state()
    assert np.all(st["E"] == -2 * N * 2 ** 20)
    assert np.all(np.abs(st["spins"].sum(axis=1)) == N)


def _island(L, a, b, j, k, rd, seed):
    """The island of one pair update by a breadth-first search over the four
    square-lattice bonds, seeded as the update states."""
    N = L * L
    differ = a != b
    nd = int(differ.sum())
    members = differ if nd <= N - nd else ~differ
    cnt = int(members.sum())
    if cnt == 0:
        return set()
    u = int(oracle.philox4x32_10([j, 4, k, TAG_ICM | rd], [seed & 0xFFFFFFFF, seed >> 32])[0])
    s0 = int(np.nonzero(members)[0][(u * cnt) >> 32])
    x, y = np.arange(N) % L, np.arange(N) // L
    nbs = [((x + 1) % L) + L * y, ((x - 1) % L) + L * y, x + L * ((y + 1) % L), x + L * ((y - 1) % L)]
    seen, todo = {s0}, [s0]
    while todo:
        s = todo.pop()
        for nb in nbs:
            t = int(nb[s])
            if members[t] and t not in seen:
                seen.add(t)
                todo.append(t)
    return seen


@pytest.mark.parametrize("L", [4, 5, 8])
def test_cluster_move_flips_a_square_lattice_island(L):
    J = pi.gaussian_couplings(L, 9, dim=2)
    seed = 31
    o = oracle.Oracle(L, J, 4, [0.0], 1, seed)
    rng = np.random.default_rng(L)
    N = L * L
    sizes = []
    for trial in range(40):
        a = (2 * rng.integers(0, 2, N) - 1).astype(np.int8)
        keep = rng.random(N) < rng.uniform(0.0, 1.0)
        b = np.where(keep, a, 2 * rng.integers(0, 2, N) - 1).astype(np.int8)
        j, k, rd = trial, 3 + trial, trial % 2
        a2, b2, size = o.icm_pair(a, b, j, k, rd)
        island = _island(L, a, b, j, k, rd, seed)
        assert size == len(island)
        assert set(np.nonzero(a2 != a)[0].tolist()) == island
        assert set(np.nonzero(b2 != b)[0].tolist()) == island
        Ea, Eb = o.energies(np.stack([a, b]))
        Ea2, Eb2 = o.energies(np.stack([a2, b2]))
        assert int(Ea) + int(Eb) == int(Ea2) + int(Eb2)
        sizes.append(size)
    assert max(sizes) > 1


def test_invalid_2d_arguments_are_rejected():
    J8 = np.ones((2, 16), dtype=np.int8)
    with pytest.raises(ValueError):
        oracle.Oracle(4, J8, 10, [0.0], 1, 1)  # +-J in 2D: pass it as real couplings
    with pytest.raises(ValueError):
        oracle.Oracle(65, pi.gaussian_couplings(65, 1, dim=2), 10, [0.0], 1, 1)
    oracle.Oracle(64, pi.gaussian_couplings(64, 1, dim=2), 10, [0.0], 1, 1).close()
