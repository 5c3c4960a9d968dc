"""Pins of the oracle's isoenergetic cluster moves (ICM, Sec. IV) against
facts it does not compute itself: bijectivity of the pairing permutation,
conservation of the pair's summed energy, the island as an independently
computed connected component of the smaller overlap sector, and the exact
Boltzmann law of a fixed-temperature population updated with ICM."""
import math

import numpy as np
import pytest

import oracle
import pamc_inputs as pi

TAG_ICM = 0x40000000


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 1000, 4097, 20011])
def test_pairing_permutation_is_a_bijection(n):
    for k, rd in [(1, 0), (1, 1), (57, 0)]:
        p = [oracle.icm_perm(12345, i, n, k, rd) for i in range(n)]
        assert sorted(p) == list(range(n)), (n, k, rd)
    if n >= 64:
        a = [oracle.icm_perm(12345, i, n, 1, 0) for i in range(n)]
        b = [oracle.icm_perm(12345, i, n, 1, 1) for i in range(n)]
        c = [oracle.icm_perm(12346, i, n, 1, 0) for i in range(n)]
        assert a != b and a != c and a != list(range(n))


def _neighbours(L):
    N = L ** 3
    idx = np.arange(N)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    return [((x + dx) % L) + L * (((y + dy) % L) + L * ((z + dz) % L))
            for dx, dy, dz in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]]


def _expected_island(L, a, b, j, k, rd, seed):
    """The island by a plain BFS written here, seeded as the update states."""
    N = L ** 3
    differ = a != b
    nd = int(differ.sum())
    want = nd <= N - nd
    members = differ if want else ~differ
    cnt = int(members.sum())
    if cnt == 0:
        return set()
    u = int(oracle.philox4x32_10([j, 4, k, TAG_ICM | rd], [seed & 0xFFFFFFFF, seed >> 32])[0])
    m = (u * cnt) >> 32
    s0 = int(np.nonzero(members)[0][m])
    nb = _neighbours(L)
    seen, todo = {s0}, [s0]
    while todo:
        s = todo.pop()
        for d in range(6):
            t = int(nb[d][s])
            if members[t] and t not in seen:
                seen.add(t)
                todo.append(t)
    return seen


@pytest.mark.parametrize("L,coupling", [(4, "pm"), (5, "real"), (6, "pm")])
def test_update_flips_one_island_and_conserves_the_pair_energy(L, coupling):
    J = pi.pm_j_couplings(L, 3) if coupling == "pm" else pi.gaussian_couplings(L, 3)
    seed = 77
    o = oracle.Oracle(L, J, 4, [0.0], 1, seed)
    rng = np.random.default_rng(L)
    N = L ** 3
    sizes = []
    for trial in range(40):
        a = (2 * rng.integers(0, 2, N) - 1).astype(np.int8)
        # partly correlated partners: overlaps away from zero, islands of many sizes
        keep = rng.random(N) < rng.uniform(0.0, 1.0)
        b = np.where(keep, a, (2 * rng.integers(0, 2, N) - 1)).astype(np.int8)
        j, k, rd = trial, 5 + trial, trial % 2
        a2, b2, size = o.icm_pair(a, b, j, k, rd)
        island = _expected_island(L, a, b, j, k, rd, seed)
        assert size == len(island)
        flipped = set(np.nonzero(a2 != a)[0].tolist())
        assert flipped == island
        assert set(np.nonzero(b2 != b)[0].tolist()) == island
        Ea, Eb = o.energies(np.stack([a, b]))
        Ea2, Eb2 = o.energies(np.stack([a2, b2]))
        assert int(Ea) + int(Eb) == int(Ea2) + int(Eb2)
        sizes.append(size)
    assert max(sizes) > 1 and min(sizes) >= 0


def test_identical_and_tied_pairs():
    L, N = 4, 64
    J = pi.pm_j_couplings(L, 1)
    o = oracle.Oracle(L, J, 4, [0.0], 1, 5)
    a = np.ones(N, dtype=np.int8)
    # identical replicas: the differing sector is empty and smaller: no move
    a2, b2, size = o.icm_pair(a, a, 0, 1, 0)
    assert size == 0 and np.array_equal(a2, a) and np.array_equal(b2, a)
    # exactly half the sites differ: the differing sector is taken
    b = a.copy()
    b[:32] = -1
    a2, b2, size = o.icm_pair(a, b, 3, 2, 1)
    assert size > 0
    changed = np.nonzero(a2 != a)[0]
    assert len(changed) == size and np.all(changed < 32)
    np.testing.assert_array_equal(np.nonzero(b2 != b)[0], changed)


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


@pytest.mark.parametrize("beta,real", [(0.5, False), (1.0, True)])
def test_fixed_beta_population_with_icm_is_boltzmann(beta, real):
    """Constant beta (after the start at beta = 0) with ICM at every step:
    the pair updates keep the product of Boltzmann laws invariant, so the
    population still follows the exact Boltzmann law over all 2^N
    configurations."""
    L, N, R = 2, 8, 6000
    J = pi.gaussian_couplings(L, 9) if real else pi.pm_j_couplings(L, 9)
    o = oracle.Oracle(L, J, R, [0.0] + [beta] * 24, 4, 3, threads=8, icm_rounds=2)
    assert o.run() == oracle.OK
    st = o.get_state()
    E_all = (oracle.all_energies_real(L, J).astype(np.float64) * 2.0 ** -20 if real
             else oracle.all_energies(L, J).astype(np.float64))
    w = np.exp(-beta * (E_all - E_all.min()))
    p = w / w.sum()
    code = ((st["spins"] > 0).astype(np.int64) << np.arange(N)[None, :]).sum(axis=1)
    counts = np.bincount(code, minlength=2 ** N).astype(np.float64)
    G, dof = _gtest_pooled(counts, p)
    assert G < dof + 10 * math.sqrt(2 * dof) + 20, (G, dof)


def test_icm_changes_the_trajectory_and_keeps_energies_consistent():
    L = 4
    J = pi.pm_j_couplings(L, 21)
    beta = pi.linear_beta(3.0, 9)
    a = oracle.Oracle(L, J, 300, beta, 4, 8)
    b = oracle.Oracle(L, J, 300, beta, 4, 8, icm_rounds=2)
    for k in range(len(beta)):
        assert a.run(1) == 0 and b.run(1) == 0
        sb = b.get_state()
        np.testing.assert_array_equal(sb["E"], b.energies(sb["spins"]))
    # step 0 has no ICM: identical after it; later steps differ
    assert not np.array_equal(a.get_state()["spins"], b.get_state()["spins"])


def test_planted_wrong_island_choice_breaks_boltzmann():
    """The fixed-beta check is not vacuous: flipping an island in only one
    replica (not energy conserving) is rejected by the same statistic."""
    L, N = 2, 8
    J = pi.pm_j_couplings(L, 9)
    E_all = oracle.all_energies(L, J).astype(np.float64)
    beta = 0.5
    w = np.exp(-beta * (E_all - E_all.min()))
    p = w / w.sum()
    rng = np.random.default_rng(1)
    # a population drawn from the law at beta, then one-sided island flips
    codes = rng.choice(2 ** N, size=6000, p=p)
    flip = rng.integers(1, 2 ** N, size=6000)
    bad = codes ^ (flip * (rng.random(6000) < 0.5))
    counts = np.bincount(bad, minlength=2 ** N).astype(np.float64)
    G, dof = _gtest_pooled(counts, p)
    assert G > dof + 10 * math.sqrt(2 * dof) + 20


def test_temperature_window():
    """icm_beta_min above every beta gives the run without cluster moves;
    a window starting mid-anneal agrees with it up to the window's start."""
    L = 4
    J = pi.pm_j_couplings(L, 23)
    beta = pi.linear_beta(3.0, 13)
    plain = oracle.Oracle(L, J, 200, beta, 4, 9)
    none = oracle.Oracle(L, J, 200, beta, 4, 9, icm_rounds=2, icm_beta_min=10.0)
    late = oracle.Oracle(L, J, 200, beta, 4, 9, icm_rounds=2, icm_beta_min=1.5)
    k_start = int(np.argmax(beta >= 1.5))
    for k in range(len(beta)):
        for o in (plain, none, late):
            assert o.run(1) == 0
        sp = plain.get_state()["spins"]
        np.testing.assert_array_equal(none.get_state()["spins"], sp)
        if k < k_start:
            np.testing.assert_array_equal(late.get_state()["spins"], sp)
    assert not np.array_equal(late.get_state()["spins"], plain.get_state()["spins"])
