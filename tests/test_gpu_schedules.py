"""The paper's annealing schedules (LBLT, TSPL, Sec. III.B, Eq. (5)) and the
clipped exponential population schedule (Sec. III.D, Eq. (6)) on the GPU,
against the oracle through the C ABI."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state

pytestmark = pytest.mark.gpu


def gpu(L, J, R, beta, NS, seed, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(L, J, R, beta, NS, seed, **kw)
    assert p.anneal() == 0
    return p


def orc(L, J, R, beta, NS, seed, pop=None):
    o = oracle.Oracle(L, J, R, beta, NS, seed, threads=THREADS, pop_schedule=pop)
    assert o.run() == oracle.OK
    return o


@pytest.mark.parametrize("schedule", ["lblt", "tspl"])
@pytest.mark.parametrize("L", [5, 8])
def test_schedules_match_oracle(schedule, L):
    beta = pi.lblt_beta(5.0, 41) if schedule == "lblt" else pi.tspl_beta(5.0, 41)
    J = pi.pm_j_couplings(L, 160 + L)
    p = gpu(L, J, 600, beta, 4, 170 + L)
    o = orc(L, J, 600, beta, 4, 170 + L)
    compare_state(p.get_state(), o.get_state(), f"{schedule} L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"{schedule} L={L}")


@pytest.mark.parametrize("L,packed", [(4, False), (6, True), (8, False), (16, False)])
def test_population_schedule_matches_oracle(L, packed):
    beta = pi.tspl_beta(5.0, 31)
    pop = pi.clipped_exponential_population(beta, {4: 1500, 6: 800, 8: 700, 16: 60}[L])
    J = pi.pm_j_couplings(L, 180 + L)
    R = int(pop[0])
    p = gpu(L, J, R, beta, 3, 190 + L, pop_schedule=pop, packed=packed)
    o = orc(L, J, R, beta, 3, 190 + L, pop=pop)
    compare_state(p.get_state(), o.get_state(), f"population schedule L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"population schedule L={L}")
    R_k = p.observables()["R"]
    assert np.all(np.abs(R_k - pop) < 6 * np.sqrt(pop) + 1)


def test_scheduled_batch_equals_separate_runs():
    from paper_1710_09025_amd import PamcBatch

    insts = []
    for i, L in enumerate([4, 8, 5]):
        beta = pi.lblt_beta(5.0, 21) if i % 2 else pi.tspl_beta(5.0, 21)
        pop = pi.clipped_exponential_population(beta, 400 + 100 * i)
        insts.append(dict(L=L, couplings=pi.pm_j_couplings(L, 200 + i), R=int(pop[0]), beta=beta, sweeps=3,
                          seed=210 + i, pop_schedule=pop))
    b = PamcBatch(insts)
    assert b.anneal() == 0
    for i, d in enumerate(insts):
        p = gpu(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"], pop_schedule=d["pop_schedule"])
        compare_state(b.get_state(i), p.get_state(), f"scheduled batch {i}")


def test_rho_f_from_independent_runs_matches_oracle_runs():
    """rho_f = R var(beta F) over independent seeds (Eq. (4)): beta F of every
    run equals the oracle's run with the same seed; at beta = 0 every run has
    beta F = -N ln 2 exactly, so the variance vanishes."""
    from paper_1710_09025_amd import free_energy_variance

    L, R, NS = 4, 800, 4
    beta = pi.linear_beta(4.0, 21)
    J = pi.pm_j_couplings(L, 220)
    seeds = list(range(300, 312))
    res = free_energy_variance(L, J, R, beta, NS, seeds)
    ref = np.stack([orc(L, J, R, beta, NS, s).observables()["betaF"] for s in seeds])
    np.testing.assert_allclose(res["betaF"], ref, rtol=1e-12, atol=0)
    assert res["var_betaF"][0] == 0.0
    # the library's Eq. (4) on the GPU runs' own beta F: the same sample
    # variance as numpy's, to rounding
    np.testing.assert_allclose(res["rho_f"], R * res["betaF"].var(axis=0, ddof=1), rtol=1e-11, atol=1e-12)
    # against the oracle runs: beta F agrees to 1e-12 relative, i.e. to
    # about 1e-12 |beta F| ~ 1e-10 absolute, while the spread between runs
    # is ~1e-3 to 1e-1, so the variance (a difference of nearly equal
    # numbers) can only agree to about 1e-10 / 1e-4 relative
    np.testing.assert_allclose(res["rho_f"], R * ref.var(axis=0, ddof=1), rtol=1e-6, atol=1e-12)
    assert np.all(res["rho_f"][1:] > 0)
