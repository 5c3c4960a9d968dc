"""The allocation-free entry point (pamc_anneal_static) against the entry
points that allocate (pamc_create + pamc_anneal), through the C ABI on the
GPU: two calls in a row, the second smaller, each equal to its allocating
run in every observable and in the final population; the second also
against the oracle."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state, same_obs

pytestmark = pytest.mark.gpu


def allocating_run(L, J, R, beta, NS, seed):
    from paper_1710_09025_amd import Pamc

    p = Pamc(L, J, R, beta, NS, seed)
    st = p.anneal()
    return p, st


@pytest.mark.parametrize("first,second", [((8, 20000, 31, 5, 41), (5, 3000, 21, 4, 43))])
def test_static_entry_equals_allocating_entry_twice(first, second):
    from paper_1710_09025_amd import anneal_static, make_pm_j

    for i, (L, R, nT, NS, seed) in enumerate((first, second)):
        J = make_pm_j(L, 100 + L)
        beta = pi.linear_beta(5.0, nT)
        st, obs, state = anneal_static(L, J, R, beta, NS, seed)
        p, st_ref = allocating_run(L, J, R, beta, NS, seed)
        assert st == st_ref == 0
        what = f"call {i + 1} (L={L}, R={R})"
        same_obs(obs, p.observables(), what)
        ref = p.get_state()
        assert state["step"] == ref["step"] == nT
        compare_state(state, ref, what)
        assert state["lnZ"] == ref["lnZ"]
        p.close()
    # the second, smaller call also against the oracle
    L, R, nT, NS, seed = second
    J = make_pm_j(L, 100 + L)
    beta = pi.linear_beta(5.0, nT)
    o = oracle.Oracle(L, J, R, beta, NS, seed, threads=THREADS)
    assert o.run() == 0
    st, obs, state = anneal_static(L, J, R, beta, NS, seed)
    compare_state(state, o.get_state(), "second call vs oracle")
    for g, r in (("R", "R"), ("sum_E", "sumE"), ("sum_E2", "sumE2"), ("E_min", "Emin"), ("E_max", "Emax")):
        assert list(obs[g]) == list(o.records()[r]), g


def test_static_entry_reports_failures_like_the_allocating_entry():
    """An oversize run is refused before any device work; a run after it
    equals the allocating run."""
    from paper_1710_09025_amd import PamcError, _capi, anneal_static

    J = pi.pm_j_couplings(16, 3)
    with pytest.raises(PamcError) as e:
        anneal_static(16, J, 100000, pi.linear_beta(5.0, 11), 2, 1)
    assert e.value.status == _capi.ERR_INVALID
    L, R, nT = 4, 700, 41
    J = pi.pm_j_couplings(L, 9)
    beta = pi.linear_beta(5.0, nT)
    st, obs, state = anneal_static(L, J, R, beta, 3, 17)
    p, st_ref = allocating_run(L, J, R, beta, 3, 17)
    assert st == st_ref == 0
    same_obs(obs, p.observables(), "small run")
    compare_state(state, p.get_state(), "small run")
