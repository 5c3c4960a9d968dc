"""Degenerate and extreme cases against the oracle, bit for bit (through
the C ABI, on the GPU): a single replica, a single temperature, a single
sweep, no change of temperature, and the largest lattices of each sweep
kernel (L = 19 runs the largest three-colour table form, 615 threads and
about 140 KB of LDS; L = 20 and 21 the largest register-form colour-major
workgroups, 1024 and 896 threads; L = 23 and 32 the per-site kernel)."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state

pytestmark = pytest.mark.gpu


def both(L, R, beta, NS, dseed, seed, **kw):
    from paper_1710_09025_amd import Pamc

    J = pi.pm_j_couplings(L, dseed)
    p = Pamc(L, J, R, beta, NS, seed, **kw)
    st = p.anneal()
    o = oracle.Oracle(L, J, R, beta, NS, seed, threads=THREADS)
    sto = o.run()
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"L={L} R={R}")
    compare_run(p.observables(), p.step_sums(), o, what=f"L={L} R={R}")
    return p, o


@pytest.mark.parametrize("L", [4, 5, 8])
def test_single_replica(L):
    p, o = both(L, 1, pi.linear_beta(4.0, 11), 3, 230 + L, 240 + L)
    assert np.all(p.observables()["R"] == 1)
    assert np.all(p.step_sums()[1][:] == 0.0)  # one family of size 1: n ln n = 0


@pytest.mark.parametrize("L", [3, 8])
def test_single_temperature(L):
    both(L, 50, np.array([0.0]), 3, 250 + L, 260 + L)


def test_first_temperature_above_zero_is_rejected():
    """The random initial population is the beta = 0 sample and ln Z is
    anchored there (Sec. II.B): a schedule that starts elsewhere is refused
    by the library (create, batch and server) and by the oracle alike."""
    from paper_1710_09025_amd import Pamc, PamcBatch, PamcError, PamcServer, _capi

    J = pi.pm_j_couplings(6, 270)
    for beta in (np.array([1.3]), np.array([0.2, 0.4, 0.6])):
        with pytest.raises(PamcError) as e:
            Pamc(6, J, 40, beta, 2, 271)
        assert e.value.status == _capi.ERR_INVALID
        with pytest.raises(PamcError) as e:
            PamcBatch([dict(L=6, couplings=J, R=40, beta=pi.linear_beta(1.0, 3), sweeps=2, seed=1),
                       dict(L=6, couplings=J, R=40, beta=beta, sweeps=2, seed=2)])
        assert e.value.status == _capi.ERR_INVALID
        with pytest.raises(ValueError):
            oracle.Oracle(6, J, 40, beta, 2, 271)
    srv = PamcServer(1 << 30)
    try:
        with pytest.raises(PamcError) as e:
            srv.submit(6, J, 40, np.array([0.5, 1.0]), 2, 3)
        assert e.value.status == _capi.ERR_INVALID
    finally:
        srv.close()


@pytest.mark.parametrize("L", [4, 7, 16])
def test_single_sweep_per_step(L):
    both(L, 120, pi.linear_beta(5.0, 15), 1, 280 + L, 290 + L)


def test_constant_beta_keeps_every_replica():
    """d beta = 0: w = 1 for every level, tau = R / R_k = 1 exactly, so every
    replica has exactly one copy and the families never change."""
    p, o = both(6, 300, np.zeros(9), 2, 300, 301)
    st = p.get_state()
    np.testing.assert_array_equal(st["family"], np.arange(300))
    assert np.all(p.observables()["R"] == 300)


def test_constant_beta_after_the_start():
    """beta = 0 then a constant 0.7: after the first resampling every weight
    is 1 and tau = R / R_k, so the copies no longer depend on the state."""
    both(6, 300, np.array([0.0] + [0.7] * 8), 2, 300, 301)


@pytest.mark.parametrize("L,R", [(19, 3), (20, 3), (21, 3), (23, 3), (32, 2)])
def test_largest_lattices(L, R):
    both(L, R, pi.linear_beta(3.0, 3), 1, 310 + L, 320 + L)
