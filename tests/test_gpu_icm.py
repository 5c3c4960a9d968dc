"""Isoenergetic cluster moves (Sec. IV) on the GPU against the CPU oracle,
through the C ABI: spins, energies, families, population sizes and the
per-step sums bit-exact, derived observables within 1e-12."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state, rel_close

pytestmark = pytest.mark.gpu


def make(L, R, nT, NS, bmax, dseed, seed, real=False):
    J = pi.gaussian_couplings(L, dseed) if real else pi.pm_j_couplings(L, dseed)
    return dict(L=L, couplings=J, R=R, beta=pi.linear_beta(bmax, nT), sweeps=NS, seed=seed)


def both(inst, rounds=2, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=rounds,
             **kw)
    st = p.anneal()
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, icm_rounds=rounds)
    sto = o.run()
    return p, st, o, sto


# every sweep kernel: colour-major with two and three colours, even/odd-x
# (L = 8, 16), per-site (L = 24, 32), real couplings; odd and even N_S, odd R;
# the island search as a queue (L < 8) and as a row flood fill (L >= 8)
CASES = [
    (3, 401, 11, 10, 4.0, False),
    (4, 1000, 21, 10, 4.0, False),
    (5, 333, 11, 5, 4.0, False),
    (8, 1001, 15, 10, 4.0, False),
    (10, 121, 7, 4, 4.0, False),
    (16, 63, 5, 3, 4.0, False),
    (24, 9, 3, 2, 3.0, False),
    (6, 500, 11, 6, 4.0, True),
    (7, 151, 9, 5, 4.0, True),
    # the row flood fill from L = 8 on: rows of a length that is not a
    # multiple of four (9), 32-lane groups (12), whole-word rows with 64-lane
    # groups (32), real couplings
    (9, 201, 7, 4, 4.0, False),
    (12, 64, 5, 3, 4.0, False),
    (32, 4, 3, 2, 3.0, False),
    (8, 300, 7, 4, 4.0, True),
]


@pytest.mark.parametrize("L,R,nT,NS,bmax,real", CASES)
def test_full_run_with_cluster_moves_bit_exact(L, R, nT, NS, bmax, real):
    inst = make(L, R, nT, NS, bmax, 800 + L, 900 + L, real)
    p, st, o, sto = both(inst)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"icm L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"icm L={L}")


@pytest.mark.parametrize("bmin", [1.7, 10.0])
def test_temperature_window_bit_exact(bmin):
    from paper_1710_09025_amd import Pamc

    inst = make(6, 400, 13, 4, 4.0, 33, 34)
    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2,
             icm_beta_min=bmin)
    assert p.anneal() == 0
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, icm_rounds=2, icm_beta_min=bmin)
    assert o.run() == 0
    compare_state(p.get_state(), o.get_state(), f"icm window {bmin}")
    compare_run(p.observables(), p.step_sums(), o, what=f"icm window {bmin}")


def test_one_round_and_eight_rounds():
    for rounds in (1, 8):
        inst = make(4, 300, 9, 4, 4.0, 31, 32)
        p, st, o, sto = both(inst, rounds=rounds)
        assert st == sto == 0
        compare_state(p.get_state(), o.get_state(), f"icm rounds={rounds}")


def test_cluster_moves_change_the_run():
    from paper_1710_09025_amd import Pamc

    inst = make(6, 600, 11, 6, 4.0, 41, 42)
    a = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    b = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2)
    assert a.anneal() == 0 and b.anneal() == 0
    assert not np.array_equal(a.get_state()["spins"], b.get_state()["spins"])


@pytest.mark.parametrize("k", [1, 120])
def test_step_parity_L8_full_population(k):
    """The L = 8, R = 10^5 workload with cluster moves: one GPU step from an
    exported state against the oracle's step."""
    from paper_1710_09025_amd import Pamc

    cfg = pi.WORKLOADS["L8_R100000"]
    inst = make(cfg["L"], cfg["R"], cfg["n_temps"], cfg["sweeps"], cfg["beta_max"], cfg["disorder_seed"], cfg["seed"])
    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2)
    assert p.anneal(k) == 0
    st = p.get_state()
    assert st["step"] == k
    assert p.anneal(1) == 0
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, icm_rounds=2)
    o.set_state(k, st["spins"], st["family"], st["lnZ"])
    assert o.run(1) == 0
    compare_state(p.get_state(), o.get_state(), f"icm step {k}")
    go, oo = p.observables(), o.records()
    assert go["sum_E"][k] == oo["sumE"][k] and go["sum_E2"][k] == oo["sumE2"][k]
    S, _ = p.step_sums()
    assert S[k] == oo["S"][k]


def test_graph_replay_direct_launches_and_separate_gather_agree():
    from paper_1710_09025_amd import Pamc

    inst = make(5, 700, 13, 4, 4.0, 51, 52)
    runs = [Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                 icm_rounds=2, **kw) for kw in ({}, {"graphs": False}, {"fuse_gather": False}, {"timing": True})]
    for p in runs:
        assert p.anneal() == 0
    s0 = runs[0].get_state()
    for p in runs[1:]:
        compare_state(s0, p.get_state(), "icm launch forms")


def test_checkpoint_resume_with_cluster_moves():
    from paper_1710_09025_amd import Pamc

    inst = make(8, 800, 21, 6, 4.0, 61, 62)
    full = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2)
    part = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2)
    assert full.anneal() == 0 and part.anneal(9) == 0
    st = part.get_state()
    resumed = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], icm_rounds=2)
    resumed.set_state(st["step"], st["spins"], st["family"], st["lnZ"])
    assert resumed.anneal() == 0
    compare_state(resumed.get_state(), full.get_state(), "icm resume")


def test_batch_with_cluster_moves_matches_oracle():
    from paper_1710_09025_amd import PamcBatch

    specs = [(3, 300, 9, 4, False), (4, 500, 11, 5, False), (8, 400, 7, 3, False), (6, 250, 9, 4, True)]
    insts = [make(L, R, nT, NS, 4.0, 70 + i, 75 + i, real) for i, (L, R, nT, NS, real) in enumerate(specs)]
    b = PamcBatch(insts, icm_rounds=2)
    assert b.anneal() == 0
    for i, inst in enumerate(insts):
        o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                          threads=THREADS, icm_rounds=2)
        assert o.run() == 0
        compare_state(b.get_state(i), o.get_state(), f"icm batch instance {i}")
        assert rel_close(b.observables(i)["lnZ"], o.observables()["lnZ"])[0]


def test_rho_f_with_cluster_moves_runs():
    from paper_1710_09025_amd import free_energy_variance

    J = pi.pm_j_couplings(4, 5)
    r = free_energy_variance(4, J, 500, pi.linear_beta(3.0, 21), 4, seeds=range(6), icm_rounds=2)
    assert np.all(np.isfinite(r["rho_f"])) and r["betaF"].shape == (6, 21)
