"""The square lattice (D = 2, Sec. II.A) on the GPU against the CPU oracle,
through the C ABI: spins, families, energies, population sizes and the
per-step integer sums bit-exact, the normaliser and family term bitwise,
derived observables within 1e-12; with and without cluster moves."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state, rel_close

pytestmark = pytest.mark.gpu


def inst2d(L, R, nT, NS, bmax, dseed, seed, pm=False):
    J = pi.pm_j_couplings_2d(L, dseed) if pm else pi.gaussian_couplings(L, dseed, dim=2)
    return dict(L=L, couplings=J, R=R, beta=pi.linear_beta(bmax, nT), sweeps=NS, seed=seed)


def gpu(inst, steps=-1, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], **kw)
    assert p.dim == 2 and p.real
    return p, p.anneal(steps)


def orc(inst, steps=-1, **kw):
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, **kw)
    assert o.dim == 2
    return o, o.run(steps)


# two and three colours, ragged quads and tiles, L = 2 with doubled bonds,
# the paper's 2D sizes 8, 16, 25, 32 and the largest accepted lattices
CASES = [
    (2, 400, 15, 10, 4.0),
    (3, 500, 21, 10, 4.0),
    (4, 1000, 31, 10, 4.0),
    (5, 301, 15, 6, 4.0),
    (8, 1001, 21, 10, 5.0),
    (16, 300, 11, 5, 4.0),
    (25, 60, 7, 4, 4.0),
    (32, 50, 6, 3, 4.0),
    (63, 9, 4, 2, 3.0),
    (64, 8, 4, 2, 3.0),
]


@pytest.mark.parametrize("L,R,nT,NS,bmax", CASES)
def test_full_run_bit_exact(L, R, nT, NS, bmax):
    inst = inst2d(L, R, nT, NS, bmax, 700 + L, 800 + L)
    p, st = gpu(inst)
    o, sto = orc(inst)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"2D L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"2D L={L}")


def test_pm_j_instance_as_real_couplings():
    inst = inst2d(8, 800, 21, 10, 5.0, 3, 4, pm=True)
    p, st = gpu(inst)
    o, sto = orc(inst)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), "2D +-J")
    compare_run(p.observables(), p.step_sums(), o, what="2D +-J")
    # +-1 couplings: every energy is an even integer (2 unsatisfied bonds - 2N) in units of 2^20
    E = p.get_state()["E"]
    assert np.all(E % (2 << 20) == 0)


# island search: breadth-first below L = 8, row flood fill from L = 8 on, in
# 4-byte rows up to L = 32 (16 lanes per pair) and 8-byte rows beyond (32
# lanes); rows filling their whole word (L = 32, 64) and lengths that are
# not a multiple of four (25, 33)
@pytest.mark.parametrize("L,R,nT,NS", [(4, 400, 11, 6), (7, 300, 9, 4), (8, 501, 15, 10), (16, 200, 9, 4),
                                       (25, 64, 7, 4), (32, 60, 6, 2), (33, 24, 5, 2), (40, 30, 5, 2),
                                       (64, 8, 4, 2)])
def test_cluster_moves_bit_exact(L, R, nT, NS):
    inst = inst2d(L, R, nT, NS, 4.0, 900 + L, 950 + L)
    p, st = gpu(inst, icm_rounds=2)
    o, sto = orc(inst, icm_rounds=2)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"2D icm L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"2D icm L={L}")


def test_cluster_move_window_bit_exact():
    inst = inst2d(8, 300, 13, 4, 4.0, 21, 22)
    p, st = gpu(inst, icm_rounds=1, icm_beta_min=2.0)
    o, sto = orc(inst, icm_rounds=1, icm_beta_min=2.0)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), "2D icm window")


def test_launch_forms_agree():
    inst = inst2d(9, 700, 13, 4, 4.0, 31, 32)
    runs = []
    for kw in ({}, {"graphs": False}, {"fuse_gather": False}, {"timing": True}):
        p, st = gpu(inst, icm_rounds=2, **kw)
        assert st == 0
        runs.append(p.get_state())
    for s in runs[1:]:
        compare_state(runs[0], s, "2D launch forms")


def test_checkpoint_resume():
    from paper_1710_09025_amd import Pamc

    inst = inst2d(16, 600, 21, 6, 4.0, 41, 42)
    full, st = gpu(inst)
    part, st2 = gpu(inst, steps=9)
    assert st == st2 == 0
    s = part.get_state()
    resumed = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    resumed.set_state(s["step"], s["spins"], s["family"], s["lnZ"])
    assert resumed.anneal() == 0
    compare_state(resumed.get_state(), full.get_state(), "2D resume")
    assert rel_close(resumed.observables()["lnZ"][-1], full.observables()["lnZ"][-1])[0]


def test_batch_of_square_lattices_matches_oracle():
    from paper_1710_09025_amd import PamcBatch

    specs = [(4, 300, 9, 4), (7, 200, 11, 5), (8, 400, 7, 3), (16, 150, 9, 4), (25, 40, 5, 2)]
    insts = [inst2d(L, R, nT, NS, 4.0, 60 + i, 65 + i) for i, (L, R, nT, NS) in enumerate(specs)]
    b = PamcBatch(insts, icm_rounds=1)
    assert b.anneal() == 0
    for i, inst in enumerate(insts):
        o, st = orc(inst, icm_rounds=1)
        assert st == 0
        compare_state(b.get_state(i), o.get_state(), f"2D batch instance {i}")
        assert rel_close(b.observables(i)["lnZ"], o.observables()["lnZ"])[0]


def test_batch_rejects_mixed_dimensions():
    from paper_1710_09025_amd import PamcBatch

    a = inst2d(4, 100, 3, 2, 1.0, 1, 1)
    b = dict(L=4, couplings=pi.gaussian_couplings(4, 2), R=100, beta=pi.linear_beta(1.0, 3), sweeps=2, seed=2)
    with pytest.raises(ValueError):
        PamcBatch([a, b])


@pytest.mark.parametrize("k,icm", [(1, 0), (80, 0), (1, 2), (80, 2)])
def test_step_parity_L32_large_population(k, icm):
    """L = 32, R = 10^5 (the paper's largest 2D lattice): one GPU step from
    an exported state against the oracle's step on the same population,
    without and with two cluster-move rounds (5 10^4 pair updates each, in
    the launch form the benchmark times)."""
    inst = inst2d(32, 100000, 101, 10, 5.0, 5, 6)
    p, st = gpu(inst, steps=k, icm_rounds=icm)
    assert st == 0
    s = p.get_state()
    assert p.anneal(1) == 0
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, icm_rounds=icm)
    o.set_state(k, s["spins"], s["family"], s["lnZ"])
    assert o.run(1) == 0
    compare_state(p.get_state(), o.get_state(), f"2D L=32 step {k} icm={icm}")
    go, rec = p.observables(), o.records()
    assert go["sum_E"][k] == rec["sumE"][k] and go["sum_E2"][k] == rec["sumE2"][k]
    assert p.step_sums()[0][k] == rec["S"][k]


def test_autotuned_shapes_are_kept_apart_from_the_cubic_lattice():
    """The tuner's cache tells the two lattices of one L apart: a cubic and a
    square instance with the same L and population, tuned in one process,
    each run on a shape of its own and match the oracle."""
    from paper_1710_09025_amd import Pamc

    beta = pi.linear_beta(4.0, 9)
    cubic = Pamc(8, pi.gaussian_couplings(8, 3), 3000, beta, 4, 5, autotune=True)
    inst = dict(L=8, couplings=pi.gaussian_couplings(8, 4, dim=2), R=3000, beta=beta, sweeps=4, seed=6)
    p, st = gpu(inst, autotune=True)
    assert st == 0 and cubic.anneal() == 0
    o, sto = orc(inst)
    assert sto == 0
    compare_state(p.get_state(), o.get_state(), "2D after a cubic tuning")


@pytest.mark.parametrize("L", [5, 16, 32])
def test_packed_spins_equal_bytes(L):
    """Bit-packed rows (one bit per site in HBM) give the byte-row run bit for
    bit on the square lattice too (rows of 16 to 128 packed bytes)."""
    inst = inst2d(L, 300, 9, 4, 4.0, 110 + L, 120 + L)
    a, st = gpu(inst)
    b, st2 = gpu(inst, packed=True)
    assert st == st2 == 0
    compare_state(a.get_state(), b.get_state(), f"2D packed L={L}")
    for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f"):
        np.testing.assert_array_equal(a.observables()[key], b.observables()[key], err_msg=f"2D packed L={L}: {key}")


@pytest.mark.parametrize("L", [6, 16])
def test_schedules_population_and_overlaps(L):
    """The square lattice with the LBLT schedule, the clipped exponential
    population schedule R(beta) and spin overlaps at several steps: every
    record bit-exact, the overlap moments within 1e-12."""
    beta = pi.lblt_beta(5.0, 31)
    pop = pi.clipped_exponential_population(beta, 500)
    J = pi.gaussian_couplings(L, 130 + L, dim=2)
    steps = [5, 15, 30]
    from paper_1710_09025_amd import Pamc

    p = Pamc(L, J, int(pop[0]), beta, 4, 140 + L, pop_schedule=pop, overlap_steps=steps)
    assert p.anneal() == 0
    o = oracle.Oracle(L, J, int(pop[0]), beta, 4, 140 + L, threads=THREADS, pop_schedule=pop, overlap_steps=steps)
    assert o.run() == 0
    compare_state(p.get_state(), o.get_state(), f"2D schedules L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"2D schedules L={L}")
    rec = o.records()
    for k in steps:
        np.testing.assert_array_equal(p.overlap_hist(k), rec["qhist"][k], err_msg=f"2D overlap histogram step {k}")
