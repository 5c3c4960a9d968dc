"""GPU library against the CPU oracle, through the C ABI.

Integers (spins, energies, families, population sizes, histograms) must
match bit for bit; the resampling normaliser and family term are compared
bitwise too (same IEEE operations in the same order); derived floating-point
observables within a relative 1e-12.
"""
import math

import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import compare_run, compare_state, instance, rel_close, run_oracle, THREADS

pytestmark = pytest.mark.gpu


def gpu_run(inst, steps=-1, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], **kw)
    st = p.anneal(steps)
    return p, st


def test_thresholds_match_oracle_bitwise():
    from paper_1710_09025_amd import Pamc

    inst = instance(4, 50, 101)
    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], 2, 1)
    T, acc = p.thresholds()
    for k, b in enumerate(inst["beta"]):
        To, ao = oracle.thresholds(float(b))
        assert bool(acc[k]) == ao
        np.testing.assert_array_equal(T[k], To)


def test_initial_population_matches_oracle():
    inst = instance(5, 700, 3)
    p, _ = gpu_run(inst, steps=0)
    o, _ = run_oracle(inst, steps=0)
    compare_state(p.get_state(), o.get_state(), "init")


# (L, R, n_temps, sweeps, beta_max): colour-major kernel with two colours
# (even L) and three (odd L), 1 to 384 threads per replica; L = 2 with
# doubled bonds; even/odd-x kernels (L = 8, 16); the lexicographic kernel
# (L = 24); tiles with ragged tails
CASES = [
    (2, 500, 21, 10, 5.0),
    (3, 800, 31, 10, 5.0),
    (4, 1000, 101, 10, 5.0),   # the L = 4, R = 1000, 101-temperature workload
    (5, 400, 21, 6, 4.0),
    (6, 333, 21, 4, 5.0),
    (7, 150, 11, 4, 3.0),
    (8, 2001, 31, 10, 5.0),
    (9, 61, 7, 3, 4.0),
    (10, 120, 11, 4, 4.0),
    (11, 37, 6, 3, 4.0),
    (12, 90, 9, 3, 4.0),
    (13, 19, 5, 2, 4.0),
    (14, 23, 5, 2, 4.0),
    (16, 150, 11, 10, 5.0),
    (24, 9, 4, 1, 4.0),
]


@pytest.mark.parametrize("L,R,nT,NS,bmax", CASES)
def test_full_run_bit_exact(L, R, nT, NS, bmax):
    inst = instance(L, R, nT, NS, bmax, disorder_seed=L, seed=100 + L)
    p, st = gpu_run(inst)
    o, sto = run_oracle(inst)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"L={L}")
    # overlap histogram of the last step
    np.testing.assert_array_equal(p.overlap_hist(nT - 1), o.records()["qhist"][nT - 1])


def test_large_temperature_steps_and_overlaps_at_every_step():
    """Six temperatures up to beta = 5 (d beta = 1): a few low-energy
    replicas receive most of the copies, so single row blocks own thousands
    of destinations.  R = 30000 spreads the overlap pairs over many
    workgroups; overlaps are recorded at every step."""
    inst = instance(6, 30000, 6, 3, 5.0, disorder_seed=21, seed=22)
    steps = list(range(6))
    p, st = gpu_run(inst, overlap_steps=steps)
    o, sto = run_oracle(inst, overlap_steps=steps)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), "large d beta")
    compare_run(p.observables(), p.step_sums(), o, what="large d beta")
    q = o.records()["qhist"]
    for k in steps:
        np.testing.assert_array_equal(p.overlap_hist(k), q[k], err_msg=f"overlap histogram, step {k}")
    # the copies really were concentrated
    assert p.observables()["R"][1] == o.records()["R"][1]


@pytest.mark.parametrize("L", [3, 8, 16])
def test_separate_gather_equals_fused(L):
    inst = instance(L, 300, 9, 4, 4.0, disorder_seed=3, seed=5)
    a, _ = gpu_run(inst, fuse_gather=True)
    b, _ = gpu_run(inst, fuse_gather=False)
    compare_state(a.get_state(), b.get_state(), "fused vs separate")
    oa, ob = a.observables(), b.observables()
    for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f"):
        np.testing.assert_array_equal(oa[key], ob[key])


def test_graph_replay_equals_direct_launches_every_step():
    """The captured step is replayed once per temperature; after every replay
    (with eager exports and synchronisation in between) the state equals the
    state of a run that launches the kernels directly."""
    inst = instance(6, 700, 12, 3, 4.0, disorder_seed=6, seed=12)
    from paper_1710_09025_amd import Pamc

    a = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], graphs=True)
    b = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], graphs=False)
    c = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], timing=True)
    for k in range(len(inst["beta"])):
        for p in (a, b, c):
            assert p.anneal(1) == 0
        sa = a.get_state()
        compare_state(sa, b.get_state(), f"graph vs direct, step {k}")
        compare_state(sa, c.get_state(), f"graph vs timed, step {k}")
    oa, ob = a.observables(), b.observables()
    for key in ("R", "sum_E", "lnZ", "S_f", "g_SG"):
        np.testing.assert_array_equal(oa[key], ob[key])


def test_torch_allocator_and_stream_give_same_result():
    inst = instance(8, 500, 11, 4, 4.0, disorder_seed=4, seed=6)
    a, _ = gpu_run(inst, torch_stream=False)
    b, _ = gpu_run(inst, torch_stream=True, torch_allocator=True)
    compare_state(a.get_state(), b.get_state(), "hipMalloc vs torch allocator")


def test_run_twice_is_identical():
    inst = instance(6, 1500, 21, 6, 5.0, disorder_seed=2, seed=9)
    a, _ = gpu_run(inst)
    b, _ = gpu_run(inst)
    compare_state(a.get_state(), b.get_state(), "run twice")


def test_checkpoint_resume_equals_uninterrupted():
    inst = instance(8, 800, 21, 5, 5.0, disorder_seed=5, seed=10)
    full, _ = gpu_run(inst)
    part, _ = gpu_run(inst, steps=9)
    st = part.get_state()
    assert st["step"] == 9
    from paper_1710_09025_amd import Pamc

    resumed = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    resumed.set_state(st["step"], st["spins"], st["family"], st["lnZ"])
    resumed.anneal()
    compare_state(resumed.get_state(), full.get_state(), "resume")
    a, b = resumed.observables(), full.observables()
    for key in ("R", "sum_E", "lnZ", "S_f"):
        np.testing.assert_array_equal(a[key][9:], b[key][9:])


@pytest.mark.parametrize("k", [0, 57, 199])
def test_step_parity_L8_full_population(k):
    """L = 8, R = 10^5, 201 temperatures: one GPU step from an exported state
    against the oracle's step from the same state."""
    cfg = pi.WORKLOADS["L8_R100000"]
    inst = instance(cfg["L"], cfg["R"], cfg["n_temps"], cfg["sweeps"], cfg["beta_max"], cfg["disorder_seed"],
                    cfg["seed"])
    p, _ = gpu_run(inst, steps=k)
    st = p.get_state()
    assert st["step"] == k
    p.anneal(1)
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS)
    o.set_state(k, st["spins"], st["family"], st["lnZ"])
    assert o.run(1) == 0
    compare_state(p.get_state(), o.get_state(), f"step {k}")
    go, oo = p.observables(), o.records()
    assert go["R"][k] == oo["R"][k] and go["sum_E"][k] == oo["sumE"][k] and go["sum_E2"][k] == oo["sumE2"][k]
    S, T = p.step_sums()
    assert T[k] == oo["T"][k]
    if k < inst["beta"].size - 1:
        assert S[k] == oo["S"][k]
        assert rel_close(go["lnQ"][k], oo["lnQ"][k])[0]


def test_sampled_parity_L16_full_population():
    """L = 16, R = 5 10^5, 301 temperatures at full size: the sweeps of a
    sample of rows at a mid-anneal step against the oracle one replica at a
    time, then the resampling of the whole GPU population against the
    oracle's resampling of the same post-sweep population."""
    from paper_1710_09025_amd import Pamc

    cfg = pi.WORKLOADS["L16_R500000"]
    inst = instance(cfg["L"], cfg["R"], cfg["n_temps"], cfg["sweeps"], cfg["beta_max"], cfg["disorder_seed"],
                    cfg["seed"])
    k = 120
    a, _ = gpu_run(inst, steps=k)
    sk = a.get_state()
    a.anneal(1)
    s_next = a.get_state()
    # post-sweep population of step k: a run whose last step is k
    b = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"][: k + 1], inst["sweeps"], inst["seed"])
    b.set_state(k, sk["spins"], sk["family"], sk["lnZ"])
    b.anneal(1)
    post = b.get_state()
    rng = np.random.default_rng(0)
    rows = np.sort(np.concatenate([[0, sk["R"] - 1], rng.choice(sk["R"], 62, replace=False)]))
    # the sweeps of a replica depend only on its row, the step and the seed
    o = oracle.Oracle(inst["L"], inst["couplings"], 64, inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS)
    sp, E = o.sweep_rows(k, rows, sk["spins"][rows])
    np.testing.assert_array_equal(sp, post["spins"][rows])
    np.testing.assert_array_equal(E, post["E"][rows])
    del o
    # resampling of the full post-sweep population
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS)
    o.set_state(k, post["spins"], post["family"], sk["lnZ"])
    np.testing.assert_array_equal(o.get_state()["E"], post["E"])
    assert o.measure_resample() == 0
    compare_state(s_next, o.get_state(), "resample at full size")


def test_capacity_overflow_is_reported_like_the_oracle():
    """A capacity barely above R fails at the same step in both, and the
    handle keeps that step's post-sweep population."""
    inst = instance(4, 400, 41, 4, 5.0, disorder_seed=8, seed=21)
    cap = 402
    p, st = gpu_run(inst, capacity=cap)
    o, sto = run_oracle(inst, capacity=cap)
    assert sto == oracle.ERR_CAPACITY
    assert st == sto
    gs = p.get_state()
    os_ = o.get_state()
    assert gs["step"] == o.step
    compare_state(gs, os_, "after capacity failure")


def test_batch_of_mixed_sizes_matches_oracle():
    from paper_1710_09025_amd import PamcBatch

    insts = [instance(L, R, nT, NS, 4.0, disorder_seed=40 + i, seed=70 + i)
             for i, (L, R, nT, NS) in enumerate([(3, 300, 11, 4), (4, 500, 15, 5), (8, 700, 9, 3), (6, 250, 15, 4),
                                                 (16, 40, 7, 3), (5, 333, 11, 4), (4, 64, 21, 2)])]
    b = PamcBatch(insts)
    assert b.anneal() == 0
    for i, inst in enumerate(insts):
        o, _ = run_oracle(inst)
        compare_state(b.get_state(i), o.get_state(), f"batch instance {i}")
        obs = b.observables(i)
        np.testing.assert_array_equal(obs["sum_E"], o.records()["sumE"])
        assert rel_close(obs["lnZ"], o.observables()["lnZ"])[0]


def test_server_results_alone_equal_mixed():
    from paper_1710_09025_amd import PamcServer

    insts = [instance(L, R, 11, 3, 4.0, disorder_seed=90 + i, seed=95 + i)
             for i, (L, R) in enumerate([(4, 600), (7, 200), (8, 900), (5, 300), (6, 450)])]
    srv = PamcServer(hbm_budget_bytes=1 << 30, max_active=8)
    alone = []
    for inst in insts:
        rid = srv.submit(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
        alone.append(srv.wait(rid))
    ids = [srv.submit(i["L"], i["couplings"], i["R"], i["beta"], i["sweeps"], i["seed"]) for i in insts]
    mixed = [srv.wait(r) for r in ids]
    srv.close()
    for i, inst in enumerate(insts):
        sa, oa, _ = alone[i]
        sm, om, _ = mixed[i]
        assert sa == sm == 0
        for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f", "g_SG"):
            np.testing.assert_array_equal(oa[key], om[key])
        o, _ = run_oracle(inst)
        np.testing.assert_array_equal(oa["sum_E"], o.records()["sumE"])
        assert rel_close(oa["lnZ"], o.observables()["lnZ"])[0]


def test_server_rejects_requests_above_budget():
    from paper_1710_09025_amd import PamcError, PamcServer

    srv = PamcServer(hbm_budget_bytes=1 << 20)
    inst = instance(8, 5000, 11)
    with pytest.raises(PamcError) as e:
        srv.submit(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    assert e.value.status == -8
    srv.close()


def test_chunked_graphs_equal_direct_launches():
    """37 temperatures: two replays of the 16-step graph and five single-step
    replays give the state of direct launches."""
    inst = instance(5, 900, 37, 3, 4.0, disorder_seed=41, seed=42)
    a, _ = gpu_run(inst, graphs=True)
    b, _ = gpu_run(inst, graphs=False)
    compare_state(a.get_state(), b.get_state(), "chunked graphs vs direct")
    oa, ob = a.observables(), b.observables()
    for key in ("R", "sum_E", "lnZ", "S_f"):
        np.testing.assert_array_equal(oa[key], ob[key])
