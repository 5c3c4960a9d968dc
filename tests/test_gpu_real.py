"""Real (Gaussian) couplings, Sec. II.A: the GPU library against the CPU
oracle through the C ABI.  Couplings are fixed point (J = j 2^-20), so
energies are exact integers and must match bit for bit, as must spins,
families, population sizes and overlap histograms; the normaliser S and the
family term are compared bitwise; derived observables within 1e-12."""
import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_run, compare_state, rel_close

pytestmark = pytest.mark.gpu


def real_instance(L, R, nT, sweeps=10, beta_max=4.0, disorder_seed=1, seed=1):
    return dict(L=L, couplings=pi.gaussian_couplings(L, disorder_seed), R=R,
                beta=pi.linear_beta(beta_max, nT), sweeps=sweeps, seed=seed)


def gpu_run(inst, steps=-1, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], **kw)
    assert p.real
    return p, p.anneal(steps)


def oracle_run(inst, steps=-1, **kw):
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, **kw)
    assert o.real
    return o, o.run(steps)


# (L, R, n_temps, sweeps, beta_max): two and three colours, 1 to 512
# threads per replica quad (L = 8 and 16 take the colour-major layout with
# real couplings), ragged quads and tiles; L = 2 with doubled bonds
CASES = [
    (2, 400, 15, 10, 4.0),
    (3, 500, 21, 10, 4.0),
    (4, 1000, 31, 10, 4.0),
    (5, 300, 15, 6, 4.0),
    (6, 333, 21, 4, 4.0),
    (7, 150, 11, 4, 3.0),
    (8, 1001, 21, 10, 4.0),
    (9, 61, 7, 3, 4.0),
    (10, 120, 11, 4, 4.0),
    (11, 37, 6, 3, 4.0),
    (12, 90, 9, 3, 4.0),
    (13, 19, 5, 2, 4.0),
    (16, 77, 7, 3, 4.0),
]


@pytest.mark.parametrize("L,R,nT,NS,bmax", CASES)
def test_full_run_bit_exact(L, R, nT, NS, bmax):
    inst = real_instance(L, R, nT, NS, bmax, disorder_seed=500 + L, seed=600 + L)
    p, st = gpu_run(inst)
    o, sto = oracle_run(inst)
    assert st == sto == 0
    gs = p.get_state()
    assert gs["E"].dtype == np.int64
    compare_state(gs, o.get_state(), f"real L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"real L={L}")
    np.testing.assert_array_equal(p.overlap_hist(nT - 1), o.records()["qhist"][nT - 1])


@pytest.mark.parametrize("L,R", [(20, 3), (21, 3)])
def test_largest_real_lattices(L, R):
    """The largest colour-major workgroups (1024 and 896 threads)."""
    inst = real_instance(L, R, 3, 1, 3.0, disorder_seed=700 + L, seed=710 + L)
    p, st = gpu_run(inst)
    o, sto = oracle_run(inst)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), f"real L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"real L={L}")


def test_large_temperature_steps_and_overlaps_at_every_step():
    inst = real_instance(6, 20000, 6, 3, 5.0, disorder_seed=21, seed=22)
    steps = list(range(6))
    p, st = gpu_run(inst, overlap_steps=steps)
    o, sto = oracle_run(inst, overlap_steps=steps)
    assert st == sto == 0
    compare_state(p.get_state(), o.get_state(), "real large d beta")
    compare_run(p.observables(), p.step_sums(), o, what="real large d beta")
    q = o.records()["qhist"]
    for k in steps:
        np.testing.assert_array_equal(p.overlap_hist(k), q[k], err_msg=f"overlap histogram, step {k}")


@pytest.mark.parametrize("k", [0, 100, 199])
def test_step_parity_L8_full_population(k):
    """The L = 8, R = 10^5, 201-temperature workload with Gaussian couplings:
    one GPU step from an exported state against the oracle's step."""
    cfg = pi.WORKLOADS["L8_R100000"]
    inst = real_instance(cfg["L"], cfg["R"], cfg["n_temps"], cfg["sweeps"], cfg["beta_max"], cfg["disorder_seed"],
                         cfg["seed"])
    p, _ = gpu_run(inst, steps=k)
    st = p.get_state()
    assert st["step"] == k
    p.anneal(1)
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS)
    o.set_state(k, st["spins"], st["family"], st["lnZ"])
    assert o.run(1) == 0
    compare_state(p.get_state(), o.get_state(), f"real step {k}")
    go, oo = p.observables(), o.records()
    assert go["R"][k] == oo["R"][k] and go["sum_E"][k] == oo["sumE"][k] and go["sum_E2"][k] == oo["sumE2"][k]
    assert go["E_min"][k] == oo["Emin"][k] and go["E_max"][k] == oo["Emax"][k]
    S, T = p.step_sums()
    assert T[k] == oo["T"][k]
    if k < inst["beta"].size - 1:
        assert S[k] == oo["S"][k]
        assert rel_close(go["lnQ"][k], oo["lnQ"][k])[0]


def test_sampled_parity_L12_large_population():
    """L = 12, R = 5 10^4: the sweeps of sampled rows at a mid-anneal step
    against the oracle one replica at a time, then the resampling of the
    whole post-sweep population."""
    from paper_1710_09025_amd import Pamc

    inst = real_instance(12, 50000, 61, 10, 4.0, disorder_seed=12, seed=13)
    k = 30
    a, _ = gpu_run(inst, steps=k)
    sk = a.get_state()
    a.anneal(1)
    s_next = a.get_state()
    b = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"][: k + 1], inst["sweeps"], inst["seed"])
    b.set_state(k, sk["spins"], sk["family"], sk["lnZ"])
    b.anneal(1)
    post = b.get_state()
    rng = np.random.default_rng(0)
    rows = np.sort(np.concatenate([[0, sk["R"] - 1], rng.choice(sk["R"], 62, replace=False)]))
    o = oracle.Oracle(inst["L"], inst["couplings"], 64, inst["beta"], inst["sweeps"], inst["seed"], threads=THREADS)
    sp, E = o.sweep_rows(k, rows, sk["spins"][rows])
    np.testing.assert_array_equal(sp, post["spins"][rows])
    np.testing.assert_array_equal(E, post["E"][rows])
    del o
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS)
    o.set_state(k, post["spins"], post["family"], sk["lnZ"])
    np.testing.assert_array_equal(o.get_state()["E"], post["E"])
    assert o.measure_resample() == 0
    compare_state(s_next, o.get_state(), "real resample at large size")


@pytest.mark.parametrize("L,shapes", [(5, [(16, 16), (40, 16), (128, 128)]), (6, [(8, 8), (36, 32), (256, 64)]),
                                      (8, [(4, 4), (24, 8), (64, 32)])])
def test_every_sweep_shape_gives_identical_results(L, shapes):
    inst = real_instance(L, 300, 7, 3, 4.0, disorder_seed=30 + L, seed=40 + L)
    base, _ = gpu_run(inst)
    for tr, g in shapes:
        p, _ = gpu_run(inst, tile_rows=tr, group_replicas=g)
        compare_state(base.get_state(), p.get_state(), f"real L={L} tile_rows={tr} group_replicas={g}")
        oa, ob = base.observables(), p.observables()
        for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f"):
            np.testing.assert_array_equal(oa[key], ob[key])


@pytest.mark.parametrize("L", [4, 7, 8])
def test_packed_spins_and_separate_gather_equal_default(L):
    inst = real_instance(L, 500, 11, 4, 4.0, disorder_seed=80 + L, seed=90 + L)
    a, _ = gpu_run(inst)
    b, _ = gpu_run(inst, packed=True)
    c, _ = gpu_run(inst, fuse_gather=False)
    sa = a.get_state()
    compare_state(sa, b.get_state(), "real packed")
    compare_state(sa, c.get_state(), "real separate gather")


def test_checkpoint_resume_equals_uninterrupted():
    from paper_1710_09025_amd import Pamc

    inst = real_instance(8, 800, 21, 5, 4.0, disorder_seed=5, seed=10)
    full, _ = gpu_run(inst)
    part, _ = gpu_run(inst, steps=9)
    st = part.get_state()
    resumed = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    resumed.set_state(st["step"], st["spins"], st["family"], st["lnZ"])
    resumed.anneal()
    compare_state(resumed.get_state(), full.get_state(), "real resume")
    a, b = resumed.observables(), full.observables()
    for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f"):
        np.testing.assert_array_equal(a[key][9:], b[key][9:])


def test_capacity_overflow_is_reported_like_the_oracle():
    inst = real_instance(4, 400, 41, 4, 5.0, disorder_seed=8, seed=21)
    cap = 402
    p, st = gpu_run(inst, capacity=cap)
    o, sto = oracle_run(inst, capacity=cap)
    assert sto == oracle.ERR_CAPACITY
    assert st == sto
    compare_state(p.get_state(), o.get_state(), "real after capacity failure")


def test_batch_mixing_pm1_and_real_instances_matches_oracle():
    from paper_1710_09025_amd import PamcBatch
    from parity import instance

    insts = []
    for i, (L, R, nT, NS, real) in enumerate([(3, 300, 11, 4, True), (4, 500, 15, 5, False), (8, 700, 9, 3, True),
                                              (6, 250, 15, 4, False), (16, 40, 7, 3, True), (5, 333, 11, 4, True)]):
        mk = real_instance if real else instance
        insts.append(mk(L, R, nT, NS, 4.0, disorder_seed=140 + i, seed=170 + i))
    b = PamcBatch(insts)
    assert b.anneal() == 0
    for i, inst in enumerate(insts):
        o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                          threads=THREADS)
        assert o.run() == 0
        compare_state(b.get_state(i), o.get_state(), f"batch instance {i}")
        obs = b.observables(i)
        np.testing.assert_array_equal(obs["sum_E"], o.records()["sumE"])
        np.testing.assert_array_equal(obs["sum_E2"], o.records()["sumE2"])
        assert rel_close(obs["lnZ"], o.observables()["lnZ"])[0]


def test_server_real_request_matches_oracle():
    from paper_1710_09025_amd import PamcServer

    inst = real_instance(6, 600, 11, 3, 4.0, disorder_seed=190, seed=191)
    srv = PamcServer(hbm_budget_bytes=1 << 30, max_active=4)
    rid = srv.submit(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"])
    st, obs, _ = srv.wait(rid)
    srv.close()
    assert st == 0
    o, _ = oracle_run(inst)
    np.testing.assert_array_equal(obs["sum_E"], o.records()["sumE"])
    np.testing.assert_array_equal(obs["E_min"], o.records()["Emin"])
    assert rel_close(obs["lnZ"], o.observables()["lnZ"])[0]


def test_single_temperature_and_single_replica():
    for L, R, beta in [(4, 50, np.array([0.0])), (5, 1, pi.linear_beta(3.0, 8)), (6, 40, np.array([0.0, 1.3]))]:
        inst = dict(L=L, couplings=pi.gaussian_couplings(L, 300 + L), R=R, beta=beta, sweeps=2, seed=301 + L)
        p, st = gpu_run(inst)
        o, sto = oracle_run(inst)
        assert st == sto == 0
        compare_state(p.get_state(), o.get_state(), f"real L={L} R={R}")
        compare_run(p.observables(), p.step_sums(), o, what=f"real L={L} R={R}")
