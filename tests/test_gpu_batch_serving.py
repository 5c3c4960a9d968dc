"""The batched and served forms at the shapes of their workloads, against
separate runs and the oracle, and the failure paths of the library (through
the C ABI, on the GPU).

* Batches whose instances span several 1024-row blocks (R >= 3000, more
  than 2048 families), so that one resampling launch scans block totals and
  folds family sums of many instances at once, bit for bit against the
  oracle at every step.
* The 2000-instance mixed-size workload's shape (L in {4, 6, 8, 10, 12},
  R = 20000, 201 temperatures, autotuned tiles): batched results equal
  separate runs at every step, and the oracle's first steps and a late step
  from an exported state.
* Serving: a request admitted while another is mid-anneal (forced by the
  memory budget, not by timing), results equal to alone runs and to the
  oracle at every step; a request cancelled in flight; the memory budget
  returns to zero.
* Failure handling: extinction at the same step as the oracle, alone and
  inside a batch; a process that stops after a checkpoint and a new
  process that resumes from it.
"""
import ctypes
import os
import subprocess
import sys
import time

import numpy as np
import pytest

import oracle
import pamc_inputs as pi
from parity import THREADS, compare_obs, compare_state, instance, same_obs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def orc(inst, steps=-1, **kw):
    o = oracle.Oracle(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
                      threads=THREADS, pop_schedule=inst.get("pop_schedule"), **kw)
    st = o.run(steps)
    return o, st


def alone(inst, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"],
             pop_schedule=inst.get("pop_schedule"), **kw)
    st = p.anneal()
    return p, st


# --------------------------------------------------------------------------
# Batches of multi-block instances
# --------------------------------------------------------------------------
MULTI_BLOCK = [(4, 3000), (5, 3100), (6, 4099), (8, 3072), (10, 3500), (12, 3001), (4, 5200), (6, 3333),
               (7, 3010), (8, 4500), (10, 3000), (12, 3800)]


def test_batch_of_multi_block_instances_matches_oracle_every_step():
    """Twelve instances of 3000-5200 replicas (three to six row blocks and
    two or more family chunks each; ragged last blocks), L = 4 ... 12 with
    both sweep kernels of the colour-major family and the even/odd-x kernel,
    autotuned shapes: spins, energies, families and every step's records
    against the oracle."""
    from paper_1710_09025_amd import PamcBatch

    insts = [instance(L, R, 21, 10, 5.0, disorder_seed=500 + i, seed=600 + i)
             for i, (L, R) in enumerate(MULTI_BLOCK)]
    b = PamcBatch(insts, autotune=True)
    assert b.anneal() == 0
    for i, inst in enumerate(insts):
        o, st = orc(inst)
        assert st == 0
        what = f"multi-block batch member {i} (L={inst['L']}, R={inst['R']})"
        compare_state(b.get_state(i), o.get_state(), what)
        compare_obs(b.observables(i), o, what=what)
    b.close()


def test_c4_shape_batch_equals_separate_runs():
    """Ten instances of the mixed-size workload (R = 20000 in 20 row blocks,
    201 temperatures, autotuned tiles, two of each L): the batch gives every
    instance the state and every observable of its separate run, and its
    first three steps equal the oracle's."""
    from paper_1710_09025_amd import PamcBatch

    insts = pi.batch_instances(10)
    assert sorted(d["L"] for d in insts) == [4, 4, 6, 6, 8, 8, 10, 10, 12, 12]
    assert all(d["R"] == 20000 and len(d["beta"]) == 201 for d in insts)
    b = PamcBatch(insts, autotune=True)
    assert b.anneal() == 0
    for i, d in enumerate(insts):
        what = f"C4-shape member {i} (L={d['L']})"
        p, st = alone(d, autotune=True)
        assert st == 0
        bo = b.observables(i)
        same_obs(bo, p.observables(), what)
        compare_state(b.get_state(i), p.get_state(), what)
        p.close()
        o, st = orc(d, steps=3)
        assert st == 0
        compare_obs(bo, o, steps=3, what=what + " vs oracle")
    b.close()


@pytest.mark.parametrize("L,k", [(10, 100), (12, 150)])
def test_c4_shape_late_step_matches_oracle(L, k):
    """R = 20000, 201 temperatures, a late step from an exported state:
    colour-major sweeps over 20 row blocks and the resampling, bit for bit."""
    from paper_1710_09025_amd import Pamc

    d = next(x for x in pi.batch_instances(10) if x["L"] == L)
    p = Pamc(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"], autotune=True)
    assert p.anneal(k) == 0
    st = p.get_state()
    assert st["step"] == k
    assert p.anneal(1) == 0
    o = oracle.Oracle(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"], threads=THREADS)
    o.set_state(k, st["spins"], st["family"], st["lnZ"])
    assert o.run(1) == 0
    compare_state(p.get_state(), o.get_state(), f"L={L} step {k}")
    go, oo = p.observables(), o.records()
    for g, r in (("R", "R"), ("sum_E", "sumE"), ("sum_E2", "sumE2"), ("E_min", "Emin"), ("E_max", "Emax")):
        assert go[g][k] == oo[r][k], g
    S, T = p.step_sums()
    assert S[k] == oo["S"][k] and T[k] == oo["T"][k]


# --------------------------------------------------------------------------
# Serving
# --------------------------------------------------------------------------
def request_bytes(d):
    """What a request occupies of the server's budget: its run's device
    footprint plus 4096 bytes."""
    from paper_1710_09025_amd import _capi

    lib = _capi.load()
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    return lib.pamc_footprint(d["L"], d["R"], len(d["beta"]), ctypes.byref(opt)) + 4096


def submit(srv, d):
    return srv.submit(d["L"], d["couplings"], d["R"], d["beta"], d["sweeps"], d["seed"])


def test_request_joins_a_running_anneal():
    """A (61 temperatures, R = 5000) and F (20 temperatures) fill the
    budget; B does not fit beside them, so it waits until F leaves after 20
    steps and joins while A is mid-anneal: A.admit < B.admit < A.finish.
    Every request's observables equal its alone run's and the oracle's at
    every step, and the budget is empty at the end."""
    from paper_1710_09025_amd import PamcServer

    A = instance(8, 5000, 61, 10, 5.0, disorder_seed=700, seed=701)
    F = instance(6, 1500, 20, 10, 5.0, disorder_seed=702, seed=703)
    B = instance(10, 3000, 31, 10, 5.0, disorder_seed=704, seed=705)
    bA, bF, bB = request_bytes(A), request_bytes(F), request_bytes(B)
    assert bB > bF
    budget = bA + bB + 1024          # A + F fit, A + F + B do not, A + B do
    assert bA + bF <= budget < bA + bF + bB
    srv = PamcServer(budget, max_active=8)
    try:
        ids = [submit(srv, d) for d in (A, F, B)]
        res = [srv.wait(r, timeout=300) for r in ids]
        usage = srv.usage()
    finally:
        srv.close()
    (sA, oA, tA), (sF, oF, tF), (sB, oB, tB) = res
    assert sA == sF == sB == 0
    assert tA["admit"] < tB["admit"] < tA["finish"], (tA, tB)
    assert tF["finish"] <= tB["admit"], (tF, tB)
    assert usage["used_bytes"] == 0 and usage["budget_bytes"] == budget
    for name, d, obs in (("A", A, oA), ("F", F, oF), ("B", B, oB)):
        p, st = alone(d)
        assert st == 0
        same_obs(obs, p.observables(), f"request {name} mixed vs alone")
        p.close()
        o, st = orc(d)
        assert st == 0
        compare_obs(obs, o, what=f"request {name} vs oracle")


def test_c5_shape_requests_alone_equal_mixed():
    """Eight requests of the serving workload (L 4 ... 14, R 5000 ... 50000,
    101 temperatures) submitted together to a 4 GiB server: each result
    equals the request's separate run at every step; the first two steps
    of each also equal the oracle's."""
    from paper_1710_09025_amd import PamcServer

    reqs = pi.serving_requests(8)
    srv = PamcServer(4 << 30, max_active=256)
    try:
        ids = [submit(srv, d) for d in reqs]
        res = [srv.wait(r, timeout=600) for r in ids]
    finally:
        srv.close()
    for i, (d, (st, obs, _)) in enumerate(zip(reqs, res)):
        assert st == 0
        what = f"C5 request {i} (L={d['L']}, R={d['R']})"
        p, st = alone(d)
        assert st == 0
        same_obs(obs, p.observables(), what)
        p.close()
        o, st = orc(d, steps=2)
        assert st == 0
        compare_obs(obs, o, steps=2, what=what + " vs oracle")


def test_cancel_a_running_request():
    """X (20001 temperatures) is cancelled once it runs: its poll reports
    PAMC_ERR_STATE, its memory returns to the budget, and Y, which ran
    beside it, equals its alone run."""
    from paper_1710_09025_amd import PamcServer, _capi

    X = instance(4, 2000, 20001, 2, 5.0, disorder_seed=710, seed=711)
    Y = instance(5, 1500, 41, 4, 5.0, disorder_seed=712, seed=713)
    srv = PamcServer(1 << 30, max_active=8)
    try:
        rx = submit(srv, X)
        t0 = time.time()
        while srv.stats()["active"] < 1:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        ry = submit(srv, Y)
        sy, oy, _ = srv.wait(ry, timeout=120)
        assert srv.poll(rx) is None, "X finished before it could be cancelled"
        assert srv.cancel(rx) == 0
        sx, _, tx = srv.wait(rx, timeout=60)
        assert sx == _capi.ERR_STATE
        assert srv.cancel(rx) == _capi.ERR_STATE  # already cancelled
        t0 = time.time()
        while srv.usage()["used_bytes"] != 0:
            assert time.time() - t0 < 10
            time.sleep(0.001)
        st = srv.stats()
        assert st["active"] == 0 and st["queued"] == 0
    finally:
        srv.close()
    assert sy == 0
    p, st = alone(Y)
    same_obs(oy, p.observables(), "request beside a cancelled one")


# --------------------------------------------------------------------------
# Failure handling
# --------------------------------------------------------------------------
def extinct_case():
    """An instance whose population schedule targets one replica after step
    1 (Sec. III.D: the nominal population R(beta)), with the first MC seed
    for which the oracle's run dies out."""
    L, R, nT = 4, 200, 6
    J = pi.pm_j_couplings(L, 720)
    beta = pi.linear_beta(2.0, nT)
    pop = np.array([R, R, 1, 1, 1, 1], dtype=np.int64)
    for seed in range(100):
        d = dict(L=L, couplings=J, R=R, beta=beta, sweeps=2, seed=seed, pop_schedule=pop)
        o, st = orc(d)
        if st == oracle.ERR_EXTINCT:
            return d, o
    raise AssertionError("no extinct run among 100 seeds")


def test_extinction_is_reported_like_the_oracle():
    from paper_1710_09025_amd import _capi

    d, o = extinct_case()
    p, st = alone(d)
    assert st == _capi.ERR_EXTINCT
    gs = p.get_state()
    assert gs["step"] == o.step
    compare_state(gs, o.get_state(), "after extinction")
    k = o.step
    obs, rec = p.observables(), o.records()
    compare_obs(obs, o, steps=k, what="records before the extinct step")
    for g, r in (("R", "R"), ("sum_E", "sumE"), ("sum_E2", "sumE2"), ("E_min", "Emin"), ("E_max", "Emax")):
        assert obs[g][k] == rec[r][k], g
    assert np.isnan(obs["lnQ"][k]) and obs["measured"][k] == 1 and obs["measured"][k + 1] == 0
    assert p.anneal() == _capi.ERR_EXTINCT  # sticky


def test_extinction_inside_a_batch_leaves_the_others_alone():
    from paper_1710_09025_amd import PamcBatch, _capi

    d, o = extinct_case()
    other = instance(5, 700, 6, 2, 2.0, disorder_seed=721, seed=722)
    b = PamcBatch([other, d, other])
    assert b.anneal() == _capi.ERR_EXTINCT
    assert b.get_state(1)["step"] == o.step
    compare_state(b.get_state(1), o.get_state(), "extinct batch member")
    oo, st = orc(other)
    assert st == 0
    for i in (0, 2):
        compare_state(b.get_state(i), oo.get_state(), f"batch member {i} beside an extinct one")
        compare_obs(b.observables(i), oo, what=f"batch member {i}")


CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, {root!r})
import pamc_inputs as pi
from paper_1710_09025_amd import Pamc
J = pi.pm_j_couplings(8, 730)
p = Pamc(8, J, 3000, pi.linear_beta(5.0, 41), 5, 731)
assert p.anneal(17) == 0
st = p.get_state()
np.savez({path!r}, step=st["step"], R=st["R"], lnZ=st["lnZ"], spins=st["spins"], family=st["family"])
p.anneal_async(10)
assert p.sync() == 0
print("checkpoint at step", st["step"], flush=True)
import os
os._exit(0)   # stop without releasing anything, as a killed process would
"""


def test_resume_in_a_new_process_after_the_first_stops(tmp_path):
    """A child process anneals to step 17, writes a checkpoint, runs on and
    stops without cleaning up; this process resumes from the checkpoint.
    The resumed run equals an uninterrupted run and the oracle resumed from
    the same checkpoint."""
    from paper_1710_09025_amd import Pamc

    path = str(tmp_path / "ckpt.npz")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, path=path)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    ck = np.load(path)
    assert int(ck["step"]) == 17
    J = pi.pm_j_couplings(8, 730)
    beta = pi.linear_beta(5.0, 41)
    res = Pamc(8, J, 3000, beta, 5, 731)
    res.set_state(int(ck["step"]), ck["spins"], ck["family"], float(ck["lnZ"]))
    assert res.anneal() == 0
    full = Pamc(8, J, 3000, beta, 5, 731)
    assert full.anneal() == 0
    compare_state(res.get_state(), full.get_state(), "resumed vs uninterrupted")
    a, b = res.observables(), full.observables()
    for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f"):
        assert list(a[key][17:]) == list(b[key][17:]), key
    o = oracle.Oracle(8, J, 3000, beta, 5, 731, threads=THREADS)
    o.set_state(17, ck["spins"], ck["family"], float(ck["lnZ"]))
    assert o.run() == 0
    compare_state(res.get_state(), o.get_state(), "resumed vs oracle")
