"""Bit-packed spin storage (one bit per site in HBM): every result equals the
byte-per-site run and the oracle (through the C ABI, on the GPU)."""
import numpy as np
import pytest

from parity import compare_run, compare_state, instance, run_oracle

pytestmark = pytest.mark.gpu


def run(inst, steps=-1, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], **kw)
    assert p.anneal(steps) == 0
    return p


# every sweep kernel: colour-major (L = 2, 3, 4, 5, 12), even/odd-x (8, 16),
# per-site (24); packed rows of 16 to 1728 bytes
@pytest.mark.parametrize("L,R,nT,NS", [(2, 300, 9, 4), (3, 200, 9, 4), (4, 700, 11, 4), (5, 150, 9, 3),
                                       (8, 900, 11, 4), (12, 60, 7, 2), (16, 40, 7, 2), (24, 6, 4, 1)])
def test_packed_equals_bytes(L, R, nT, NS):
    inst = instance(L, R, nT, NS, 4.0, disorder_seed=80 + L, seed=90 + L)
    steps = list(range(nT))
    a = run(inst, overlap_steps=steps)
    b = run(inst, overlap_steps=steps, packed=True)
    compare_state(a.get_state(), b.get_state(), f"packed L={L}")
    oa, ob = a.observables(), b.observables()
    for key in ("R", "sum_E", "sum_E2", "E_min", "E_max", "lnZ", "S_f", "g_SG"):
        np.testing.assert_array_equal(oa[key], ob[key], err_msg=f"L={L} {key}")
    for k in steps:
        np.testing.assert_array_equal(a.overlap_hist(k), b.overlap_hist(k), err_msg=f"L={L} overlap {k}")


@pytest.mark.parametrize("L", [5, 8])
def test_packed_matches_oracle(L):
    inst = instance(L, 500, 21, 5, 5.0, disorder_seed=100 + L, seed=110 + L)
    p = run(inst, packed=True)
    o, st = run_oracle(inst)
    assert st == 0
    compare_state(p.get_state(), o.get_state(), f"packed vs oracle L={L}")
    compare_run(p.observables(), p.step_sums(), o, what=f"packed L={L}")


@pytest.mark.parametrize("L", [4, 8, 16])
def test_packed_separate_gather_and_resume(L):
    inst = instance(L, 300, 13, 3, 4.0, disorder_seed=120 + L, seed=130 + L)
    full = run(inst, packed=True)
    sep = run(inst, packed=True, fuse_gather=False)
    compare_state(full.get_state(), sep.get_state(), "packed, separate gather")
    part = run(inst, steps=6, packed=True)
    st = part.get_state()
    from paper_1710_09025_amd import Pamc

    res = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], packed=True)
    res.set_state(st["step"], st["spins"], st["family"], st["lnZ"])
    assert res.anneal() == 0
    compare_state(res.get_state(), full.get_state(), "packed resume")


def test_packed_batch_equals_byte_batch():
    from paper_1710_09025_amd import PamcBatch

    insts = [instance(L, 300 + 40 * i, 6, 3, 4.0, disorder_seed=140 + i, seed=150 + i)
             for i, L in enumerate([4, 6, 8, 5])]
    a = PamcBatch(insts)
    b = PamcBatch(insts, packed=True)
    assert a.anneal() == 0 and b.anneal() == 0
    for i in range(len(insts)):
        compare_state(a.get_state(i), b.get_state(i), f"batch {i}")
