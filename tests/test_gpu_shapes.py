"""Sweep workgroup shapes and the autotuner: the shape changes speed only,
never results (through the C ABI, on the GPU)."""
import numpy as np
import pytest

from parity import compare_state, instance

pytestmark = pytest.mark.gpu


def run(inst, **kw):
    from paper_1710_09025_amd import Pamc

    p = Pamc(inst["L"], inst["couplings"], inst["R"], inst["beta"], inst["sweeps"], inst["seed"], **kw)
    assert p.anneal() == 0
    return p


def same_run(a, b, what):
    compare_state(a.get_state(), b.get_state(), what)
    oa, ob = a.observables(), b.observables()
    for key in ("R", "sum_E", "sum_E2", "lnZ", "S_f", "g_SG"):
        np.testing.assert_array_equal(oa[key], ob[key], err_msg=f"{what}: {key}")


# (L, shapes as (tile_rows, group_replicas)): colour-major with two and three
# colours (8 threads per replica quad at L = 4, 125 at L = 10, 216 at L = 12,
# 194 at L = 13, 343 at L = 14: quads above 64 threads leave the last wave
# partly idle, and groups of them take the 512-, 768- and 1024-thread
# kernels; tiles that are not multiples of four leave a quad partly empty),
# even/odd-x (L = 8, 16), per-site (L = 24); ragged tiles and single-pass
# workgroups
SHAPES = [
    (4, [(32, 32), (40, 32), (128, 64), (1000, 256)]),
    (5, [(16, 16), (40, 16), (128, 128)]),
    (10, [(4, 4), (7, 4), (16, 8), (6, 16), (24, 12)]),
    (12, [(4, 4), (12, 12), (24, 8), (40, 16)]),
    (13, [(8, 4), (16, 8), (24, 12), (32, 16)]),
    (14, [(8, 4), (16, 8), (10, 8)]),
    (8, [(8, 0), (16, 0), (64, 0)]),
    (16, [(2, 0), (4, 0), (14, 0)]),
    (24, [(1, 0), (3, 0)]),
]


@pytest.mark.parametrize("L,shapes", SHAPES)
def test_every_sweep_shape_gives_identical_results(L, shapes):
    R = {4: 700, 5: 300, 10: 90, 12: 61, 13: 61, 14: 37, 8: 333, 16: 40, 24: 7}[L]
    inst = instance(L, R, 7, 3, 4.0, disorder_seed=30 + L, seed=40 + L)
    base = run(inst)
    for tr, g in shapes:
        p = run(inst, tile_rows=tr, group_replicas=g)
        got = p.sweep_shape()
        assert got[0] >= tr, got
        same_run(base, p, f"L={L} tile_rows={tr} group_replicas={g}")


def test_autotune_is_cached_and_applied():
    from paper_1710_09025_amd import autotune

    inst = instance(6, 3000, 9, 4, 4.0, disorder_seed=50, seed=51)
    t1, g1, ns1 = autotune(6, 3000, 4)
    assert t1 >= 1 and g1 >= 1 and ns1 > 0
    t2, g2, ns2 = autotune(6, 3000, 4)
    assert (t1, g1, ns1) == (t2, g2, ns2)  # cached: no second measurement
    p = run(inst, autotune=True)
    assert p.sweep_shape() == (t1, g1)
    same_run(run(inst), p, "autotuned vs default")


def test_autotuned_batch_equals_default_batch():
    from paper_1710_09025_amd import PamcBatch

    insts = []
    for i, L in enumerate([4, 8, 5, 6, 4]):
        d = instance(L, 400 + 50 * i, 6, 3, 4.0, disorder_seed=60 + i, seed=70 + i)
        insts.append(d)
    a = PamcBatch(insts)
    b = PamcBatch(insts, autotune=True)
    assert a.anneal() == 0 and b.anneal() == 0
    for i in range(len(insts)):
        compare_state(a.get_state(i), b.get_state(i), f"batch instance {i}")
        oa, ob = a.observables(i), b.observables(i)
        for key in ("R", "sum_E", "lnZ", "S_f"):
            np.testing.assert_array_equal(oa[key], ob[key])
