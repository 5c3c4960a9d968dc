"""The C-ABI library loads and exports every entry point declared in
include/pamc.h; host-side argument validation returns the documented status
codes before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pamc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(pamc_[a-z_0-9]+)\s*\(", text))
    # typedef'd struct names are not functions
    return sorted(n for n in names if not n.endswith("_t"))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_09025_amd import _capi

    return _capi.load()


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("pamc_create", "pamc_anneal", "pamc_observables", "pamc_get_state", "pamc_set_state",
              "pamc_batch_create", "pamc_server_submit"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_1710_09025_amd import _capi

    assert set(declared_functions()) == set(_capi.SIGNATURES)


def test_status_strings(lib):
    for st in range(0, -9, -1):
        assert lib.pamc_status_string(st)


def test_default_options(lib):
    from paper_1710_09025_amd import _capi

    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    assert opt.fuse_gather == 1 and opt.device == -1 and opt.capacity == 0


def test_footprint_scales_with_population(lib):
    a = lib.pamc_footprint(8, 10000, 201, None)
    b = lib.pamc_footprint(8, 20000, 201, None)
    assert 0 < a < b
    # two spin buffers of R_cap rows of N bytes dominate
    cap = 20000 + int(np.ceil(8 * np.sqrt(20000))) + 64
    assert b >= 2 * cap * 512
    assert lib.pamc_footprint(1, 10, 10, None) == -1


STRUCTS = {
    "pamc_options": "Options",
    "pamc_step_obs": "StepObs",
    "pamc_state": "State",
    "pamc_instance": "Instance",
    "pamc_server_options": "ServerOptions",
    "pamc_result": "Result",
}


def test_struct_layouts_match_the_header(tmp_path):
    """Every field of the binding's ctypes structures sits at the offset the
    C compiler gives it in include/pamc.h, and the sizes agree."""
    from paper_1710_09025_amd import _capi

    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(_capi, pyname)
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{pyname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        pyname, field, value = line.split()
        cls = getattr(_capi, pyname)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (pyname, field, got, value)


@pytest.mark.parametrize("case", ["tile_rows", "lds", "group_waves", "group_large"])
def test_invalid_sweep_shapes_are_rejected_on_the_host(lib, case):
    from paper_1710_09025_amd import _capi

    L = {"tile_rows": 8, "lds": 16, "group_waves": 4, "group_large": 10}[case]
    J = np.ones((3, L ** 3), dtype=np.int8)
    beta = np.linspace(0, 1, 3)
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    if case == "tile_rows":
        opt.tile_rows = 5000
    elif case == "lds":
        opt.tile_rows = 64          # 64 rows of 4096 bytes exceed the workgroup's LDS
    elif case == "group_waves":
        opt.group_replicas = 6      # not a multiple of four: replicas are swept in fours
    else:
        opt.group_replicas = 64     # 128 threads per replica quad: 2048 threads
    h = ctypes.c_void_p()
    st = lib.pamc_create(L, J.ctypes.data_as(ctypes.c_void_p), 100, beta.ctypes.data_as(ctypes.c_void_p),
                         len(beta), 1, 1, ctypes.byref(opt), ctypes.byref(h))
    assert st == _capi.ERR_INVALID, lib.pamc_last_error()
    assert not h.value


@pytest.mark.parametrize("case", ["range", "lattice", "capacity", "null"])
def test_invalid_real_couplings_are_rejected_on_the_host(lib, case):
    from paper_1710_09025_amd import _capi

    L = 22 if case == "lattice" else 6
    J = np.zeros((3, L ** 3), dtype=np.int32)
    R = 100
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    if case == "range":
        J[2, 7] = 1 << 23           # |J| = 8
    elif case == "capacity":
        opt.capacity = (1 << 29) + 1
    beta = np.linspace(0, 1, 3)
    h = ctypes.c_void_p()
    ptr = None if case == "null" else J.ctypes.data_as(ctypes.c_void_p)
    st = lib.pamc_create_real(L, ptr, R, beta.ctypes.data_as(ctypes.c_void_p), len(beta), 1, 1,
                              ctypes.byref(opt), ctypes.byref(h))
    assert st == _capi.ERR_INVALID, lib.pamc_last_error()
    assert not h.value


@pytest.mark.parametrize("case", ["packed", "rounds", "window"])
def test_invalid_cluster_move_options_are_rejected_on_the_host(lib, case):
    from paper_1710_09025_amd import _capi

    L = 4
    J = np.ones((3, L ** 3), dtype=np.int8)
    beta = np.linspace(0, 1, 3)
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    if case == "packed":
        opt.icm_rounds = 2
        opt.spin_format = _capi.SPINS_PACKED
    elif case == "rounds":
        opt.icm_rounds = 9
    else:
        opt.icm_rounds = 2
        opt.icm_beta_min = float("nan")
    h = ctypes.c_void_p()
    st = lib.pamc_create(L, J.ctypes.data_as(ctypes.c_void_p), 100, beta.ctypes.data_as(ctypes.c_void_p),
                         len(beta), 2, 1, ctypes.byref(opt), ctypes.byref(h))
    assert st == _capi.ERR_INVALID, lib.pamc_last_error()
    assert not h.value


def test_real_footprint_adds_64_bit_energies_and_weights(lib):
    from paper_1710_09025_amd import _capi

    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    a = lib.pamc_footprint(8, 100000, 201, ctypes.byref(opt))
    opt.real_couplings = 1
    b = lib.pamc_footprint(8, 100000, 201, ctypes.byref(opt))
    cap = 100000 + int(np.ceil(8 * np.sqrt(100000))) + 64
    # two 8-byte energy buffers and the weights replace two 4-byte buffers
    assert b - a >= cap * (3 * 8 - 2 * 4)
    # no kernel for real couplings at L = 22
    assert lib.pamc_footprint(22, 1000, 11, ctypes.byref(opt)) == -1


def test_packed_footprint_saves_the_spin_bytes(lib):
    from paper_1710_09025_amd import _capi

    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    a = lib.pamc_footprint(16, 500000, 301, ctypes.byref(opt))
    opt.spin_format = _capi.SPINS_PACKED
    b = lib.pamc_footprint(16, 500000, 301, ctypes.byref(opt))
    cap = 500000 + int(np.ceil(8 * np.sqrt(500000))) + 64
    # two buffers of cap rows shrink from 4096 to 512 bytes (256-byte carving slack)
    assert abs((a - b) - 2 * cap * (4096 - 512)) <= 512


@pytest.mark.parametrize("case", ["L", "coupling", "beta_order", "beta_nan", "R", "sweeps", "capacity",
                                  "pop_first", "pop_zero", "beta0_positive", "beta0_negative_zero_only"])
def test_invalid_arguments_are_rejected_on_the_host(lib, case):
    from paper_1710_09025_amd import _capi

    L, R, NS = 4, 100, 2
    J = np.ones((3, 64), dtype=np.int8)
    beta = np.linspace(0, 1, 5)
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    if case == "L":
        L = 1
    elif case == "coupling":
        J[1, 5] = 0
    elif case == "beta_order":
        beta = beta[::-1].copy()
    elif case == "beta_nan":
        beta[2] = np.nan
    elif case == "beta0_positive":
        # the random initial population is the beta = 0 sample and ln Z is
        # anchored there (Sec. II.B): any other first temperature is refused
        beta = beta + 0.25
    elif case == "beta0_negative_zero_only":
        beta = np.full(5, 0.4)
    elif case == "R":
        R = 0
    elif case == "sweeps":
        NS = 0
    elif case == "capacity":
        opt.capacity = 50
    elif case in ("pop_first", "pop_zero"):
        pop = np.full(len(beta), R, dtype=np.int64)
        if case == "pop_first":
            pop[0] = R + 1
        else:
            pop[3] = 0
        opt.pop_schedule = pop.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    h = ctypes.c_void_p()
    st = lib.pamc_create(L, J.ctypes.data_as(ctypes.c_void_p), R, beta.ctypes.data_as(ctypes.c_void_p),
                         len(beta), NS, 1, ctypes.byref(opt), ctypes.byref(h))
    assert st == _capi.ERR_INVALID
    assert not h.value
    assert lib.pamc_last_error()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_1710_09025_amd import _capi

    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(_capi.LibraryMissing):
        _capi.load()


def test_square_lattice_options_on_the_host(lib):
    """dim = 2 sizes a real-coupling run of L^2 spins; +-1 couplings, a
    dimension other than 2 or 3 and L > 64 are rejected before any device
    work."""
    from paper_1710_09025_amd import _capi

    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    assert opt.dim == 0
    three = lib.pamc_footprint(8, 10000, 101, ctypes.byref(opt))
    opt.dim = 2
    two = lib.pamc_footprint(32, 10000, 101, ctypes.byref(opt))
    cap = 10000 + int(np.ceil(8 * np.sqrt(10000))) + 64
    assert two >= 2 * cap * 1024 and three > 0
    assert lib.pamc_footprint(64, 100, 11, ctypes.byref(opt)) > 0
    assert lib.pamc_footprint(65, 100, 11, ctypes.byref(opt)) == -1
    opt.dim = 4
    assert lib.pamc_footprint(8, 100, 11, ctypes.byref(opt)) == -1
    beta = np.linspace(0, 1, 3)
    for dim, real, Lc in [(2, False, 4), (4, True, 4), (2, True, 65)]:
        opt.dim = dim
        N = Lc ** (3 if dim == 4 else dim)
        J = np.ones((3 if dim == 4 else dim) * N, dtype=np.int32 if real else np.int8)
        h = ctypes.c_void_p()
        create = lib.pamc_create_real if real else lib.pamc_create
        st = create(Lc, J.ctypes.data_as(ctypes.c_void_p), 100, beta.ctypes.data_as(ctypes.c_void_p), len(beta),
                    2, 1, ctypes.byref(opt), ctypes.byref(h))
        assert st == _capi.ERR_INVALID, (dim, real, Lc, lib.pamc_last_error())
        assert not h.value


def _batch_instance(L, J, R, beta, NS, seed):
    from paper_1710_09025_amd import _capi

    return _capi.Instance(L, J.ctypes.data_as(ctypes.c_void_p).value, R, beta.ctypes.data_as(ctypes.c_void_p).value,
                          len(beta), NS, seed, None, None)


def test_batch_rejects_a_positive_first_temperature_on_the_host(lib):
    """pamc_batch_create validates every instance before any device work;
    the error names the instance."""
    from paper_1710_09025_amd import _capi

    J = np.ones((3, 64), dtype=np.int8)
    good = np.linspace(0, 1, 5)
    bad = np.linspace(0.1, 1, 5)
    arr = (_capi.Instance * 2)(_batch_instance(4, J, 50, good, 2, 1), _batch_instance(4, J, 50, bad, 2, 2))
    h = ctypes.c_void_p()
    st = lib.pamc_batch_create(2, arr, None, ctypes.byref(h))
    assert st == _capi.ERR_INVALID and not h.value
    assert b"instance 1" in lib.pamc_last_error() and b"beta[0]" in lib.pamc_last_error()


def test_real_couplings_reject_a_positive_first_temperature_on_the_host(lib):
    from paper_1710_09025_amd import _capi

    Jq = np.full((3, 64), 1 << 20, dtype=np.int32)
    beta = np.array([0.5, 1.0])
    h = ctypes.c_void_p()
    st = lib.pamc_create_real(4, Jq.ctypes.data_as(ctypes.c_void_p), 10, beta.ctypes.data_as(ctypes.c_void_p), 2,
                              1, 1, None, ctypes.byref(h))
    assert st == _capi.ERR_INVALID and not h.value


def test_oracle_rejects_a_positive_first_temperature():
    import oracle
    import pamc_inputs as pi

    J = pi.pm_j_couplings(3, 1)
    with pytest.raises(ValueError):
        oracle.Oracle(3, J, 10, [0.3, 0.6], 1, 1)
    oracle.Oracle(3, J, 10, [0.0, 0.6], 1, 1)


@pytest.mark.parametrize("L,seed", [(2, 0), (3, 1), (4, 1), (5, 2 ** 63 + 7), (8, 2), (12, 99), (16, 3),
                                    (32, 123456789)])
def test_make_pm_j_matches_the_oracle_and_the_input_module(lib, L, seed):
    """The library's coupling stream (its own host Philox) draws the same
    instance as the oracle's generator and the input module's; the values
    are +-1 and about half of each."""
    import oracle
    import pamc_inputs as pi
    from paper_1710_09025_amd import make_pm_j

    a = make_pm_j(L, seed)
    np.testing.assert_array_equal(a, oracle.make_pm_j(L, seed))
    np.testing.assert_array_equal(a, pi.pm_j_couplings(L, seed))
    assert set(np.unique(a)) <= {-1, 1}
    n = a.size
    assert abs(int((a > 0).sum()) - n / 2) < 6 * np.sqrt(n / 4) + 2


def test_make_pm_j_words_are_bit_31_of_the_coupling_stream(lib):
    """Bond b is +1 exactly when bit 31 of word (b & 3) of the oracle's
    Philox at counter (b >> 2, 0, 0, 5 * 2^28) is set."""
    import oracle
    from paper_1710_09025_amd import make_pm_j

    L, seed = 3, 0x1234_5678_9ABC
    a = make_pm_j(L, seed).reshape(-1)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for b in range(a.size):
        w = oracle.philox4x32_10([b >> 2, 0, 0, 0x50000000], key)[b & 3]
        assert a[b] == (1 if int(w) >> 31 else -1), b


def test_make_pm_j_rejects_bad_arguments(lib):
    from paper_1710_09025_amd import _capi

    out = np.zeros(3 * 64, dtype=np.int8)
    assert lib.pamc_make_pm_j(1, 5, out.ctypes.data_as(ctypes.c_void_p)) == _capi.ERR_INVALID
    assert lib.pamc_make_pm_j(33, 5, out.ctypes.data_as(ctypes.c_void_p)) == _capi.ERR_INVALID
    assert lib.pamc_make_pm_j(4, 5, None) == _capi.ERR_INVALID


def test_rho_f_is_the_sample_variance_times_the_nominal_population(lib):
    """Eq. (4) through the library: against numpy's ddof-1 variance, a case
    with a known answer, constant runs (variance 0) and invalid inputs."""
    from paper_1710_09025_amd import _capi, rho_f

    rng = np.random.default_rng(7)
    bf = rng.normal(-40.0, 0.3, size=(13, 9))
    Rn = rng.integers(100, 10000, size=9).astype(np.float64)
    mean, var, rf = rho_f(bf, Rn)
    np.testing.assert_allclose(mean, bf.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(var, bf.var(axis=0, ddof=1), rtol=1e-12)
    np.testing.assert_allclose(rf, Rn * bf.var(axis=0, ddof=1), rtol=1e-12)
    # two runs at -1 and +1: mean 0, variance (1 + 1) / 1 = 2
    mean, var, rf = rho_f(np.array([[-1.0], [1.0]]), [50.0])
    assert mean[0] == 0.0 and var[0] == 2.0 and rf[0] == 100.0
    mean, var, rf = rho_f(np.full((4, 3), -7.25), 10.0)
    assert np.all(var == 0.0) and np.all(rf == 0.0) and np.all(mean == -7.25)
    one = np.zeros((1, 3))
    out = np.zeros(3)
    assert lib.pamc_rho_f(one.ctypes.data_as(ctypes.c_void_p), 1, 3, out.ctypes.data_as(ctypes.c_void_p), None,
                          None, None) == _capi.ERR_INVALID


def test_static_entry_refuses_oversize_runs_on_the_host(lib):
    """pamc_anneal_static takes every device buffer from a fixed array; a run
    that needs more is refused with PAMC_ERR_INVALID before any device work
    (no GPU needed for the refusal)."""
    from paper_1710_09025_amd import _capi

    L, R = 16, 100000
    J = np.ones((3, L ** 3), dtype=np.int8)
    beta = np.linspace(0.0, 1.0, 11)
    obs = (_capi.StepObs * 11)()
    st = lib.pamc_anneal_static(L, J.ctypes.data_as(ctypes.c_void_p), R, beta.ctypes.data_as(ctypes.c_void_p), 11,
                                2, 1, None, obs, None)
    assert st == _capi.ERR_INVALID
    assert b"allocation-free" in lib.pamc_last_error()
    # invalid arguments are refused the same way
    assert lib.pamc_anneal_static(L, None, R, beta.ctypes.data_as(ctypes.c_void_p), 11, 2, 1, None, obs,
                                  None) == _capi.ERR_INVALID
