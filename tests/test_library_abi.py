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
                                  "pop_first", "pop_zero"])
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
