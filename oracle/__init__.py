"""Plain CPU oracle for population annealing Monte Carlo (arXiv:1710.09025).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never imports, links or calls it, and it shares no code with the GPU
library.

The C sources follow the paper step by step:

* ``pamc_oracle.c`` -- the PAMC algorithm of Sec. II.B (random start at
  beta = 0, N_S checkerboard Metropolis sweeps per temperature, resampling
  with mean copy numbers proportional to exp[-(beta'-beta) E_i]), the
  observables of Eq. (2) and Eq. (9), and the free energy by free-energy
  perturbation.
* ``enumerate.c`` -- exact enumeration of every configuration of tiny
  lattices (Eq. (1)): density of states and overlap distribution.

Couplings are int8 +-1, or int32 fixed-point real couplings J = j 2^-20
(the paper's Gaussian case study, Sec. II.A); the dtype of the array picks
the model.  Energies of real-coupling runs are int64 in units of 2^-20.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAMC_ORACLE_LIB points the binding at another build of the same sources
# (the sanitizer and mutation tests use it); default: the in-tree build
LIB_PATH = os.environ.get("PAMC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SOURCES = ["pamc_oracle.c", "enumerate.c"]

OK = 0
ERR_INVALID = -1
ERR_NOMEM = -2
ERR_CAPACITY = -3
ERR_EXTINCT = -4

OBS_FIELDS = ("beta", "R", "mean_E", "e", "C_V", "lnQ", "lnZ", "betaF", "f", "S_f", "rho_s", "g_SG")


def build(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (IEEE doubles, no FMA contraction)."""
    cmd = [
        "gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
        *[os.path.join(_HERE, s) for s in SOURCES],
        "-o", LIB_PATH + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        L.orc_create.restype = P
        L.orc_create.argtypes = [i32, P, i64, i64, P, i32, i32, u64, P, P]
        L.orc_create_real.restype = P
        L.orc_create_real.argtypes = [i32, P, i64, i64, P, i32, i32, u64, P, P]
        L.orc_create_real_dim.restype = P
        L.orc_create_real_dim.argtypes = [i32, i32, P, i64, i64, P, i32, i32, u64, P, P]
        L.orc_records_wide.argtypes = [P, P]
        L.orc_get_state64.argtypes = [P, P, P, P]
        L.orc_energies64.argtypes = [P, P, i64, P]
        L.orc_sweep_rows64.argtypes = [P, i32, i64, P, P, P]
        L.orc_exp_f32.restype = ctypes.c_float
        L.orc_exp_f32.argtypes = [ctypes.c_float]
        L.orc_real_accept.argtypes = [ctypes.c_float, i64, ctypes.c_uint32]
        L.enum_energies_real.argtypes = [i32, P, P]
        L.orc_set_icm.argtypes = [P, i32, dbl]
        L.orc_icm_perm.restype = ctypes.c_uint32
        L.orc_icm_perm.argtypes = [u64, ctypes.c_uint32, ctypes.c_uint32, i32, i32]
        L.orc_icm_pair.argtypes = [P, P, P, ctypes.c_uint32, i32, i32]
        L.orc_destroy.argtypes = [P]
        L.orc_set_threads.argtypes = [P, i32]
        L.orc_run.argtypes = [P, i32]
        L.orc_step.argtypes = [P]
        L.orc_population.restype = i64
        L.orc_population.argtypes = [P]
        L.orc_num_spins.argtypes = [P]
        L.orc_lnZ.restype = dbl
        L.orc_lnZ.argtypes = [P]
        L.orc_records.argtypes = [P, P, P, P]
        L.orc_get_state.argtypes = [P, P, P, P]
        L.orc_set_state.argtypes = [P, i32, i64, P, P, dbl]
        L.orc_energies.argtypes = [P, P, i64, P]
        L.orc_colouring.argtypes = [P, P, P]
        L.orc_neighbours.argtypes = [P, P]
        L.orc_observables.argtypes = [P, P, P]
        L.orc_thresholds.argtypes = [dbl, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_make_pm_j.argtypes = [i32, u64, P]
        L.orc_sweep_rows.argtypes = [P, i32, i64, P, P, P]
        L.orc_measure_resample.argtypes = [P]
        L.enum_dos.argtypes = [i32, P, P]
        L.enum_energies.argtypes = [i32, P, P]
        L.enum_overlap.argtypes = [i32, P, dbl, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_capacity(R: int) -> int:
    """Population capacity R + ceil(8 sqrt(R)) + 64 (a >= 16 sigma margin)."""
    return int(R + int(np.ceil(8.0 * np.sqrt(R))) + 64)


def philox4x32_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def make_pm_j(L: int, disorder_seed: int) -> np.ndarray:
    """The oracle's +-J instance for a disorder seed, int8 [3][L^3]."""
    out = np.zeros(3 * L ** 3, dtype=np.int8)
    if lib().orc_make_pm_j(int(L), ctypes.c_uint64(int(disorder_seed) & (2**64 - 1)), _ptr(out)) != OK:
        raise ValueError("orc_make_pm_j: invalid arguments")
    return out.reshape(3, L ** 3)


def exp_f32(x: float) -> float:
    """The oracle's binary32 exponential (acceptance with real couplings)."""
    return float(lib().orc_exp_f32(ctypes.c_float(x)))


def real_accept(bq: float, dE: int, u: int) -> bool:
    """Acceptance of a move with dE > 0 (units of 2^-20) at binary32 bq."""
    return bool(lib().orc_real_accept(ctypes.c_float(bq), int(dE), ctypes.c_uint32(u)))


def real_beta(beta: float) -> np.float32:
    """beta 2^-20 rounded to binary32."""
    return np.float32(beta * 2.0 ** -20)


def icm_perm(seed: int, i: int, n: int, step: int, round_: int) -> int:
    """The oracle's keyed permutation of [0, n) used to pair replicas."""
    return int(lib().orc_icm_perm(ctypes.c_uint64(seed & (2**64 - 1)), i, n, step, round_))


def thresholds(beta: float):
    T = np.zeros(3, dtype=np.uint32)
    flag = ctypes.c_int(0)
    lib().orc_thresholds(ctypes.c_double(beta), _ptr(T), ctypes.byref(flag))
    return T, bool(flag.value)


def lattice_dim(L: int, couplings) -> int:
    """Dimension of the lattice a coupling array describes: [3][L^3] is the
    cubic lattice, [2][L^2] the square one."""
    n = np.asarray(couplings).size
    if n == 3 * L ** 3:
        return 3
    if n == 2 * L ** 2:
        return 2
    raise ValueError(f"couplings of size {n} fit neither [3][L^3] nor [2][L^2] for L = {L}")


class Oracle:
    """One PAMC run on the CPU.  ``couplings`` is int8 [3][L^3] of +-1, or
    int32 [D][L^D] of fixed-point real couplings (J = j 2^-20, |J| < 8) on
    the cubic (D = 3) or square (D = 2) lattice."""

    def __init__(self, L, couplings, R, beta, sweeps, seed, capacity=None, overlap_steps=None,
                 threads=1, pop_schedule=None, icm_rounds=0, icm_beta_min=0.0):
        self.L = int(L)
        self.dim = lattice_dim(self.L, couplings)
        self.N = self.L ** self.dim
        self.R = int(R)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.nT = len(self.beta)
        self.sweeps = int(sweeps)
        self.seed = int(seed)
        self._pop = None
        if pop_schedule is not None:
            self._pop = np.ascontiguousarray(pop_schedule, dtype=np.int64)
        peak = int(self._pop.max()) if self._pop is not None else self.R
        self.capacity = int(capacity) if capacity is not None else default_capacity(peak)
        self.real = np.asarray(couplings).dtype == np.int32
        dt = np.int32 if self.real else np.int8
        J = np.ascontiguousarray(couplings, dtype=dt).reshape(self.dim, self.N)
        self._J = J
        if self.real:
            dim = self.dim

            def create(*args):
                return lib().orc_create_real_dim(dim, *args)
        elif self.dim == 3:
            create = lib().orc_create
        else:
            raise ValueError("oracle: 2D lattices take real couplings")
        ov = None
        if overlap_steps is not None:
            ov = np.zeros(self.nT, dtype=np.uint8)
            ov[np.asarray(overlap_steps, dtype=np.int64)] = 1
            self._ov = ov
        h = create(self.L, _ptr(J), self.R, self.capacity, _ptr(self.beta), self.nT,
                             self.sweeps, ctypes.c_uint64(self.seed & (2**64 - 1)),
                             _ptr(ov) if ov is not None else None,
                             _ptr(self._pop) if self._pop is not None else None)
        if not h:
            raise ValueError("oracle: invalid arguments")
        self._h = ctypes.c_void_p(h)
        lib().orc_set_threads(self._h, int(threads))
        lib().orc_set_icm(self._h, int(icm_rounds), ctypes.c_double(icm_beta_min))

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_threads(self, n: int):
        lib().orc_set_threads(self._h, int(n))

    def run(self, n_steps: int = -1) -> int:
        return lib().orc_run(self._h, int(n_steps))

    @property
    def step(self) -> int:
        return lib().orc_step(self._h)

    @property
    def population(self) -> int:
        return lib().orc_population(self._h)

    @property
    def lnZ(self) -> float:
        return lib().orc_lnZ(self._h)

    def records(self):
        """Per-step records; sumE2 is a Python int per step (exact)."""
        ints = np.zeros((self.nT, 5), dtype=np.int64)
        dbl = np.zeros((self.nT, 4), dtype=np.float64)
        q = np.zeros((self.nT, 2 * self.N + 1), dtype=np.int64)
        lib().orc_records(self._h, _ptr(ints), _ptr(dbl), _ptr(q))
        wide = np.zeros((self.nT, 6), dtype=np.int64)
        lib().orc_records_wide(self._h, _ptr(wide))
        sumE2 = [int(np.uint64(lo)) + (int(hi) << 64) for lo, hi in zip(wide[:, 2], wide[:, 3])]
        return {"R": ints[:, 0], "sumE": wide[:, 1], "sumE2": np.array(sumE2, dtype=object),
                "Emin": wide[:, 4], "Emax": wide[:, 5], "S": dbl[:, 0], "T": dbl[:, 1],
                "lnQ": dbl[:, 2], "lnZ": dbl[:, 3], "qhist": q}

    def observables(self):
        out = np.zeros((self.nT, 12), dtype=np.float64)
        ovl = np.zeros((self.nT, 3), dtype=np.float64)
        lib().orc_observables(self._h, _ptr(out), _ptr(ovl))
        d = {name: out[:, i] for i, name in enumerate(OBS_FIELDS)}
        d["q_abs"], d["q2"], d["q4"] = ovl[:, 0], ovl[:, 1], ovl[:, 2]
        return d

    def get_state(self):
        Rk = self.population
        spins = np.zeros((Rk, self.N), dtype=np.int8)
        E = np.zeros(Rk, dtype=np.int64 if self.real else np.int32)
        fam = np.zeros(Rk, dtype=np.uint32)
        get = lib().orc_get_state64 if self.real else lib().orc_get_state
        get(self._h, _ptr(spins), _ptr(E), _ptr(fam))
        return {"step": self.step, "R": Rk, "spins": spins, "E": E, "family": fam, "lnZ": self.lnZ}

    def set_state(self, step, spins, family, lnZ):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        family = np.ascontiguousarray(family, dtype=np.uint32)
        Rk = spins.shape[0]
        st = lib().orc_set_state(self._h, int(step), int(Rk), _ptr(spins), _ptr(family),
                                 ctypes.c_double(lnZ))
        if st != OK:
            raise ValueError(f"oracle set_state failed: {st}")

    def sweep_rows(self, step, rows, spins):
        """N_S sweeps of step `step` applied to the given replicas, keyed by
        their row indices; returns (spins after, energies)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        sp = np.array(spins, dtype=np.int8, order="C", copy=True)
        E = np.zeros(len(rows), dtype=np.int64 if self.real else np.int32)
        sweep = lib().orc_sweep_rows64 if self.real else lib().orc_sweep_rows
        st = sweep(self._h, int(step), len(rows), _ptr(rows), _ptr(sp), _ptr(E))
        if st != OK:
            raise ValueError(f"oracle sweep_rows failed: {st}")
        return sp, E

    def measure_resample(self) -> int:
        """Measure and resample the current population without sweeping it."""
        return lib().orc_measure_resample(self._h)

    def icm_pair(self, a, b, pair_index, step, round_):
        """One cluster update of the configurations a, b (int8 +-1, copied);
        returns (a', b', island size)."""
        sa = np.array(a, dtype=np.int8, order="C", copy=True)
        sb = np.array(b, dtype=np.int8, order="C", copy=True)
        n = lib().orc_icm_pair(self._h, _ptr(sa), _ptr(sb), int(pair_index), int(step), int(round_))
        return sa, sb, n

    def energies(self, spins):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        E = np.zeros(spins.shape[0], dtype=np.int64 if self.real else np.int32)
        en = lib().orc_energies64 if self.real else lib().orc_energies
        en(self._h, _ptr(spins), int(spins.shape[0]), _ptr(E))
        return E

    def colouring(self):
        c = np.zeros(self.N, dtype=np.int32)
        r = np.zeros(self.N, dtype=np.int32)
        ncol = lib().orc_colouring(self._h, _ptr(c), _ptr(r))
        return ncol, c, r

    def neighbours(self):
        nb = np.zeros((self.N, 6), dtype=np.int32)
        lib().orc_neighbours(self._h, _ptr(nb))
        return nb


def density_of_states(L, couplings) -> np.ndarray:
    """g[(E + 3N)/2] = number of configurations with energy E (N <= 30)."""
    N = L ** 3
    J = np.ascontiguousarray(couplings, dtype=np.int8).reshape(3, N)
    g = np.zeros(3 * N + 1, dtype=np.int64)
    st = lib().enum_dos(int(L), _ptr(J), _ptr(g))
    if st != 0:
        raise ValueError("enumeration too large")
    return g


def all_energies(L, couplings) -> np.ndarray:
    N = L ** 3
    J = np.ascontiguousarray(couplings, dtype=np.int8).reshape(3, N)
    E = np.zeros(2 ** N, dtype=np.int32)
    if lib().enum_energies(int(L), _ptr(J), _ptr(E)) != 0:
        raise ValueError("enumeration too large")
    return E


def all_energies_real(L, couplings) -> np.ndarray:
    """Energies (int64, units of 2^-20) of all 2^N configurations of an
    instance with fixed-point real couplings; bit s of the index is S_s = +1."""
    N = L ** 3
    J = np.ascontiguousarray(couplings, dtype=np.int32).reshape(3, N)
    E = np.zeros(2 ** N, dtype=np.int64)
    if lib().enum_energies_real(int(L), _ptr(J), _ptr(E)) != 0:
        raise ValueError("enumeration too large")
    return E


def exact_thermo_real(E_fixed: np.ndarray, N: int, beta):
    """Exact ln Z, <E>, C_V at each beta from every configuration's energy."""
    E = E_fixed.astype(np.float64) * 2.0 ** -20
    out = {"lnZ": [], "mean_E": [], "C_V": []}
    for b in np.atleast_1d(beta):
        a = -b * E
        amax = a.max()
        w = np.exp(a - amax)
        Z = w.sum()
        m1 = (w * E).sum() / Z
        m2 = (w * E * E).sum() / Z
        out["lnZ"].append(amax + np.log(Z))
        out["mean_E"].append(m1)
        out["C_V"].append(b * b * (m2 - m1 * m1) / N)
    return {k: np.array(v) for k, v in out.items()}


def overlap_distribution(L, couplings, beta) -> np.ndarray:
    N = L ** 3
    J = np.ascontiguousarray(couplings, dtype=np.int8).reshape(3, N)
    P = np.zeros(2 * N + 1, dtype=np.float64)
    if lib().enum_overlap(int(L), _ptr(J), ctypes.c_double(beta), _ptr(P)) != 0:
        raise ValueError("enumeration too large")
    return P


def exact_thermo(g: np.ndarray, N: int, beta):
    """Exact ln Z, <E>, C_V at each beta from the density of states."""
    E = np.arange(len(g)) * 2 - 3 * N
    mask = g > 0
    E, lg = E[mask].astype(np.float64), np.log(g[mask].astype(np.float64))
    out = {"lnZ": [], "mean_E": [], "C_V": []}
    for b in np.atleast_1d(beta):
        a = lg - b * E
        amax = a.max()
        w = np.exp(a - amax)
        Z = w.sum()
        m1 = (w * E).sum() / Z
        m2 = (w * E * E).sum() / Z
        out["lnZ"].append(amax + np.log(Z))
        out["mean_E"].append(m1)
        out["C_V"].append(b * b * (m2 - m1 * m1) / N)
    return {k: np.array(v) for k, v in out.items()}
