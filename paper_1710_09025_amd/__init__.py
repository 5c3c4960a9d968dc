"""Population annealing Monte Carlo for Edwards-Anderson spin glasses on
AMD Instinct MI355X (gfx950).

Couplings are int8 +-1, or int32 fixed-point real couplings J = j 2^-20
with |J| < 8 (the paper's Gaussian case study, Sec. II.A); the dtype of the
array picks the model.  Their shape picks the lattice: [3][L^3] is the
periodic cubic lattice, [2][L^2] the periodic square lattice (Sec. II.A
studies both; 2D takes real couplings).  Energies of real-coupling runs
(E_min, E_max, sum_E, sum_E2, state energies) are exact integers in units
of 2^-20.

Python binding of the C ABI in ``include/pamc.h``: it marshals arguments and
results; every step of the method runs in the HIP kernels of ``libpamc.so``.
PyTorch, when present, supplies the HIP stream and (optionally) the caching
allocator for device memory.  There is no CPU fallback: if the library is
missing, construction raises.

The method is that of Barzegar, Pattison, Wang and Katzgraber,
arXiv:1710.09025: Sec. II.B (population annealing with N_S Metropolis sweeps
per temperature and resampling proportional to exp[-(beta'-beta) E_i]),
Sec. III.A (checkerboard spin selection), Eq. (2) (family entropy), Sec. V.A
(observables, overlap histograms).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import _capi

__all__ = ["Pamc", "PamcBatch", "PamcServer", "PamcError", "OBS_FIELDS", "default_capacity", "make_pm_j", "rho_f",
           "free_energy_variance", "autotune", "calibrate", "anneal_static"]

OBS_FIELDS = ("beta", "R", "sum_E", "sum_E2", "E_min", "E_max", "mean_E", "e", "C_V", "lnQ", "lnZ",
              "betaF", "f", "S_f", "rho_s", "q_abs", "q2", "q4", "g_SG", "measured")


class PamcError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        lib = _capi.load()
        msg = lib.pamc_last_error().decode(errors="replace")
        name = lib.pamc_status_string(status).decode()
        super().__init__(f"{what}: {name} ({status}): {msg}")
        self.status = status


def _check(status: int, what: str):
    if status != _capi.OK:
        raise PamcError(status, what)


def default_capacity(R: int) -> int:
    return int(R + int(np.ceil(8.0 * np.sqrt(R))) + 64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _obs_to_dict(arr) -> dict:
    out = {}
    for name in OBS_FIELDS:
        if name == "sum_E2":
            # exact: low and high 64-bit halves of the 128-bit sum
            out[name] = np.array([(o.sum_E2 & (2**64 - 1)) + (o.sum_E2_hi << 64) for o in arr], dtype=object)
        else:
            out[name] = np.array([getattr(o, name) for o in arr])
    return out


def lattice_dim(L, couplings) -> int:
    """3 for couplings of size 3 L^3 (cubic lattice), 2 for size 2 L^2
    (square lattice)."""
    n = np.asarray(couplings).size
    if n == 3 * int(L) ** 3:
        return 3
    if n == 2 * int(L) ** 2:
        return 2
    raise ValueError(f"couplings of size {n} fit neither [3][L^3] nor [2][L^2] for L = {L}")


def _couplings(L, couplings):
    """(array, real, dim): int32 fixed-point real couplings, else int8 +-1,
    on the lattice of dimension dim."""
    real = np.asarray(couplings).dtype == np.int32
    dim = lattice_dim(L, couplings)
    J = np.ascontiguousarray(couplings, dtype=np.int32 if real else np.int8).reshape(dim, int(L) ** dim)
    return J, real, dim


class _TorchGlue:
    """Stream and caching-allocator callbacks from PyTorch (plumbing only)."""

    def __init__(self, use_allocator: bool):
        import torch  # noqa: F401

        self.torch = torch
        self.device = torch.cuda.current_device()
        # a stream of our own at the default priority; its handle is non-null
        self.stream = torch.cuda.Stream(device=self.device)
        self._alloc = None
        self._free = None
        if use_allocator:
            def _a(nbytes, _user):
                try:
                    return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
                except Exception:
                    return None

            def _f(ptr, _user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._alloc = _capi.ALLOC_FN(_a)
            self._free = _capi.FREE_FN(_f)

    def fill(self, opt: _capi.Options):
        opt.stream = ctypes.c_void_p(self.stream.cuda_stream)
        opt.device = self.device
        if self._alloc is not None:
            opt.alloc = self._alloc
            opt.free = self._free


def _torch_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def _make_options(capacity=None, overlap_steps=None, fuse_gather=True, spin_format=_capi.SPINS_INT8,
                  torch_stream=True, torch_allocator=False, keep=None, timing=False, tile_rows=0,
                  graphs=True, group_replicas=0, autotune=False, pop_schedule=None, icm_rounds=0,
                  icm_beta_min=0.0, dim=3):
    lib = _capi.load()
    opt = _capi.Options()
    lib.pamc_default_options(ctypes.byref(opt))
    opt.dim = int(dim)
    opt.spin_format = int(spin_format)
    if capacity is not None:
        opt.capacity = int(capacity)
    opt.fuse_gather = 1 if fuse_gather else 0
    opt.timing = 1 if timing else 0
    opt.tile_rows = int(tile_rows)
    opt.group_replicas = int(group_replicas)
    opt.autotune = 1 if autotune else 0
    opt.graphs = 1 if graphs else 0
    opt.icm_rounds = int(icm_rounds)
    opt.icm_beta_min = float(icm_beta_min)
    if pop_schedule is not None:
        pop = np.ascontiguousarray(pop_schedule, dtype=np.int64)
        keep.append(pop)
        opt.pop_schedule = pop.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if overlap_steps is not None:
        ov = np.ascontiguousarray(overlap_steps, dtype=np.int32)
        keep.append(ov)
        opt.overlap_steps = ov.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        opt.n_overlap_steps = len(ov)
    if torch_stream and _torch_available():
        glue = _TorchGlue(torch_allocator)
        glue.fill(opt)
        keep.append(glue)
    return opt


def autotune(L, R, sweeps, torch_stream=True, packed=False, real=False, dim=3):
    """Sweep workgroup shape chosen by measurement (``pamc_autotune``):
    (tile_rows, group_replicas, sweep ns per attempt).  Choices are cached
    per process and read from the tuning file shipped beside the library and
    from the file ``PAMC_TUNE_CACHE`` names, to which new ones are appended."""
    keep = []
    opt = _make_options(torch_stream=torch_stream, keep=keep, dim=dim,
                        spin_format=_capi.SPINS_PACKED if packed else _capi.SPINS_INT8)
    opt.real_couplings = 1 if real else 0
    t, g, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_capi.load().pamc_autotune(int(L), int(R), int(sweeps), ctypes.byref(opt), ctypes.byref(t),
                                      ctypes.byref(g), ctypes.byref(ns)), "pamc_autotune")
    return t.value, g.value, ns.value


def make_pm_j(L: int, disorder_seed: int) -> np.ndarray:
    """+-J instance of the library's coupling stream (``pamc_make_pm_j``),
    int8 [3][L^3]."""
    out = np.zeros(3 * int(L) ** 3, dtype=np.int8)
    _check(_capi.load().pamc_make_pm_j(int(L), ctypes.c_uint64(int(disorder_seed) & (2**64 - 1)), _ptr(out)),
           "pamc_make_pm_j")
    return out.reshape(3, int(L) ** 3)


def anneal_static(L, couplings, R, beta, sweeps, seed, stream=None, state=True):
    """One whole anneal without device allocation (``pamc_anneal_static``):
    returns (status, observables dict, final state dict or None)."""
    J = np.ascontiguousarray(couplings, dtype=np.int8).reshape(3, int(L) ** 3)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    nT = len(b)
    arr = (_capi.StepObs * nT)()
    st_ptr = None
    bufs = None
    if state:
        cap = default_capacity(int(R))
        N = int(L) ** 3
        bufs = (np.zeros((cap, N), dtype=np.int8), np.zeros(cap, dtype=np.int32), np.zeros(cap, dtype=np.uint32))
        st_ptr = _capi.State(0, 0, 0.0, _ptr(bufs[0]).value, _ptr(bufs[1]).value, _ptr(bufs[2]).value, None)
    status = _capi.load().pamc_anneal_static(int(L), _ptr(J), int(R), _ptr(b), nT, int(sweeps),
                                             ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                             ctypes.c_void_p(stream or 0), arr,
                                             ctypes.byref(st_ptr) if st_ptr is not None else None)
    if status not in (_capi.OK, _capi.ERR_CAPACITY, _capi.ERR_EXTINCT):
        raise PamcError(status, "pamc_anneal_static")
    out_state = None
    if st_ptr is not None:
        n = st_ptr.R
        out_state = {"step": st_ptr.step, "R": n, "lnZ": st_ptr.lnZ, "spins": bufs[0][:n], "E": bufs[1][:n],
                     "family": bufs[2][:n]}
    return status, _obs_to_dict(arr), out_state


def calibrate(device: int = -1):
    """(Philox words per ns, int32 VALU operations per ns) of the device's
    calibration kernels (``pamc_calibrate``)."""
    w, v = ctypes.c_double(), ctypes.c_double()
    _check(_capi.load().pamc_calibrate(int(device), ctypes.byref(w), ctypes.byref(v)), "pamc_calibrate")
    return w.value, v.value


def rho_f(betaF, nominal_R):
    """Eq. (4) through ``pamc_rho_f``: betaF [runs][n_temps] of independent
    runs, nominal_R [n_temps]; returns (mean beta F, var beta F with ddof 1,
    rho_f), each [n_temps]."""
    bf = np.ascontiguousarray(betaF, dtype=np.float64)
    runs, nT = bf.shape
    Rn = np.ascontiguousarray(np.broadcast_to(np.asarray(nominal_R, dtype=np.float64), (nT,)))
    mean, var, rf = np.zeros(nT), np.zeros(nT), np.zeros(nT)
    _check(_capi.load().pamc_rho_f(_ptr(bf), runs, nT, _ptr(Rn), _ptr(mean), _ptr(var), _ptr(rf)), "pamc_rho_f")
    return mean, var, rf


def free_energy_variance(L, couplings, R, beta, sweeps, seeds, pop_schedule=None, packed=False, autotune=False,
                         icm_rounds=0, icm_beta_min=0.0):
    """rho_f = R var(beta F) (Sec. II.B, Eq. (4)) from independent runs of one
    instance: the runs (one per seed, at least two; the paper asks for ten or
    more) are annealed together as one batch, and per temperature step the
    library's ``pamc_rho_f`` takes the sample variance (ddof 1) of
    beta F = -ln Z across runs times the nominal population R(beta_k).  Returns a dict of arrays over steps:
    beta, mean_betaF, var_betaF, rho_f, and the per-run beta F [runs, steps]."""
    seeds = [int(x) for x in seeds]
    if len(seeds) < 2:
        raise ValueError("rho_f needs at least two independent runs")
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    inst = [dict(L=L, couplings=couplings, R=R, beta=beta, sweeps=sweeps, seed=sd, pop_schedule=pop_schedule)
            for sd in seeds]
    b = PamcBatch(inst, packed=packed, autotune=autotune, icm_rounds=icm_rounds, icm_beta_min=icm_beta_min)
    try:
        st = b.anneal()
        if st != _capi.OK:
            raise PamcError(st, "free_energy_variance")
        bf = np.stack([b.observables(i)["betaF"] for i in range(len(seeds))])
    finally:
        b.close()
    nominal = np.full(len(beta), float(R)) if pop_schedule is None else np.asarray(pop_schedule, dtype=np.float64)
    mean, var, rf = rho_f(bf, nominal)
    return {"beta": beta, "mean_betaF": mean, "var_betaF": var, "rho_f": rf, "betaF": bf}


class Pamc:
    """One population-annealing run on the GPU (``pamc_create``, or
    ``pamc_create_real`` for int32 real couplings; [2][L^2] couplings select
    the square lattice)."""

    def __init__(self, L, couplings, R, beta, sweeps, seed, capacity=None, overlap_steps=None,
                 fuse_gather=True, torch_stream=True, torch_allocator=False, timing=False, tile_rows=0,
                 graphs=True, group_replicas=0, autotune=False, packed=False, pop_schedule=None, icm_rounds=0,
                 icm_beta_min=0.0):
        lib = _capi.load()
        self.L = int(L)
        self.R = int(R)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        self.nT = len(self.beta)
        self._keep = []
        J, self.real, self.dim = _couplings(self.L, couplings)
        self.N = self.L ** self.dim
        opt = _make_options(capacity, overlap_steps, fuse_gather, dim=self.dim,
                            spin_format=_capi.SPINS_PACKED if packed else _capi.SPINS_INT8, torch_stream=torch_stream,
                            torch_allocator=torch_allocator, keep=self._keep, timing=timing,
                            tile_rows=tile_rows, graphs=graphs, group_replicas=group_replicas,
                            autotune=autotune, pop_schedule=pop_schedule, icm_rounds=icm_rounds,
                            icm_beta_min=icm_beta_min)
        self._opt = opt
        h = ctypes.c_void_p()
        create = lib.pamc_create_real if self.real else lib.pamc_create
        _check(create(self.L, _ptr(J), self.R, _ptr(self.beta), self.nT, int(sweeps),
                      ctypes.c_uint64(int(seed) & (2**64 - 1)), ctypes.byref(opt), ctypes.byref(h)),
               "pamc_create_real" if self.real else "pamc_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _capi.load().pamc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def anneal(self, n_steps: int = -1) -> int:
        """Runs up to n_steps steps; returns the status (raises on device errors)."""
        st = _capi.load().pamc_anneal(self._h, int(n_steps))
        if st not in (_capi.OK, _capi.ERR_CAPACITY, _capi.ERR_EXTINCT):
            raise PamcError(st, "pamc_anneal")
        return st

    def anneal_async(self, n_steps: int = -1):
        _check(_capi.load().pamc_anneal_async(self._h, int(n_steps)), "pamc_anneal_async")

    def sync(self) -> int:
        return _capi.load().pamc_sync(self._h)

    def observables(self) -> dict:
        arr = (_capi.StepObs * self.nT)()
        _check(_capi.load().pamc_observables(self._h, arr, self.nT), "pamc_observables")
        return _obs_to_dict(arr)

    def overlap_hist(self, step: int) -> np.ndarray:
        h = np.zeros(2 * self.N + 1, dtype=np.int64)
        _check(_capi.load().pamc_overlap_hist(self._h, int(step), _ptr(h)), "pamc_overlap_hist")
        return h

    def step_sums(self):
        S = np.zeros(self.nT)
        T = np.zeros(self.nT)
        _check(_capi.load().pamc_step_sums(self._h, _ptr(S), _ptr(T), self.nT), "pamc_step_sums")
        return S, T

    def shape(self):
        k = ctypes.c_int()
        R = ctypes.c_int64()
        _check(_capi.load().pamc_get_shape(self._h, ctypes.byref(k), ctypes.byref(R)), "pamc_get_shape")
        return k.value, R.value

    def sweep_shape(self):
        """(tile_rows, group_replicas) of the sweep workgroups."""
        t = ctypes.c_int()
        g = ctypes.c_int()
        _check(_capi.load().pamc_sweep_shape(self._h, ctypes.byref(t), ctypes.byref(g)), "pamc_sweep_shape")
        return t.value, g.value

    def get_state(self) -> dict:
        """Energies are int32 (+-1 couplings) or int64 in units of 2^-20."""
        k, Rk = self.shape()
        spins = np.zeros((Rk, self.N), dtype=np.int8)
        E = np.zeros(Rk, dtype=np.int64 if self.real else np.int32)
        fam = np.zeros(Rk, dtype=np.uint32)
        st = _state(spins, E, fam, self.real)
        _check(_capi.load().pamc_get_state(self._h, ctypes.byref(st)), "pamc_get_state")
        return {"step": st.step, "R": st.R, "lnZ": st.lnZ, "spins": spins[: st.R], "E": E[: st.R],
                "family": fam[: st.R]}

    def set_state(self, step, spins, family, lnZ):
        spins = np.ascontiguousarray(spins, dtype=np.int8)
        family = np.ascontiguousarray(family, dtype=np.uint32)
        st = _capi.State(int(step), spins.shape[0], float(lnZ), _ptr(spins).value, None, _ptr(family).value, None)
        _check(_capi.load().pamc_set_state(self._h, ctypes.byref(st)), "pamc_set_state")

    def phase_times(self):
        """(sweep ms, resampling ms, stand-alone gather ms, steps) since the
        last call (timing=True)."""
        a, b, g, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(_capi.load().pamc_phase_times(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(g),
                                             ctypes.byref(n)), "pamc_phase_times")
        return a.value, b.value, g.value, n.value

    @property
    def stream_handle(self) -> int:
        return int(self._opt.stream or 0)

    def thresholds(self):
        T = np.zeros((self.nT, 3), dtype=np.uint32)
        acc = np.zeros(self.nT, dtype=np.uint8)
        _check(_capi.load().pamc_thresholds(self._h, _ptr(T), _ptr(acc)), "pamc_thresholds")
        return T, acc


def _state(spins, E, fam, real):
    """A pamc_state over caller buffers: E goes to E_fixed for real couplings."""
    return _capi.State(0, 0, 0.0, _ptr(spins).value, None if real else _ptr(E).value, _ptr(fam).value,
                       _ptr(E).value if real else None)


class PamcBatch:
    """Many independent instances annealed together (``pamc_batch_*``)."""

    def __init__(self, instances, fuse_gather=True, torch_stream=True, graphs=True, autotune=False, packed=False,
                 icm_rounds=0, icm_beta_min=0.0):
        lib = _capi.load()
        self._keep = []
        n = len(instances)
        arr = (_capi.Instance * n)()
        self.nT = []
        self.N = []
        self.real = []
        dims = set()
        for i, d in enumerate(instances):
            L = int(d["L"])
            J, real, dim = _couplings(L, d["couplings"])
            dims.add(dim)
            b = np.ascontiguousarray(d["beta"], dtype=np.float64)
            self._keep += [J, b]
            pop = None
            if d.get("pop_schedule") is not None:
                pop = np.ascontiguousarray(d["pop_schedule"], dtype=np.int64)
                self._keep.append(pop)
            arr[i] = _capi.Instance(L, None if real else _ptr(J).value, int(d["R"]), _ptr(b).value, len(b),
                                    int(d["sweeps"]), int(d["seed"]) & (2**64 - 1),
                                    _ptr(pop).value if pop is not None else None,
                                    _ptr(J).value if real else None)
            self.nT.append(len(b))
            self.N.append(L ** dim)
            self.real.append(real)
        if len(dims) > 1:
            raise ValueError("the instances of a batch share one lattice dimension")
        opt = _make_options(fuse_gather=fuse_gather, torch_stream=torch_stream, keep=self._keep, graphs=graphs,
                            dim=dims.pop(),
                            autotune=autotune, spin_format=_capi.SPINS_PACKED if packed else _capi.SPINS_INT8,
                            icm_rounds=icm_rounds, icm_beta_min=icm_beta_min)
        h = ctypes.c_void_p()
        _check(lib.pamc_batch_create(n, arr, ctypes.byref(opt), ctypes.byref(h)), "pamc_batch_create")
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            _capi.load().pamc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def anneal(self) -> int:
        st = _capi.load().pamc_batch_anneal(self._h)
        if st not in (_capi.OK, _capi.ERR_CAPACITY, _capi.ERR_EXTINCT):
            raise PamcError(st, "pamc_batch_anneal")
        return st

    def observables(self, i: int) -> dict:
        arr = (_capi.StepObs * self.nT[i])()
        _check(_capi.load().pamc_batch_observables(self._h, int(i), arr, self.nT[i]), "pamc_batch_observables")
        return _obs_to_dict(arr)

    def get_state(self, i: int) -> dict:
        k = ctypes.c_int()
        R = ctypes.c_int64()
        _check(_capi.load().pamc_batch_shape(self._h, int(i), ctypes.byref(k), ctypes.byref(R)), "shape")
        N = self.N[i]
        spins = np.zeros((R.value, N), dtype=np.int8)
        E = np.zeros(R.value, dtype=np.int64 if self.real[i] else np.int32)
        fam = np.zeros(R.value, dtype=np.uint32)
        st = _state(spins, E, fam, self.real[i])
        _check(_capi.load().pamc_batch_get_state(self._h, int(i), ctypes.byref(st)), "pamc_batch_get_state")
        return {"step": st.step, "R": st.R, "lnZ": st.lnZ, "spins": spins, "E": E, "family": fam}


class PamcServer:
    """Request loop with continuous batching under an HBM budget."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 256, autotune: bool = False, packed: bool = False):
        lib = _capi.load()
        opt = _capi.ServerOptions(int(max_active), -1, 1 if autotune else 0,
                                  _capi.SPINS_PACKED if packed else _capi.SPINS_INT8)
        h = ctypes.c_void_p()
        _check(lib.pamc_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), ctypes.byref(opt),
                                      ctypes.byref(h)), "pamc_server_create")
        self._h = h
        self._keep = {}
        self._nT = {}

    def submit(self, L, couplings, R, beta, sweeps, seed, pop_schedule=None) -> int:
        L = int(L)
        J, real, dim = _couplings(L, couplings)
        if dim != 3:
            raise ValueError("the serving API runs cubic lattices only")
        b = np.ascontiguousarray(beta, dtype=np.float64)
        pop = None if pop_schedule is None else np.ascontiguousarray(pop_schedule, dtype=np.int64)
        inst = _capi.Instance(L, None if real else _ptr(J).value, int(R), _ptr(b).value, len(b), int(sweeps),
                              int(seed) & (2**64 - 1), _ptr(pop).value if pop is not None else None,
                              _ptr(J).value if real else None)
        rid = ctypes.c_uint64()
        _check(_capi.load().pamc_server_submit(self._h, ctypes.byref(inst), ctypes.byref(rid)), "submit")
        self._nT[rid.value] = len(b)
        return rid.value

    def poll(self, rid: int):
        """None while running; else (status, observables dict, times)."""
        nT = self._nT[rid]
        arr = (_capi.StepObs * nT)()
        res = _capi.Result(0, nT, ctypes.cast(arr, ctypes.POINTER(_capi.StepObs)), 0.0, 0.0, 0.0)
        st = _capi.load().pamc_server_poll(self._h, ctypes.c_uint64(rid), ctypes.byref(res))
        if st == _capi.ERR_BUSY:
            return None
        _check(st, "poll")
        times = {"submit": res.submit_time_s, "admit": res.admit_time_s, "finish": res.finish_time_s}
        return res.status, _obs_to_dict(arr), times

    def wait(self, rid: int, timeout: float = 600.0, interval: float = 0.002):
        t0 = time.time()
        while True:
            r = self.poll(rid)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"request {rid} not finished")
            time.sleep(interval)

    def cancel(self, rid: int) -> int:
        return _capi.load().pamc_server_cancel(self._h, ctypes.c_uint64(rid))

    def stats(self):
        c, q, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        st = _capi.load().pamc_server_stats(self._h, ctypes.byref(c), ctypes.byref(q), ctypes.byref(a))
        return {"status": st, "completed": c.value, "queued": q.value, "active": a.value}

    def usage(self):
        """Budget held by admitted requests, the budget, device busy time
        and wall time since creation (``pamc_server_usage``)."""
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        busy, wall = ctypes.c_double(), ctypes.c_double()
        st = _capi.load().pamc_server_usage(self._h, ctypes.byref(u), ctypes.byref(b), ctypes.byref(busy),
                                            ctypes.byref(wall))
        return {"status": st, "used_bytes": u.value, "budget_bytes": b.value, "busy_s": busy.value,
                "wall_s": wall.value}

    def close(self):
        if getattr(self, "_h", None):
            _capi.load().pamc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
