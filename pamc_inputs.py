"""Seeded synthetic inputs for population annealing runs.

This module holds no part of the method's arithmetic: it only draws problem
instances (couplings), builds temperature schedules and the workload
descriptions, so that the GPU library, the oracle, the tests and the
benchmark all see the same inputs.  The paper's own disorder instances are not
published; +-J couplings with probability 1/2 each (from the Philox stream
that the library's pamc_make_pm_j also draws), or Gaussian couplings in
fixed point from a seeded generator, stand in for them.
"""
from __future__ import annotations

import numpy as np


_M32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counters: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) of every row of
    counters (uint32 [n][4]) under the key (low, high 32 bits of seed):
    ten rounds, each multiplying words 0 and 2 by the round multipliers
    (full 64-bit products), the high halves mixed with words 1 and 3 and the
    round key by XOR; the key advances by the Weyl constants.  uint32 [n][4].
    Used here only to draw +-J instances."""
    c = np.asarray(counters, dtype=np.uint64).reshape(-1, 4).copy()
    k0 = np.uint64(int(seed) & 0xFFFFFFFF)
    k1 = np.uint64((int(seed) >> 32) & 0xFFFFFFFF)
    for _ in range(10):
        a = np.uint64(0xD2511F53) * c[:, 0]
        b = np.uint64(0xCD9E8D57) * c[:, 2]
        n = np.empty_like(c)
        n[:, 0] = (b >> np.uint64(32)) ^ c[:, 1] ^ k0
        n[:, 1] = b & _M32
        n[:, 2] = (a >> np.uint64(32)) ^ c[:, 3] ^ k1
        n[:, 3] = a & _M32
        c = n
        k0 = (k0 + np.uint64(0x9E3779B9)) & _M32
        k1 = (k1 + np.uint64(0xBB67AE85)) & _M32
    return c.astype(np.uint32)


# counter word 3 of the coupling draws (the library's pamc_make_pm_j draws
# the same stream)
COUPLING_TAG = 0x50000000


def pm_j_couplings(L: int, disorder_seed: int) -> np.ndarray:
    """+-J couplings, int8 [3][L^3]: J[d][s] couples site s to s + e_d.
    Bond b = d L^3 + s is +1 when bit 31 of word (b & 3) of Philox4x32-10 at
    counter (b >> 2, 0, 0, COUPLING_TAG), keyed by the disorder seed, is set,
    else -1, so a C caller gets the same instance from pamc_make_pm_j."""
    N = L ** 3
    nblk = (3 * N + 3) // 4
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 3] = COUPLING_TAG
    words = philox4x32_10(ctr, disorder_seed).reshape(-1)[: 3 * N]
    return np.where(words >> np.uint32(31), 1, -1).astype(np.int8).reshape(3, N)


# Real couplings are carried in fixed point, J = j 2^-20 with int32 j and
# |J| < 8, so that energies are exact integers (units of 2^-20).
REAL_SCALE_BITS = 20
REAL_LIMIT = (1 << 23) - 1


def gaussian_couplings(L: int, disorder_seed: int, dim: int = 3) -> np.ndarray:
    """Gaussian couplings (mean 0, variance 1; the paper's case study,
    Sec. II.A) rounded to the fixed-point grid, int32 [D][L^D] of j with
    J = j 2^-20 on the cubic (D = 3) or square (D = 2) lattice; the rare
    draws with |J| >= 8 are clipped."""
    N = L ** dim
    rng = np.random.Generator(np.random.PCG64(np.uint64(disorder_seed)))
    g = rng.standard_normal(size=(dim, N))
    j = np.rint(g * float(1 << REAL_SCALE_BITS))
    return np.clip(j, -REAL_LIMIT, REAL_LIMIT).astype(np.int32)


def ferro_couplings(L: int) -> np.ndarray:
    return np.ones((3, L ** 3), dtype=np.int8)


def mattis_couplings(L: int, seed: int):
    """Mattis instance J_ij = eps_i eps_j: ground state energy exactly -3N."""
    N = L ** 3
    rng = np.random.Generator(np.random.PCG64(np.uint64(seed)))
    eps = (2 * rng.integers(0, 2, size=N) - 1).astype(np.int8)
    J = np.empty((3, N), dtype=np.int8)
    idx = np.arange(N)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    nb = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z),
          x + L * (y + L * ((z + 1) % L))]
    for d in range(3):
        J[d] = eps * eps[nb[d]]
    return J, eps


def square_neighbours(L: int):
    """+x and +y neighbours of every site of the periodic L x L lattice,
    site s = x + L y."""
    idx = np.arange(L * L)
    x, y = idx % L, idx // L
    return [((x + 1) % L) + L * y, x + L * ((y + 1) % L)]


def pm_couplings_as_real(couplings: np.ndarray) -> np.ndarray:
    """+-1 couplings as fixed-point real couplings (J = j 2^-20, exact)."""
    return np.asarray(couplings).astype(np.int32) * np.int32(1 << REAL_SCALE_BITS)


def pm_j_couplings_2d(L: int, disorder_seed: int) -> np.ndarray:
    """Random +-1 couplings on the periodic square lattice as fixed-point
    real couplings, int32 [2][L^2]."""
    rng = np.random.Generator(np.random.PCG64(np.uint64(disorder_seed)))
    return pm_couplings_as_real(2 * rng.integers(0, 2, size=(2, L * L)) - 1)


def gauge_transform(L: int, couplings: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """J_ij -> eps_i J_ij eps_j for a +-1 vector eps over the sites (cubic
    [3][L^3] or square [2][L^2] couplings)."""
    dim = 3 if np.asarray(couplings).size == 3 * L ** 3 else 2
    N = L ** dim
    idx = np.arange(N)
    if dim == 3:
        x, y, z = idx % L, (idx // L) % L, idx // (L * L)
        nb = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z),
              x + L * (y + L * ((z + 1) % L))]
    else:
        nb = square_neighbours(L)
    dt = np.int32 if np.asarray(couplings).dtype == np.int32 else np.int8
    J = np.array(couplings, dtype=dt).reshape(dim, N).copy()
    for d in range(dim):
        J[d] = (eps.astype(np.int64) * J[d] * eps[nb[d]]).astype(dt)
    return J


def linear_beta(beta_max: float, n_temps: int) -> np.ndarray:
    """Linear-in-beta schedule beta_k = beta_max k / (n_temps - 1)."""
    if n_temps == 1:
        return np.zeros(1)
    return np.array([beta_max * k / (n_temps - 1) for k in range(n_temps)], dtype=np.float64)


def lblt_beta(beta_max: float, n_temps: int, T_N: float = 1.0) -> np.ndarray:
    """Linear-in-beta linear-in-T schedule (Sec. III.B): the first half of
    the temperatures, from beta = 0 down to T_N, equally spaced in beta, the
    second half from T_N to T_min = 1/beta_max equally spaced in T.  The two
    halves meet at step k_N = (n_temps - 1) // 2 with beta = 1/T_N (3D
    optimum T_N = 1.0, Fig. 3(d)); requires T_N > 1/beta_max."""
    if n_temps < 3:
        return linear_beta(beta_max, n_temps)
    kN = (n_temps - 1) // 2
    bN, Tmin = 1.0 / T_N, 1.0 / beta_max
    if not bN < beta_max:
        raise ValueError("T_N must lie above 1/beta_max")
    beta = np.empty(n_temps)
    for k in range(kN + 1):
        beta[k] = bN * k / kN
    n2 = n_temps - 1 - kN
    for j in range(1, n2 + 1):
        beta[kN + j] = 1.0 / (T_N + (Tmin - T_N) * j / n2)
    return beta


def tspl_beta(beta_max: float, n_temps: int, alpha1: float = float(np.exp(-0.0734)),
              alpha2: float = float(np.exp(2.15)), beta0: float = 1.63) -> np.ndarray:
    """Two-stage power-law schedule, Eq. (5): beta(tau) = a tau^alpha1 below
    tau_0 and b tau^alpha2 above, tau = k / (n_temps - 1).  b = beta_max
    fixes the final temperature, tau_0 = (beta0 / beta_max)^(1/alpha2) puts
    the switch-over at beta0, a = beta0 / tau_0^alpha1 makes it continuous.
    Defaults are the paper's parameters for 3D."""
    if n_temps == 1:
        return np.zeros(1)
    tau0 = (beta0 / beta_max) ** (1.0 / alpha2)
    a = beta0 / tau0 ** alpha1
    tau = np.arange(n_temps, dtype=np.float64) / (n_temps - 1)
    return np.where(tau < tau0, a * tau ** alpha1, beta_max * tau ** alpha2)


def clipped_exponential_population(beta: np.ndarray, R_mean: int, beta0: float = 0.9, r: float = 33.8,
                                   S: float = float(np.exp(-2.52))) -> np.ndarray:
    """Nominal population R(beta_k) of the clipped exponential schedule,
    Eq. (6): R_0 up to beta0, then falling to R_0 / r at beta_max with
    slope S (the paper's 3D parameters by default).  R_0 is scaled so that
    the mean over the steps is R_mean (comparable to a uniform run); the
    entries are rounded to integers >= 1."""
    beta = np.asarray(beta, dtype=np.float64)
    bmax = beta[-1]
    a = np.exp(bmax * S) - np.exp(beta0 * S)
    f = np.where(beta <= beta0, 1.0, a / ((r - 1.0) * (np.exp(beta * S) - np.exp(beta0 * S)) + a))
    R0 = R_mean * len(beta) / f.sum()
    return np.maximum(1, np.rint(R0 * f)).astype(np.int64)


def random_spins(R: int, N: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.uint64(seed)))
    return (2 * rng.integers(0, 2, size=(R, N), dtype=np.int8) - 1).astype(np.int8)


# Workloads (3D +-J Edwards-Anderson, periodic boundaries, N_S = 10 sweeps).
WORKLOADS = {
    "L4_R1000": dict(L=4, R=1000, n_temps=101, beta_max=5.0, sweeps=10, disorder_seed=1, seed=1),
    "L8_R100000": dict(L=8, R=100_000, n_temps=201, beta_max=5.0, sweeps=10, disorder_seed=2,
                       seed=2),
    "L16_R500000": dict(L=16, R=500_000, n_temps=301, beta_max=5.0, sweeps=10, disorder_seed=3,
                        seed=3),
    # the square lattice at the largest size of the paper's cluster-update
    # runs (L = 32, R = 10^6, 301 temperatures, T_min = 0.2), Gaussian
    # couplings
    "L32_2D_R1000000": dict(L=32, R=1_000_000, n_temps=301, beta_max=5.0, sweeps=10, disorder_seed=6,
                            seed=6, dim=2),
}


def batch_instances(n: int, sizes=(4, 6, 8, 10, 12), R: int = 20_000, n_temps: int = 201,
                    sweeps: int = 10, shuffle_seed: int = 4):
    """Mixed-size instance list: n/len(sizes) instances of each L, shuffled."""
    per = n // len(sizes)
    Ls = np.repeat(np.array(sizes), per)
    Ls = np.concatenate([Ls, np.array(sizes[: n - len(Ls)], dtype=Ls.dtype)])
    rng = np.random.Generator(np.random.PCG64(np.uint64(shuffle_seed)))
    rng.shuffle(Ls)
    out = []
    for i, L in enumerate(Ls):
        out.append(dict(L=int(L), couplings=pm_j_couplings(int(L), 1_000_000 + i), R=R,
                        beta=linear_beta(5.0, n_temps), sweeps=sweeps, seed=2_000_000 + i))
    return out


def serving_requests(n: int, rate: float = 50.0, seed: int = 5, Lmin: int = 4, Lmax: int = 14,
                     Rmin: int = 5000, Rmax: int = 50000, n_temps: int = 101, sweeps: int = 10):
    """Poisson arrivals (exponential gaps) of random instances."""
    rng = np.random.Generator(np.random.PCG64(np.uint64(seed)))
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        L = int(rng.integers(Lmin, Lmax + 1))
        R = int(rng.integers(Rmin, Rmax + 1))
        out.append(dict(arrival=float(t[i]), L=L, couplings=pm_j_couplings(L, 3_000_000 + i), R=R,
                        beta=linear_beta(5.0, n_temps), sweeps=sweeps, seed=4_000_000 + i))
    return out
