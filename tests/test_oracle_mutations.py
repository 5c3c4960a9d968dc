"""Mutation check of the oracle's pins: each plausible mistake, planted in a
copy of the oracle's C source (a dropped term, a flipped sign, a wrong
index, a wrong normalisation target, a wrong weight, a wrong family term,
an improper colouring, a dropped copy), is built into a separate library,
and the oracle's pin tests are run against it; at least one must fail.  The
unmodified oracle passes the same tests in the main suite (CPU, slow)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pamc_oracle.c")
ENUM = os.path.join(ROOT, "oracle", "enumerate.c")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_pins.py", "test_oracle_real.py", "test_oracle_icm.py", "test_oracle_2d.py")]

pytestmark = pytest.mark.slow

# name -> (text in the oracle, planted replacement)
MUTATIONS = {
    # Eq. (1) without the z bonds
    "energy_drops_a_term": ("for (int d = 0; d < o->dim; ++d) e -= coupling(o, d, s)",
                            "for (int d = 0; d < o->dim - 1; ++d) e -= coupling(o, d, s)"),
    # Metropolis with the sign of dE flipped
    "dE_sign": ("int64_t dE = 2 * S[s] * h;", "int64_t dE = -2 * S[s] * h;"),
    # the bond to the -x neighbour read at the site instead of the neighbour
    "coupling_index": ("jn[1] = o->J[0 * N + xm];", "jn[1] = o->J[0 * N + s];"),
    # copies normalised to the current population instead of the nominal one
    "normalisation_target": ("double tau = ((double)o->Rt[k + 1] * w[m]) / S;",
                             "double tau = ((double)o->Rk * w[m]) / S;"),
    # level weights exp(-dbeta m) instead of exp(-2 dbeta m)
    "weight_ratio": ("double rho = exp(-2.0 * dbeta);", "double rho = exp(-1.0 * dbeta);"),
    # the threshold of another dE
    "threshold_index": ("u < T[dE / 4 - 1]", "u < T[(dE / 4) % 3]"),
    # free-energy perturbation with the sign of the E_min shift flipped
    "lnQ_sign": ("double lnQ = (-dbeta * (double)Emin) + log(S) - log((double)o->Rk);",
                 "double lnQ = (dbeta * (double)Emin) + log(S) - log((double)o->Rk);"),
    # family term n ln n replaced by n ln(n + 1)
    "family_term": ("leaf[f] = cnt[f] > 0 ? (double)cnt[f] * log((double)cnt[f]) : 0.0;",
                    "leaf[f] = cnt[f] > 0 ? (double)cnt[f] * log((double)cnt[f] + 1.0) : 0.0;"),
    # odd L coloured like even L (not a proper colouring of the periodic lattice)
    "colouring": ("int gx = (x == L - 1) ? 2 : x % 2;", "int gx = x % 2;"),
    # nearest-integer resampling without the extra copy
    "resample_floor_only": ("o->ncopy[r] = B[m] + (u < F[m] ? 1u : 0u);", "o->ncopy[r] = B[m];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_oracle_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site of {name} not found once"
    mutant = tmp_path / "pamc_oracle.c"
    mutant.write_text(text.replace(old, new))
    lib = str(tmp_path / "liboracle_mutant.so")
    r = subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                        "-shared", str(mutant), ENUM, "-o", lib, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, PAMC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow"], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=900)
    assert r.returncode == 1, f"no pin failed with mutation {name}:\n{r.stdout[-1500:]}"
