"""Writes thresholds.txt: Metropolis thresholds floor(e^{-beta dE} 2^32) for
dE = 4, 8, 12 (acceptance min(1, e^{-beta dE}), Sec. II.B of the paper),
evaluated with 60-digit decimal arithmetic, independent of any libm."""
from decimal import Decimal, getcontext
import os

getcontext().prec = 60
BETAS = ["5", "1", "0.5", "0.25", "0.05", "2.7", "2.8", "3", "0.001"]
lines = ["# Metropolis acceptance min(1, exp(-beta dE)) of Sec. II.B as uint32 thresholds",
         "# written by make_thresholds.py with 60-digit decimal arithmetic",
         "# beta  T(dE=4)  T(dE=8)  T(dE=12)  accept_all",
         "# floor(exp(-beta dE) * 2^32), capped at 2^32 - 1; beta = 0 accepts every move",
         "0 0 0 0 1"]
for b in BETAS:
    row = []
    for dE in (4, 8, 12):
        x = (-(Decimal(b) * dE)).exp() * (2 ** 32)
        t = int(x)  # floor for positive x
        frac = x - t
        # a double evaluation is off by ~1e-16 x: the floor must not be that close
        margin = x * Decimal("1e-12")
        assert t == 0 or (margin < frac < 1 - margin), "too close to an integer"
        row.append(str(min(t, 2 ** 32 - 1)))
    lines.append(f"{b} {' '.join(row)} 0")
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "thresholds.txt"), "w") as f:
    f.write("\n".join(lines) + "\n")
