"""Measures the sweep workgroup shapes of the common run sizes on this GPU
and writes them to a tuning cache file, by default ``tune_cache.jsonl``
beside the library, which every process reads at start-up: runs of those
sizes then start without the autotuner's trial launches.

    python -m paper_1710_09025_amd.make_tune_cache [--out FILE]

A choice is keyed by device (architecture and compute units), sweep kernel,
lattice (dimension, L), sweeps per step, capacity class (the population
capacity rounded up to a power of two) and spin format; any size not listed
here is still tuned on first use.  Every shape gives bit-identical results,
so the file only affects speed.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

# single runs of the request sizes of the serving mix: every L of 4 .. 14
# over a grid of populations covering the capacity classes of 5e3 .. 5e4 rows
SERVING_L = range(4, 15)
SERVING_R = (5000, 8000, 12000, 16000, 24000, 32000, 40000, 50000)

# (L, R, sweeps, packed, real couplings, dimension)
NAMED = [
    (4, 1000, 10, False, False, 3),        # the small single-instance run
    (8, 100_000, 10, False, False, 3),     # L = 8, R = 10^5
    (8, 100_000, 10, False, True, 3),      # the same with Gaussian couplings
    (16, 500_000, 10, False, False, 3),    # L = 16, R = 5 10^5, one byte per spin
    (16, 500_000, 10, True, False, 3),     # the same, one bit per spin
    (32, 1_000_000, 10, False, True, 2),   # square lattice, L = 32, R = 10^6
] + [(L, 20_000, 10, False, False, 3) for L in (4, 6, 8, 10, 12)] \
  + [(L, 200_000, 10, False, False, 3) for L in range(4, 15)] \
  + [(L, 100_000, 10, False, False, 3) for L in range(4, 15)]


def main(argv=None) -> int:
    here = os.path.dirname(os.path.abspath(__file__))
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(here, "tune_cache.jsonl"))
    args = ap.parse_args(argv)
    out = os.path.abspath(args.out)
    # start from an empty file: the library also reads the file beside it,
    # and a choice it finds there is not measured again
    beside = os.path.join(here, "tune_cache.jsonl")
    for path in {out, beside}:
        if os.path.exists(path):
            os.remove(path)
    os.environ["PAMC_TUNE_CACHE"] = out  # new choices are appended here
    from paper_1710_09025_amd import autotune

    t0 = time.perf_counter()
    jobs = [(L, R, 10, False, False, 3) for L in SERVING_L for R in SERVING_R] + NAMED
    for i, (L, R, sweeps, packed, real, dim) in enumerate(jobs):
        tr, gr, ns = autotune(L, R, sweeps, torch_stream=False, packed=packed, real=real, dim=dim)
        print(f"[{i + 1}/{len(jobs)}] L={L} R={R} dim={dim} packed={int(packed)} real={int(real)}: "
              f"tile_rows={tr} group_replicas={gr} {ns * 1e3:.3f} ps/attempt", flush=True)
    with open(out) as f:
        n = sum(1 for line in f if line.strip())
    print(f"{n} choices in {out} ({time.perf_counter() - t0:.1f} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
