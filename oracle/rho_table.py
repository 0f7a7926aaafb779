"""Speed ratio of Section 5 (eq. 5.1) on the host: seconds per CP_ALS sweep
with the gradients by their definition (Algorithm 1: explicit unfoldings and
Khatri-Rao products, ``cp_oracle.als_sweep``) over seconds per fast sweep
(Algorithm 2 with the updates of Section 4, ``alg2_host.als_sweep_fast``), on
random tensors of the shapes of Table 5.1 and the 7-D example of Section 5.
Test infrastructure (float64 NumPy on the host's cores; nothing here runs on
the GPU).  Run from the repository root:
    python -m oracle.rho_table [--quick]
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import alg2_host as H
from . import cp_oracle as O

TABLE_5_1 = [(5, 20, (1, 10, 20)), (5, 30, (1, 10, 20, 30)), (5, 40, (1, 10, 20, 30, 40)), (6, 20, (1, 10, 20))]
EXTRA_7D = [(7, 10, (10,))]
QUICK = [(4, 24, (10,)), (5, 14, (1, 10)), (6, 9, (10,)), (7, 7, (10,))]


def sweep_seconds(fn, Y, A, reps):
    fn(Y, A)   # warm-up (allocations, BLAS threads)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn(Y, A)
    return (time.perf_counter() - t0) / reps


def rho(N, I, R, reps=2, seed=0):
    g = np.random.default_rng([1204, 1586, 51, N, I, R, seed])
    Y = g.standard_normal((I,) * N)
    Y = np.asfortranarray(Y)
    A = [g.standard_normal((I, R)) for _ in range(N)]
    t1 = sweep_seconds(lambda y, a: O.als_sweep(y, a), Y, A, reps)
    t2 = sweep_seconds(lambda y, a: H.als_sweep_fast(y, a), Y, A, reps)
    return t1, t2, t1 / t2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    rows = QUICK if args.quick else TABLE_5_1 + EXTRA_7D
    print(f"host: {os.cpu_count()} logical CPUs")
    print("| N | I | R | s/sweep, Algorithm 1 | s/sweep, fast (Alg. 2 + Section 4) | rho |")
    print("|---|---|---|---|---|---|")
    for N, I, Rs in rows:
        for R in Rs:
            t1, t2, r = rho(N, I, R)
            print(f"| {N} | {I} | {R} | {t1:.3g} | {t2:.3g} | {r:.1f} |", flush=True)


if __name__ == "__main__":
    main()
