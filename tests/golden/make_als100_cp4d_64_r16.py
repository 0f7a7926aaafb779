"""Writes als100_cp4d_64_r16.json: the float64 oracle's CP_ALS run (eq. 2.14 in
the Section 4 order, cost by eq. 2.12) over 100 sweeps on the 64x64x64x64,
rank-16, 20 dB float32 workload (rep 0), started from the float32 initial
factors that the device receives.  Calls only the oracle and the seeded input
generator.  Run from the repository root:
    python tests/golden/make_als100_cp4d_64_r16.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cpgen  # noqa: E402
import oracle as O  # noqa: E402

SWEEPS = 100


def main():
    pr = cpgen.make_problem("cp4d_64_r16_f32", rep=0)
    dims = pr["dims"]
    Y = O.as_tensor(cpgen.storage_to_f64(pr["y"], pr["storage"]), dims)
    A = [np.asarray(M, dtype=np.float32).astype(np.float64) for M in pr["init"]]
    normY2 = O.norm2(Y)
    fits, costs = [], []
    for s in range(SWEEPS):
        A, D, f = O.als_sweep(Y, A, normY2=normY2)
        fits.append(f)
        costs.append(D)
        print(s, f, flush=True)
    out = {"description": "float64 oracle CP_ALS on workload cp4d_64_r16_f32 rep 0 (64^4, R=16, 20 dB, float32 "
                          "storage), 100 sweeps in the Section 4 order from the float32-rounded initial factors; "
                          "fit = 1 - sqrt(D)/||Y|| with D from eq. 2.12",
           "workload": "cp4d_64_r16_f32", "rep": 0, "sweeps": SWEEPS, "normY2": normY2,
           "fits": fits, "costs": costs,
           "final_factor_norms": [float(np.linalg.norm(M)) for M in A]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "als100_cp4d_64_r16.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
