"""CPU oracle for the fast CP gradient and CP_ALS — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct float64 NumPy implementation of what the
device library computes, written from the paper's definitions.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
library never does, and this package imports nothing from the library.

Functions whose result has a plain definition compute that definition
(explicit unfoldings, explicit Khatri-Rao products, one GEMM per mode), not the
paper's fast algorithm.  See ``cp_oracle`` and ``mlp_oracle``.
"""
from .cp_oracle import *  # noqa: F401,F403
