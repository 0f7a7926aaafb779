"""Seeded synthetic inputs for the CP-gradient and CP_ALS workloads.

This module serves both sides of every check: the CPU oracle under ``oracle/``
and the device library under ``paper_1204_1586_amd/``.  It only draws random
numbers and assembles the input tensor from them; it computes none of the
gradients, factor updates, Gram matrices or costs that the two sides compute,
and it imports neither side.

Conventions (Section 2 of the paper, eq. 2.1):

* a tensor of size I_1 x ... x I_N is handed over as ``vec(Y)``, a flat array
  whose first mode varies fastest (column-major, the ``ivec`` order);
* a factor A^(n) is an I_n x R array;
* every random stream is keyed by ``SeedSequence([1204, 1586, workload, rep,
  stream])`` with stream 0 = true factors, 1 = noise, 2 = initial factors,
  3 = auxiliary draws (the rank of the learned-step tensors).

The CP model itself (Def. 2.4, eq. 2.7) is assembled here with a private
Khatri-Rao helper; the oracle has its own, written separately.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = (1204, 1586)

STREAM_TRUE = 0
STREAM_NOISE = 1
STREAM_INIT = 2
STREAM_AUX = 3


def rng(workload_id: int, rep: int, stream: int) -> np.random.Generator:
    """Independent, reproducible generator for one (workload, rep, stream)."""
    return np.random.default_rng(np.random.SeedSequence([*SEED_BASE, workload_id, rep, stream]))


# ----------------------------------------------------------------------------
# factors
# ----------------------------------------------------------------------------

def gaussian_factors(dims, R, g: np.random.Generator):
    """Factors with i.i.d. N(0,1) entries, one I_n x R float64 array per mode."""
    return [g.standard_normal((int(I), int(R))) for I in dims]


def congruent_factors(dims, R, c, g: np.random.Generator):
    """Factors whose columns have pairwise cosine exactly ``c`` in every mode.

    A^(n) = sqrt(I_n) * Q_n * chol(C)^T with C = (1-c) I + c 11^T and Q_n the
    orthonormal columns of the QR factorisation of an I_n x R Gaussian matrix,
    so that A^(n)^T A^(n) = I_n * C.  Needs I_n >= R.
    """
    R = int(R)
    C = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
    Lc = np.linalg.cholesky(C)
    out = []
    for I in dims:
        if I < R:
            raise ValueError("congruent factors need I_n >= R")
        Q, _ = np.linalg.qr(g.standard_normal((int(I), R)))
        out.append(math.sqrt(I) * Q @ Lc.T)
    return out


# ----------------------------------------------------------------------------
# tensor assembly
# ----------------------------------------------------------------------------

def _kr_rows(mats):
    """Khatri-Rao product of ``mats`` = [M_a, ..., M_b] with the FIRST matrix's
    row index varying fastest: row index = i_a + I_a*(i_{a+1} + ...)."""
    out = np.ones((1, mats[0].shape[1]))
    for M in mats:
        # new row = i_prev + rows(out) * i_M  (previous modes stay fastest)
        out = (M[:, None, :] * out[None, :, :]).reshape(-1, M.shape[1])
    return out


def cp_full(factors, split=None, col_lo=0, col_hi=None):
    """Columns [col_lo, col_hi) of the (I_1..I_s) x (I_{s+1}..I_N) matrix view of
    the CP tensor sum_r a_r^(1) o ... o a_r^(N), as a float64 array."""
    N = len(factors)
    s = split if split is not None else max(1, N // 2)
    left = _kr_rows(factors[:s])
    right = _kr_rows(factors[s:])
    if col_hi is None:
        col_hi = right.shape[0]
    return left @ right[col_lo:col_hi].T


def to_bf16_bits(x) -> np.ndarray:
    """Round float values to bfloat16 (round to nearest even); returns uint16 bits."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    bias = np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    return ((u + bias) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f64(b) -> np.ndarray:
    """Exact value of stored bfloat16 bits, as float64."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def noisy_cp_tensor(factors, snr_db, g_noise: np.random.Generator, storage="f64", chunk_cols=4096):
    """vec(Y) for Y = [[A^(1..N)]] + E, E i.i.d. N(0, s^2),
    s^2 = ||Yhat||^2 / (J_N * 10^(snr_db/10)); snr_db=None means no noise.

    The clean tensor is built and the noise added in float64 column chunks of
    the (I_1..I_s) x (I_{s+1}..I_N) view, then cast to the storage type:
    'f64', 'f32', 'f16' (round to nearest even) or 'bf16' (uint16 bit
    patterns, round to nearest even).
    """
    dims = [A.shape[0] for A in factors]
    N = len(dims)
    s = max(1, N // 2)
    J = int(np.prod(dims[:s]))
    K = int(np.prod(dims[s:]))
    dt = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16, "f16": np.float16}[storage]
    out = np.empty(J * K, dtype=dt)
    # pass 1: norm of the clean tensor (the chunks are rebuilt in pass 2)
    nrm2 = 0.0
    if snr_db is not None:
        for c0 in range(0, K, chunk_cols):
            blk = cp_full(factors, s, c0, min(K, c0 + chunk_cols))
            nrm2 += float(np.sum(blk * blk))
        sigma = math.sqrt(nrm2 / (J * K * 10.0 ** (snr_db / 10.0)))
    for c0 in range(0, K, chunk_cols):
        c1 = min(K, c0 + chunk_cols)
        blk = cp_full(factors, s, c0, c1)
        if snr_db is not None:
            blk = blk + sigma * g_noise.standard_normal(blk.shape)
        flat = blk.reshape(-1, order="F")
        if storage == "bf16":
            out[c0 * J:c1 * J] = to_bf16_bits(flat)
        else:
            out[c0 * J:c1 * J] = flat.astype(dt)
    return out


def storage_to_f64(y, storage) -> np.ndarray:
    """The exact values held in a storage array, as float64."""
    if storage == "bf16":
        return bf16_bits_to_f64(y)
    return np.asarray(y, dtype=np.float64)


# ----------------------------------------------------------------------------
# the paper-shaped workloads
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    """A synthetic CP problem: tensor shape, rank, noise, storage and factor law."""
    workload_id: int
    name: str
    dims: tuple
    rank: object          # int, or (lo, hi) for a rank drawn uniformly per rep
    snr_db: float
    storage: str          # 'f64' | 'f32' | 'bf16'
    congruence: float = None
    sweeps: int = 0
    notes: str = field(default="", compare=False)


WORKLOADS = {
    "cp3d_20_r3_f64": Workload(1, "cp3d_20_r3_f64", (20, 20, 20), 3, 30.0, "f64", None, 50,
                               "3-D 20^3, rank 3, FP64, 30 dB; all-mode gradient + 50 ALS sweeps"),
    "cp4d_64_r16_f32": Workload(2, "cp4d_64_r16_f32", (64, 64, 64, 64), 16, 20.0, "f32", None, 100,
                                "4-D 64^4, rank 16, FP32, 20 dB; all-mode gradient + 100 ALS sweeps"),
    "cp7d_10_r10_f32": Workload(3, "cp7d_10_r10_f32", (10,) * 7, 10, 20.0, "f32", None, 0,
                                "7-D 10^7, rank 10, FP32 storage; FP32 vs BF16-refined contraction"),
    "cp5d_48_r32_bf16": Workload(4, "cp5d_48_r32_bf16", (48,) * 5, 32, 25.0, "bf16", 0.5, 0,
                                 "5-D 48^5 stored BF16, rank 32, congruence 0.5, 25 dB; ALS to fit 1e-6"),
    "cp4d_40x70_learned": Workload(5, "cp4d_40x70_learned", (40, 50, 60, 70), (8, 20), 30.0, "f32", 0.9, 0,
                                   "4-D 40x50x60x70, rank U{8..20}, congruence 0.9, 30 dB; learned-step ALS"),
}


def workload_rank(w: Workload, rep: int) -> int:
    if isinstance(w.rank, tuple):
        lo, hi = w.rank
        return int(rng(w.workload_id, rep, STREAM_AUX).integers(lo, hi + 1))
    return int(w.rank)


def make_problem(w, rep=0, dims=None, rank=None, snr_db="default", storage=None):
    """Build one seeded problem.

    Returns a dict with ``dims``, ``R``, ``storage``, ``y`` (vec(Y) in its
    storage type), ``truth`` (true factors, float64) and ``init`` (initial
    factors, i.i.d. N(0,1), float64).  ``dims``/``rank``/``snr_db``/``storage``
    override the workload's values (used for small versions of a workload).
    """
    if isinstance(w, str):
        w = WORKLOADS[w]
    dims = tuple(int(d) for d in (dims if dims is not None else w.dims))
    R = int(rank) if rank is not None else workload_rank(w, rep)
    snr = w.snr_db if snr_db == "default" else snr_db
    st = storage or w.storage
    g_true = rng(w.workload_id, rep, STREAM_TRUE)
    if w.congruence is not None and min(dims) >= R:
        truth = congruent_factors(dims, R, w.congruence, g_true)
    else:
        truth = gaussian_factors(dims, R, g_true)
    y = noisy_cp_tensor(truth, snr, rng(w.workload_id, rep, STREAM_NOISE), st)
    init = gaussian_factors(dims, R, rng(w.workload_id, rep, STREAM_INIT))
    return {"dims": dims, "R": R, "storage": st, "y": y, "truth": truth, "init": init,
            "workload": w.name, "rep": rep, "snr_db": snr}


def random_tensor(dims, g: np.random.Generator, storage="f64"):
    """vec(Y) with i.i.d. N(0,1) entries (a tensor with no CP structure)."""
    n = int(np.prod(dims))
    x = g.standard_normal(n)
    if storage == "bf16":
        return to_bf16_bits(x)
    return x.astype({"f64": np.float64, "f32": np.float32}[storage])


NTF_WORKLOAD_ID = 6


def make_nonnegative_problem(dims, R, rep=0, snr_db=30.0, storage="f32"):
    """A seeded nonnegative CP problem (for the multiplicative update of
    eq. 2.18): true factors i.i.d. U(0, 1), Y = max([[A]] + E, 0) with E at the
    given SNR (entries clipped at zero after the noise, before the cast), and
    initial factors i.i.d. U(0.1, 1.1).  storage: 'f64' or 'f32'."""
    dims = tuple(int(d) for d in dims)
    R = int(R)
    g_true = rng(NTF_WORKLOAD_ID, rep, STREAM_TRUE)
    truth = [g_true.uniform(0.0, 1.0, (I, R)) for I in dims]
    y = noisy_cp_tensor(truth, snr_db, rng(NTF_WORKLOAD_ID, rep, STREAM_NOISE), storage)
    np.maximum(y, 0, out=y)
    g = rng(NTF_WORKLOAD_ID, rep, STREAM_INIT)
    init = [g.uniform(0.1, 1.1, (I, R)) for I in dims]
    return {"dims": dims, "R": R, "storage": storage, "y": y, "truth": truth, "init": init,
            "workload": "ntf_nonnegative", "rep": rep, "snr_db": snr_db}
