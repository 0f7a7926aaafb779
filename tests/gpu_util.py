"""Helpers shared by the GPU tests: move a seeded problem to the device and
give the oracle the exact values the device holds (upcast to float64)."""
import numpy as np
import torch

import cpgen
import oracle as O

TDT = {"f64": torch.float64, "f32": torch.float32}


def factor_storage(storage):
    return "f64" if storage == "f64" else "f32"


def to_device_y(y, storage):
    if storage == "bf16":
        return torch.from_numpy(np.ascontiguousarray(y).view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(np.ascontiguousarray(y)).cuda()


def to_device_factors(mats, fst):
    return [torch.tensor(np.asarray(M), dtype=TDT[fst]).contiguous().cuda() for M in mats]


def exact_factors(dev):
    return [M.detach().cpu().double().numpy() for M in dev]


def exact_tensor(y, storage, dims):
    return O.as_tensor(cpgen.storage_to_f64(y, storage), dims)


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def problem(dims, R, storage, seed=0, snr=25.0, workload="cp4d_64_r16_f32"):
    return cpgen.make_problem(workload, rep=1000 + seed, dims=dims, rank=R, snr_db=snr, storage=storage)
