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


# Per-entry rounding bound of a computed gradient: |G - G_ref| <= c * Gabs,
# where Gabs is the same gradient of |Y| and |A^(k)| (the sum of the
# magnitudes of an entry's terms).  Any evaluation order with at most d
# roundings per term obeys c = gamma_d = d u / (1 - d u) (recursive-summation
# bound).  The float32 path rounds a term at most d <= 3300 times (product of
# the Khatri-Rao factors, up to 1920 columns accumulated in one split partial,
# the chain sums over I_n, the float32 stores between kernels), so
# c = 2e-4 >= gamma_3300 at u = 2^-24; float64: c = 1e-12 >= gamma_3300 at
# u = 2^-53.  The bf16-refined form: the hi/lo split leaves O(u_bf16^2) per
# operand (u_bf16 = 2^-8), c = 4 u_bf16^2 + 2e-5.
U_BF16 = 2.0 ** -8
ENTRY_BOUND = {"f64": 1e-12, "f32": 2e-4, "bf16_refined": 4 * U_BF16 ** 2 + 2e-5,
               "bf16": 2 * U_BF16 + U_BF16 ** 2 + 2e-5}
# relative Frobenius error per mode and max|dG| / max|G_ref| (the tolerance of
# the float64 / float32 forms; the bf16-refined form is held to the same)
FRO_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16_refined": 1e-5}


def magnitude_gradients(Y, A):
    return O.cp_gradient_all(np.abs(Y), [np.abs(M) for M in A])


def check_gradients(G, ref, gabs, form, label=""):
    """Element-wise parity of every mode's gradient; returns per-mode
    (relative Frobenius error, max|dG|/max|G_ref|, max |dG|/Gabs)."""
    out = []
    for n, (g, r, a) in enumerate(zip(G, ref, gabs)):
        d = np.abs(np.asarray(g, dtype=np.float64) - r)
        fro = rel_fro(g, r)
        mx = float(d.max() / max(float(np.abs(r).max()), 1e-300))
        ent = float(np.max(d / (a + 1e-300)))
        out.append((fro, mx, ent))
        if form in FRO_TOL:
            assert fro <= FRO_TOL[form] and mx <= FRO_TOL[form], (label, n, fro, mx)
        bad = np.argwhere(d > ENTRY_BOUND[form] * a + 1e-300)
        assert bad.size == 0, (label, n, bad[:4].tolist(), ent)
    print(f"  {label} fro/max/entry: " + " ".join(f"{f:.1e}/{m:.1e}/{e:.1e}" for f, m, e in out), flush=True)
    return out
