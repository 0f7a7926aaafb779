"""The seeded input generators: reproducibility, the congruence and SNR recipes,
and bfloat16 rounding.  CPU only."""
import numpy as np
import torch

import cpgen


def test_seeded_reproducible():
    a = cpgen.make_problem("cp3d_20_r3_f64", rep=0)
    b = cpgen.make_problem("cp3d_20_r3_f64", rep=0)
    c = cpgen.make_problem("cp3d_20_r3_f64", rep=1)
    assert np.array_equal(a["y"], b["y"])
    assert not np.array_equal(a["y"], c["y"])
    assert a["y"].dtype == np.float64 and a["y"].size == 8000


def test_congruent_factors_have_exact_cosines():
    g = cpgen.rng(99, 0, 0)
    A = cpgen.congruent_factors((40, 50, 20), 8, 0.9, g)
    for M in A:
        Gm = M.T @ M
        d = np.sqrt(np.diag(Gm))
        C = Gm / np.outer(d, d)
        off = C[~np.eye(8, dtype=bool)]
        assert np.allclose(off, 0.9, atol=1e-12)
        assert np.allclose(d, np.sqrt(M.shape[0]), rtol=1e-12)


def test_snr_recipe():
    g = cpgen.rng(98, 0, 0)
    A = cpgen.gaussian_factors((20, 30, 25), 4, g)
    clean = cpgen.noisy_cp_tensor(A, None, None, "f64")
    noisy = cpgen.noisy_cp_tensor(A, 20.0, cpgen.rng(98, 0, 1), "f64")
    snr = 10 * np.log10(np.sum(clean ** 2) / np.sum((noisy - clean) ** 2))
    assert abs(snr - 20.0) < 0.2


def test_bf16_round_to_nearest_even_matches_torch():
    g = np.random.default_rng(3)
    x = np.concatenate([g.standard_normal(10000) * 10 ** g.uniform(-5, 5, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]]).astype(np.float32)
    bits = cpgen.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bits, ref)
    back = cpgen.bf16_bits_to_f64(bits)
    assert np.array_equal(back, torch.from_numpy(x).to(torch.bfloat16).double().numpy())


def test_learned_workload_rank_range():
    w = cpgen.WORKLOADS["cp4d_40x70_learned"]
    ranks = {cpgen.workload_rank(w, rep) for rep in range(200)}
    assert min(ranks) >= 8 and max(ranks) <= 20 and len(ranks) > 8
