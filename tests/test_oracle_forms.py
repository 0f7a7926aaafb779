"""Pins for the oracle's further uses of the CP gradient (CPU only):
the multiplicative nonnegative update (eq. 2.18), the full gradient of
eq. 2.13, and the host Algorithm 2 / fast ALS of Sections 3.3 and 4 used by
the speed-ratio experiment (eq. 5.1)."""
import itertools

import numpy as np
import pytest

import cpgen
import oracle as O
from oracle import alg2_host as H


def _pos_factors(dims, R, seed, lo=0.1, hi=1.1):
    g = np.random.default_rng(seed)
    return [g.uniform(lo, hi, (I, R)) for I in dims]


# --------------------------------------------------------------------------
# eq. 2.18
# --------------------------------------------------------------------------

def test_ntf_update_brute_force():
    """eq. 2.18 for one mode with every sum written out: G(i,r) by eq. 3.2 and
    (A Gamma)(i,r) = sum_s A(i,s) prod_{k≠n} sum_j A_k(j,s) A_k(j,r)."""
    dims, R = (3, 2, 4), 2
    g = np.random.default_rng(3)
    Y = g.uniform(0, 1, dims)
    A = _pos_factors(dims, R, 4)
    for n in range(3):
        new = O.ntf_update(O.mttkrp(Y, A, n), A[n], O.gamma(A, n))
        for i, r in itertools.product(range(dims[n]), range(R)):
            gir = 0.0
            for idx in itertools.product(*[range(I) for I in dims]):
                if idx[n] != i:
                    continue
                p = Y[idx]
                for k in range(3):
                    if k != n:
                        p *= A[k][idx[k], r]
                gir += p
            den = 0.0
            for s in range(R):
                prod = 1.0
                for k in range(3):
                    if k != n:
                        prod *= sum(A[k][j, s] * A[k][j, r] for j in range(dims[k]))
                den += A[n][i, s] * prod
            assert abs(new[i, r] - A[n][i, r] * gir / den) <= 1e-13 * abs(new[i, r])


def test_ntf_rank_one_equals_als():
    """For R = 1, a ⊛ g ⊘ (a gamma) = g / gamma: the multiplicative sweep is the
    ALS sweep (eq. 2.14) whenever the denominators a gamma are positive (here:
    positive starting factors; the data and later factors may have any sign)."""
    g = np.random.default_rng(5)
    for dims in [(4, 5, 6), (3, 4, 5, 2)]:
        Y = g.uniform(0.0, 1.0, dims)
        A = [g.uniform(0.5, 1.5, (I, 1)) for I in dims]
        A1, D1, f1 = O.ntf_sweep(Y, A)
        A2, D2, f2 = O.als_sweep(Y, A)
        for a, b in zip(A1, A2):
            assert np.allclose(a, b, rtol=1e-12, atol=0)
        assert abs(D1 - D2) <= 1e-12 * O.norm2(Y)


def test_ntf_exact_model_is_fixed_point():
    """Y = [[A]] with positive factors: G^(n) = A^(n) Gamma^(n) exactly, so every
    ratio is one and the factors do not move; the cost is zero."""
    dims, R = (5, 4, 6, 3), 3
    A = _pos_factors(dims, R, 6)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, np.random.default_rng(0), "f64"), dims)
    A1, D, fit = O.ntf_sweep(Y, A)
    for a, b in zip(A1, A):
        assert np.allclose(a, b, rtol=1e-12, atol=0)
    assert abs(D) <= 1e-10 * O.norm2(Y)


def test_ntf_keeps_nonnegativity_and_never_raises_the_cost():
    """Nonnegative data and factors: each multiplicative step is a majorise-
    minimise step of the least-squares cost, so the explicit cost never
    increases, and the factors stay nonnegative."""
    pr = cpgen.make_nonnegative_problem((6, 7, 8, 5), 4, rep=3, storage="f64")
    Y = O.as_tensor(pr["y"], pr["dims"])
    A = [M.copy() for M in pr["init"]]
    c = O.cost_explicit(Y, A)
    for _ in range(8):
        A, D, fit = O.ntf_sweep(Y, A)
        c1 = O.cost_explicit(Y, A)
        assert c1 <= c * (1 + 1e-12)
        assert abs(D - c1) <= 1e-9 * O.norm2(Y)
        assert all(np.all(M >= 0) for M in A)
        c = c1


def test_ntf_planted_mistake_is_caught():
    """A rule that forgot A^(n) in the denominator (G ⊘ Gamma's row sums) breaks
    the fixed point of an exact model."""
    dims, R = (5, 4, 6), 3
    A = _pos_factors(dims, R, 8)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, np.random.default_rng(0), "f64"), dims)
    G = O.mttkrp(Y, A, 0)
    wrong = A[0] * G / O.gamma(A, 0).sum(axis=0)[None, :]
    assert not np.allclose(wrong, A[0], rtol=1e-6)
    assert np.allclose(O.ntf_update(G, A[0], O.gamma(A, 0)), A[0], rtol=1e-12)


# --------------------------------------------------------------------------
# eq. 2.13 in full
# --------------------------------------------------------------------------

def test_e_gradient_is_half_the_negative_cost_derivative():
    """eq. 2.13: dD/dA^(n) = -2 (G^(n) - A^(n) Gamma^(n)); checked against central
    differences of the explicit cost."""
    dims, R = (3, 4, 2), 2
    g = np.random.default_rng(9)
    Y = g.standard_normal(dims)
    A = [g.standard_normal((I, R)) for I in dims]
    E = O.e_gradient_all(Y, A)
    h = 1e-6
    for n in range(3):
        for i, r in itertools.product(range(dims[n]), range(R)):
            Ap = [M.copy() for M in A]
            Am = [M.copy() for M in A]
            Ap[n][i, r] += h
            Am[n][i, r] -= h
            d = (O.cost_explicit(Y, Ap) - O.cost_explicit(Y, Am)) / (2 * h)
            assert abs(d + 2 * E[n][i, r]) <= 1e-6 * (1 + abs(d))


# --------------------------------------------------------------------------
# host Algorithm 2 and fast ALS (Sections 3.3, 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(3, 4, 5), (4, 3, 5, 6), (3, 4, 2, 5, 3), (2, 3, 2, 3, 2, 3), (5, 6),
                                  (2, 3, 4, 1, 6, 2, 3)])
def test_host_algorithm2_matches_definition_at_every_split(dims):
    g = np.random.default_rng(len(dims))
    R = 3
    Y = g.standard_normal(dims)
    A = [g.standard_normal((I, R)) for I in dims]
    ref = O.cp_gradient_all(Y, A)
    for s in range(1, len(dims)):
        G = H.cp_gradient_all_fast(Y, A, s)
        for a, b in zip(G, ref):
            assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_host_algorithm2_brute_force():
    dims, R = (2, 3, 2, 2), 2
    g = np.random.default_rng(12)
    Y = g.standard_normal(dims)
    A = [g.standard_normal((I, R)) for I in dims]
    G = H.cp_gradient_all_fast(Y, A)
    for n in range(4):
        ref = np.zeros((dims[n], R))
        for idx in itertools.product(*[range(I) for I in dims]):
            for r in range(R):
                p = Y[idx]
                for k in range(4):
                    if k != n:
                        p *= A[k][idx[k], r]
                ref[idx[n], r] += p
        assert np.allclose(G[n], ref, rtol=1e-12, atol=1e-12)


def test_host_fast_als_matches_definition_sweep():
    pr = cpgen.make_problem("cp4d_64_r16_f32", rep=5, dims=(9, 8, 10, 7), rank=4)
    Y = O.as_tensor(cpgen.storage_to_f64(pr["y"], pr["storage"]), pr["dims"])
    A1, D1, f1 = O.als_sweep(Y, pr["init"])
    A2, D2, f2 = H.als_sweep_fast(Y, pr["init"])
    for a, b in zip(A1, A2):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
    assert abs(D1 - D2) <= 1e-10 * O.norm2(Y)
