"""Pins for the CPU oracle: each test checks it against something other than
itself — hand-derived values, closed forms, brute-force sums, textbook special
cases and invariants of the mathematics.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import cpgen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_factors(dims, R, seed):
    g = np.random.default_rng(seed)
    return [g.standard_normal((I, R)) for I in dims]


def _brute_gradient(Y, A, n):
    """eq. 3.2 element by element with plain Python loops (tiny tensors only)."""
    dims = Y.shape
    R = A[0].shape[1]
    G = np.zeros((dims[n], R))
    for idx in itertools.product(*[range(I) for I in dims]):
        y = Y[idx]
        for r in range(R):
            p = y
            for k, i in enumerate(idx):
                if k != n:
                    p *= A[k][i, r]
            G[idx[n], r] += p
    return G


# --------------------------------------------------------------------------
# layout (eq. 2.1, Def. 2.1, Def. 2.2)
# --------------------------------------------------------------------------

def test_ivec_is_first_index_fastest():
    dims = (2, 3, 4)
    vec = np.arange(24, dtype=float)
    Y = O.as_tensor(vec, dims)
    for i, j, k in itertools.product(range(2), range(3), range(4)):
        assert Y[i, j, k] == vec[i + 2 * j + 6 * k]
        assert O.ivec((i, j, k), dims) == i + 2 * j + 6 * k


def test_unfold_matches_definition_elementwise():
    dims = (2, 3, 4, 2)
    Y = O.as_tensor(np.arange(48, dtype=float) * 1.5 - 7, dims)
    for n in range(4):
        Yn = O.unfold(Y, n)
        others = [m for m in range(4) if m != n]
        assert Yn.shape == (dims[n], 48 // dims[n])
        for idx in itertools.product(*[range(I) for I in dims]):
            col, stride = 0, 1
            for m in others:            # Def. 2.2: column = ivec of the other modes
                col += idx[m] * stride
                stride *= dims[m]
            assert Yn[idx[n], col] == Y[idx]


def test_unfold_leading_modes_is_a_free_reshape():
    """Remark 2.1.4 / eq. 2.3: Y_(1:n) = reshape(Y, [J_n, K_n]) of the same vector."""
    dims = (3, 2, 4, 5)
    vec = np.arange(120, dtype=float)
    Y = O.as_tensor(vec, dims)
    for n in range(1, 4):
        J = int(np.prod(dims[:n]))
        M = O.unfold_rc(Y, list(range(n)), list(range(n, 4)))
        assert np.array_equal(M, vec.reshape((J, -1), order="F"))
        # column c holds J contiguous entries of vec(Y) (eq. 2.11)
        for c in range(M.shape[1]):
            assert np.array_equal(M[:, c], vec[c * J:(c + 1) * J])
    # Remark 2.1.3 / eq. 2.10: Y_(N) = Y_(1:N-1)^T
    assert np.array_equal(O.unfold(Y, 3), O.unfold_rc(Y, [0, 1, 2], [3]).T)


def test_khatri_rao_reverse_order_index():
    """Notation 2.1: in A^(3) (.) A^(2) (.) A^(1) the row index is ivec(i_1,i_2,i_3)."""
    A = _rand_factors((2, 3, 4), 3, 1)
    K = O.khatri_rao([A[2], A[1], A[0]])
    for i1, i2, i3 in itertools.product(range(2), range(3), range(4)):
        row = i1 + 2 * i2 + 6 * i3
        assert np.allclose(K[row], A[0][i1] * A[1][i2] * A[2][i3], rtol=0, atol=1e-15)
    Kx = O.kr_except(A, 1)
    for i1, i3 in itertools.product(range(2), range(4)):
        assert np.allclose(Kx[i1 + 2 * i3], A[0][i1] * A[2][i3], rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# the gradient (eq. 2.13, eq. 3.1-3.2)
# --------------------------------------------------------------------------

def test_hand_worked_example():
    with open(os.path.join(GOLDEN, "hand_2x2x2.json")) as f:
        gold = json.load(f)
    Y = O.as_tensor(np.array(gold["vec_y"], dtype=float), gold["dims"])
    A = [np.array(M, dtype=float) for M in gold["factors"]]
    G = O.cp_gradient_all(Y, A)
    for n in range(3):
        assert np.array_equal(G[n], np.array(gold["gradients"]["G"][n], dtype=float))
    A1, _, _ = O.als_sweep(Y, A)
    for n in range(3):
        assert np.allclose(A1[n], np.array(gold["als_sweep"]["factors"][n]), rtol=1e-14, atol=0)


@pytest.mark.parametrize("dims,R", [((2, 3, 4), 2), ((3, 2, 2, 3), 3), ((2, 2, 3, 2, 2), 2), ((4, 3), 2)])
def test_brute_force(dims, R):
    g = np.random.default_rng(7)
    Y = O.as_tensor(g.standard_normal(int(np.prod(dims))), dims)
    A = _rand_factors(dims, R, 8)
    for n in range(len(dims)):
        assert np.allclose(O.mttkrp(Y, A, n), _brute_gradient(Y, A, n), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims,R", [((3, 4, 5, 6), 3), ((5, 2, 7), 4), ((2, 3, 2, 3, 2), 2)])
def test_closed_form_exact_model(dims, R):
    """Y = [[A]] exactly  =>  G^(n) = A^(n) (⊛_{k≠n} A^(k)T A^(k)) (Def. 2.4, eq. 2.13),
    with the tensor assembled by the input generator, not by the oracle."""
    A = _rand_factors(dims, R, 3)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, None, "f64"), dims)
    for n in range(len(dims)):
        ref = A[n] @ O.gamma(A, n)
        assert np.allclose(O.mttkrp(Y, A, n), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # the full gradient of eq. 2.13 vanishes at an exact model
    for E in O.e_gradient_all(Y, A):
        assert np.abs(E).max() < 1e-10


def test_rank_one_is_tensor_times_vectors():
    """R = 1: G^(n) is Y contracted with one vector along every other mode (eq. 2.6)."""
    dims = (3, 4, 2, 5)
    g = np.random.default_rng(11)
    Y = O.as_tensor(g.standard_normal(120), dims)
    A = _rand_factors(dims, 1, 12)
    a, b, c, d = (M[:, 0] for M in A)
    refs = [np.einsum("ijkl,j,k,l->i", Y, b, c, d), np.einsum("ijkl,i,k,l->j", Y, a, c, d),
            np.einsum("ijkl,i,j,l->k", Y, a, b, d), np.einsum("ijkl,i,j,k->l", Y, a, b, c)]
    for n in range(4):
        assert np.allclose(O.mttkrp(Y, A, n)[:, 0], refs[n], rtol=1e-13, atol=1e-13)


def test_matrix_case():
    """N = 2: G^(1) = Y A^(2) and G^(2) = Y^T A^(1) (Remark 2.1.3)."""
    g = np.random.default_rng(5)
    M = g.standard_normal((6, 9))
    Y = O.as_tensor(M.reshape(-1, order="F"), (6, 9))
    A = _rand_factors((6, 9), 4, 6)
    assert np.allclose(O.mttkrp(Y, A, 0), M @ A[1], rtol=1e-14, atol=1e-14)
    assert np.allclose(O.mttkrp(Y, A, 1), M.T @ A[0], rtol=1e-14, atol=1e-14)


def test_gradient_entry_matches_full():
    dims = (3, 5, 2, 4)
    g = np.random.default_rng(9)
    Y = O.as_tensor(g.standard_normal(120), dims)
    A = _rand_factors(dims, 3, 10)
    for n in range(4):
        G = O.mttkrp(Y, A, n)
        for i in range(dims[n]):
            for r in range(3):
                assert abs(O.gradient_entry(Y, A, n, i, r) - G[i, r]) < 1e-12


def test_gradient_row_matches_entries_and_full():
    """Rows of G^(n) from the slice contraction agree with the element-wise
    sums (eq. 3.2) and with Algorithm 1; a transposed factor (a planted
    mistake in the oracle's contraction order) would not."""
    dims = (4, 3, 5, 2, 3)
    g = np.random.default_rng(11)
    Y = O.as_tensor(g.standard_normal(int(np.prod(dims))), dims)
    A = _rand_factors(dims, 3, 12)
    for n in range(5):
        G = O.mttkrp(Y, A, n)
        for i in range(dims[n]):
            row = O.gradient_row(Y, A, n, i)
            assert np.allclose(row, G[i], rtol=1e-13, atol=1e-13)
            assert abs(row[1] - O.gradient_entry(Y, A, n, i, 1)) < 1e-12
    # planted: the factors of modes 2 and 5 (both of size 3) swapped
    n, i = 3, 1
    S = np.take(Y, i, axis=n)   # axes: modes 1, 2, 3, 5
    bad = np.einsum("abcd,ar,br,cr,dr->r", S, A[0], A[4], A[2], A[1])
    assert not np.allclose(bad, O.gradient_row(Y, A, n, i), rtol=1e-6)


# --------------------------------------------------------------------------
# n* (Algorithm 2, step 1)
# --------------------------------------------------------------------------

def test_n_star():
    for N in range(2, 9):
        assert O.n_star((10,) * N) == N // 2          # cubic: J_n <= K_n  <=>  n <= N/2
    assert O.n_star((64,) * 4) == 2                    # tie J_2 = K_2 counts
    assert O.n_star((20, 20, 20)) == 1
    assert O.n_star((48,) * 5) == 2
    assert O.n_star((40, 50, 60, 70)) == 2
    assert O.n_star((100, 2, 2)) == 1                  # no n qualifies -> 1
    assert O.n_star((2, 3, 100)) == 2
    assert O.als_order(5, 2) == [1, 0, 2, 3, 4]
    assert O.als_order(7, 3) == [2, 1, 0, 3, 4, 5, 6]


# --------------------------------------------------------------------------
# CP_ALS (eq. 2.14, Section 4) and the cost (eq. 2.12)
# --------------------------------------------------------------------------

def test_als_each_update_does_not_increase_cost():
    """Each update of eq. 2.14 is the exact least-squares minimiser over A^(n)."""
    dims = (4, 5, 3, 6)
    g = np.random.default_rng(21)
    Y = O.as_tensor(g.standard_normal(360), dims)
    A = _rand_factors(dims, 3, 22)
    D = O.cost_explicit(Y, A)
    for _ in range(4):
        for n in O.als_order(4, O.n_star(dims)):
            A[n] = O.cholesky_jitter_solve(O.mttkrp(Y, A, n), O.gamma(A, n))
            Dn = O.cost_explicit(Y, A)
            assert Dn <= D * (1 + 1e-12)
            D = Dn


def test_als_update_solves_normal_equations():
    dims = (5, 4, 6)
    g = np.random.default_rng(31)
    Y = O.as_tensor(g.standard_normal(120), dims)
    A = _rand_factors(dims, 3, 32)
    for n in range(3):
        G = O.mttkrp(Y, A, n)
        Gam = O.gamma(A, n)
        X = O.cholesky_jitter_solve(G, Gam)
        assert np.linalg.norm(X @ Gam - G) <= 1e-13 * np.linalg.norm(G)
        # least-squares optimality: the full gradient (eq. 2.13) at the update is 0
        B = list(A)
        B[n] = X
        E = O.mttkrp(Y, B, n) - X @ O.gamma(B, n)
        assert np.abs(E).max() < 1e-10 * np.abs(G).max()


def test_true_factors_are_a_fixed_point():
    dims = (4, 5, 6, 3)
    A = _rand_factors(dims, 2, 41)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, None, "f64"), dims)
    A1, D, fit = O.als_sweep(Y, A)
    for n in range(4):
        assert np.allclose(A1[n], A[n], rtol=1e-10, atol=1e-10)
    assert abs(D) < 1e-9 * O.norm2(Y)
    assert abs(fit - 1.0) < 1e-6


def test_cost_identity_equals_explicit_residual():
    dims = (3, 4, 5, 2)
    g = np.random.default_rng(51)
    Y = O.as_tensor(g.standard_normal(120), dims)
    A = _rand_factors(dims, 3, 52)
    A1, D, fit = O.als_sweep(Y, A)
    De = O.cost_explicit(Y, A1)
    assert abs(D - De) <= 1e-11 * O.norm2(Y)
    assert abs(fit - (1 - np.sqrt(De / O.norm2(Y)))) < 1e-10


def test_als_recovers_noiseless_low_rank():
    dims = (6, 7, 8)
    A = _rand_factors(dims, 2, 61)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, None, "f64"), dims)
    A0 = _rand_factors(dims, 2, 62)
    _, fits = O.cp_als(Y, A0, 300, tol=1e-12)
    assert fits[-1] > 1 - 1e-6


def test_not_spd_and_jitter():
    R = 3
    G = np.ones((4, R))
    with pytest.raises(O.NotSPD):
        O.cholesky_jitter_solve(G, np.zeros((R, R)))
    # a Gamma with one exactly-zero row/column is rescued by the jitter retry
    Gam = np.diag([2.0, 0.0, 3.0])
    X = O.cholesky_jitter_solve(G, Gam)
    assert np.all(np.isfinite(X))
    with pytest.raises(O.NotSPD):
        O.cholesky_jitter_solve(G, np.diag([1.0, np.nan, 1.0]))


# --------------------------------------------------------------------------
# the pins have teeth: plant a mistake in the oracle and watch a pin fail
# --------------------------------------------------------------------------

def test_planted_kr_order_mistake_is_caught(monkeypatch):
    """Forward-ordered Khatri-Rao products (A^(1) fastest reversed) break the brute-force pin."""
    dims, R = (2, 3, 4), 2
    g = np.random.default_rng(71)
    Y = O.as_tensor(g.standard_normal(24), dims)
    A = _rand_factors(dims, R, 72)
    wrong = lambda A_, n: O.khatri_rao([A_[k] for k in range(len(A_)) if k != n])  # noqa: E731
    monkeypatch.setattr(O.cp_oracle, "kr_except", wrong)
    bad = [not np.allclose(O.cp_oracle.mttkrp(Y, A, n), _brute_gradient(Y, A, n)) for n in range(3)]
    assert any(bad)


def test_planted_transpose_mistake_is_caught(monkeypatch):
    """Using Y_(n) columns in the wrong mode order breaks the closed-form pin."""
    dims, R = (3, 4, 5), 2
    A = _rand_factors(dims, R, 81)
    Y = O.as_tensor(cpgen.noisy_cp_tensor(A, None, None, "f64"), dims)

    def wrong_unfold(Y_, n):
        others = [m for m in range(Y_.ndim) if m != n][::-1]
        return O.unfold_rc(Y_, [n], others)
    monkeypatch.setattr(O.cp_oracle, "unfold", wrong_unfold)
    n = 1
    assert not np.allclose(O.cp_oracle.mttkrp(Y, A, n), A[n] @ O.gamma(A, n))
