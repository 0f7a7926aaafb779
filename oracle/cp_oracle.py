"""Plain float64 CP oracle — test infrastructure only (see the package header).

Every function states the passage of the paper it follows.  Mode numbers in
the API are 0-based (mode ``n`` here is the paper's mode n+1) except
``n_star``, which returns the paper's 1-based n*.

Tensors: ``vec`` is vec(Y) with the first mode fastest (eq. 2.1), and
``as_tensor(vec, dims)`` views it as an N-way array Y[i_1, ..., i_N].
Factors: A[n] is an I_n x R float64 array.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = [
    "as_tensor", "ivec", "unfold", "unfold_rc", "khatri_rao", "kr_except",
    "mttkrp", "cp_gradient_all", "gradient_entry", "n_star", "gram", "gamma",
    "cholesky_jitter_solve", "NotSPD", "als_order", "als_sweep", "cp_als", "cp_full",
    "cost_explicit", "cost_identity", "fit_from_cost", "norm2", "e_gradient_all",
    "gradient_row", "ntf_update", "ntf_sweep",
]

JITTER = 1e-12


class NotSPD(ArithmeticError):
    """The normal-equation matrix of eq. 2.14 could not be factorised."""


# ----------------------------------------------------------------------------
# storage, reshaping and unfolding (Section 2: eq. 2.1, Def. 2.1, Def. 2.2)
# ----------------------------------------------------------------------------

def as_tensor(vec, dims):
    """Y[i_1,...,i_N] with vec(Y)[ivec(i)] = Y[i] (eq. 2.1: first index fastest)."""
    return np.asarray(vec, dtype=np.float64).reshape(tuple(dims), order="F")


def ivec(idx, dims):
    """0-based linear index of eq. 2.1: i_1 + sum_n i_n * prod_{j<n} I_j."""
    lin, stride = 0, 1
    for i, I in zip(idx, dims):
        lin += int(i) * stride
        stride *= int(I)
    return lin


def unfold_rc(Y, rows, cols):
    """Def. 2.2: Y_(r x c)(j1, j2) = Y(i_r, i_c), j1 = ivec(i_r), j2 = ivec(i_c).

    ``rows`` and ``cols`` are 0-based mode lists that together permute 0..N-1.
    """
    perm = list(rows) + list(cols)
    P = np.transpose(Y, perm)
    nr = int(np.prod([Y.shape[m] for m in rows])) if rows else 1
    return P.reshape((nr, -1), order="F")


def unfold(Y, n):
    """Mode-n unfolding Y_(n) (Remark 2.1.2): rows = mode n, columns = ivec of the
    other modes in increasing order — Algorithm 1, steps 1-2 (permute, reshape)."""
    N = Y.ndim
    return unfold_rc(Y, [n], [m for m in range(N) if m != n])


# ----------------------------------------------------------------------------
# Khatri-Rao products (Notation 2.1, eq. 3.3)
# ----------------------------------------------------------------------------

def khatri_rao(mats):
    """M_1 (.) M_2 (.) ... (.) M_m: column r is kron(m1_r, kron(m2_r, ...)), so the
    LAST matrix's row index varies fastest (standard Kronecker convention)."""
    R = mats[0].shape[1]
    rows = int(np.prod([M.shape[0] for M in mats]))
    out = np.empty((rows, R))
    for r in range(R):
        t = np.ones(1)
        for M in mats:
            t = np.kron(t, M[:, r])
        out[:, r] = t
    return out


def kr_except(A, n):
    """Notation 2.1: the reverse-ordered product A^(N) (.) ... (.) A^(n+1) (.) A^(n-1)
    (.) ... (.) A^(1) (0-based: every mode except ``n``, highest mode first)."""
    return khatri_rao([A[k] for k in reversed(range(len(A))) if k != n])


# ----------------------------------------------------------------------------
# the CP gradient (eq. 2.13 / eq. 3.1) by its definition
# ----------------------------------------------------------------------------

def mttkrp(Y, A, n):
    """G^(n) = Y_(n) (⊙_{k≠n} A^(k)) — Algorithm 1 (explicit unfolding, explicit
    Khatri-Rao product, one matrix product), in float64."""
    return unfold(Y, n) @ kr_except(A, n)


def cp_gradient_all(Y, A):
    """All N CP gradients, each by Algorithm 1 (the result Algorithm 2 must reach)."""
    return [mttkrp(Y, A, n) for n in range(Y.ndim)]


def gradient_entry(Y, A, n, i, r):
    """One entry g_r^(n)(i) of eq. 3.2: the slice Y(i_n = i) contracted with
    a_r^(k) along every other mode k (Def. 2.3 mode products), float64.
    Used to check single entries of the gradient on tensors too big for the
    full unfoldings."""
    S = Y[(slice(None),) * n + (i,)]   # (N-1)-way slice (a view: no copy of Y)
    modes = [k for k in range(Y.ndim) if k != n]
    for ax in reversed(range(S.ndim)):  # contract the last axis each time
        S = np.tensordot(S, A[modes[ax]][:, r], axes=([ax], [0]))
    return float(S)


def gradient_row(Y, A, n, i):
    """Row i of G^(n) (eq. 3.2 for every r at once): the slice Y(i_n = i)
    contracted along every other mode k with A^(k), keeping the rank index,
    float64.  For sampling rows of the gradient of large tensors."""
    S = np.ascontiguousarray(Y[(slice(None),) * n + (i,)])   # (N-1)-way slice, copied alone
    modes = [k for k in range(Y.ndim) if k != n]
    # contract the last slice axis with A^(last), then each remaining axis
    # against the matching factor while keeping r (a Hadamard step over r)
    T = np.tensordot(S, A[modes[-1]], axes=([S.ndim - 1], [0]))   # (..., R)
    for ax in reversed(range(S.ndim - 1)):
        T = np.einsum("...jr,jr->...r", T, A[modes[ax]])
    return np.asarray(T, dtype=np.float64)


def e_gradient_all(Y, A):
    """eq. 2.13 in full: E_(n)(⊙A) = Y_(n)(⊙A) - A^(n) (⊛_{k≠n} A^(k)T A^(k))."""
    return [mttkrp(Y, A, n) - A[n] @ gamma(A, n) for n in range(Y.ndim)]


# ----------------------------------------------------------------------------
# the split point n* (Algorithm 2, step 1; eq. 2.3)
# ----------------------------------------------------------------------------

def n_star(dims):
    """Paper's 1-based n* = max{n in [1, N-1] : J_n <= K_n}, J_n = I_1...I_n,
    K_n = I_{n+1}...I_N; 1 if no n qualifies."""
    N = len(dims)
    best = 1
    for n in range(1, N):
        J = int(np.prod(dims[:n]))
        K = int(np.prod(dims[n:]))
        if J <= K:
            best = n
    return best


# ----------------------------------------------------------------------------
# CP_ALS (eq. 2.14, Section 4)
# ----------------------------------------------------------------------------

def gram(M):
    """A^T A (float64)."""
    return M.T @ M


def gamma(A, n, grams=None):
    """⊛_{k≠n} A^(k)T A^(k) (eq. 2.14), float64."""
    R = A[0].shape[1]
    G = np.ones((R, R))
    for k in range(len(A)):
        if k != n:
            G = G * (grams[k] if grams is not None else gram(A[k]))
    return G


def cholesky_jitter_solve(G, Gam):
    """X = G Gam^{-1} for symmetric positive definite Gam (eq. 2.14; for SPD Gam
    the pseudo-inverse is the inverse).  LAPACK Cholesky; if it fails, one retry
    with Gam + 1e-12 * trace(Gam)/R * I; if that fails too, NotSPD."""
    R = Gam.shape[0]
    for attempt in range(2):
        M = Gam if attempt == 0 else Gam + (JITTER * np.trace(Gam) / R) * np.eye(R)
        try:
            L = np.linalg.cholesky(M)
        except np.linalg.LinAlgError:
            continue
        if not np.all(np.isfinite(L)):
            continue
        return scipy.linalg.cho_solve((L, True), G.T).T
    raise NotSPD("normal-equation matrix is not positive definite")


def als_order(N, nstar):
    """Section 4 update order: n*, n*-1, ..., 1, n*+1, ..., N (returned 0-based)."""
    return [n - 1 for n in range(nstar, 0, -1)] + [n - 1 for n in range(nstar + 1, N + 1)]


def norm2(Y):
    return float(np.sum(np.asarray(Y, dtype=np.float64) ** 2))


def cost_identity(normY2, G_last, A_last, grams):
    """eq. 2.12 expanded: D = ||Y||^2 - 2<Y,Yhat> + ||Yhat||^2, with
    <Y,Yhat> = sum_{i,r} G^(N)(i,r) A^(N)(i,r) (G^(N) = Y_(N)(⊙_{k≠N}A^(k))) and
    ||Yhat||^2 = sum_{r,s} (⊛_n A^(n)T A^(n))_{rs}."""
    inner = float(np.sum(G_last * A_last))
    H = np.ones_like(grams[0])
    for Gm in grams:
        H = H * Gm
    return normY2 - 2.0 * inner + float(np.sum(H))


def cp_full(A):
    """Yhat of Def. 2.4 (eq. 2.7) as an N-way array: Yhat_(1) = A^(1) (⊙_{k≠1} A^(k))^T."""
    dims = [M.shape[0] for M in A]
    Y1 = A[0] @ kr_except(A, 0).T
    # fold back: columns of Y_(1) are ivec of modes 2..N, i.e. plain column-major
    return Y1.reshape(dims, order="F")


def cost_explicit(Y, A):
    """eq. 2.12 from the residual tensor itself: ||Y - Yhat||_F^2."""
    E = Y - cp_full(A)
    return float(np.sum(E * E))


def fit_from_cost(D, normY2):
    """fit = 1 - ||Y - Yhat||_F / ||Y||_F (D clamped at 0)."""
    return 1.0 - np.sqrt(max(D, 0.0)) / np.sqrt(normY2)


def als_sweep(Y, A, order=None, normY2=None):
    """One CP_ALS sweep (eq. 2.14) in the Section 4 order by default.

    Each G^(n) is the definition with the current factors (modes already
    updated in this sweep enter with their new values).  Returns
    ``(A_new, cost, fit)``: the cost is the identity form, using G^(N) from the
    sweep and the final factors, exactly as the device computes it.
    """
    N = Y.ndim
    A = [M.copy() for M in A]
    if order is None:
        order = als_order(N, n_star(Y.shape))
    grams = [gram(M) for M in A]
    G_last = None
    for n in order:
        G = mttkrp(Y, A, n)
        A[n] = cholesky_jitter_solve(G, gamma(A, n, grams))
        grams[n] = gram(A[n])
        if n == order[-1]:
            G_last = G
    if normY2 is None:
        normY2 = norm2(Y)
    D = cost_identity(normY2, G_last, A[order[-1]], grams)
    return A, D, fit_from_cost(D, normY2)


def cp_als(Y, A, sweeps, tol=None, order=None):
    """Plain CP_ALS: ``sweeps`` sweeps, or stop when |fit_k - fit_{k-1}| < tol.
    Returns (A, fits)."""
    normY2 = norm2(Y)
    fits = []
    for _ in range(sweeps):
        A, _, f = als_sweep(Y, A, order=order, normY2=normY2)
        fits.append(f)
        if tol is not None and len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    return A, fits


# ----------------------------------------------------------------------------
# the multiplicative nonnegative update (eq. 2.18)
# ----------------------------------------------------------------------------

def ntf_update(G, An, Gam, tiny=np.finfo(np.float64).tiny):
    """eq. 2.18 for one mode: A^(n) ⊛ G^(n) ⊘ (A^(n) Gamma^(n)); a denominator
    below ``tiny`` (the factor type's smallest normal number) is raised to it."""
    den = An @ Gam
    return An * G / np.maximum(den, tiny)


def ntf_sweep(Y, A, order=None, normY2=None, tiny=np.finfo(np.float64).tiny):
    """One sweep of eq. 2.18, each G^(n) by the definition with the current
    factors, in the Section 4 order by default (the order in which the fast
    gradients of Algorithm 2 become available).  Returns ``(A_new, cost, fit)``
    with the cost by the identity of eq. 2.12, as ``als_sweep``."""
    N = Y.ndim
    A = [M.copy() for M in A]
    if order is None:
        order = als_order(N, n_star(Y.shape))
    G_last = None
    for n in order:
        G = mttkrp(Y, A, n)
        A[n] = ntf_update(G, A[n], gamma(A, n), tiny)
        if n == order[-1]:
            G_last = G
    if normY2 is None:
        normY2 = norm2(Y)
    grams = [gram(M) for M in A]
    D = cost_identity(normY2, G_last, A[order[-1]], grams)
    return A, D, fit_from_cost(D, normY2)
