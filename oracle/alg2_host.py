"""Algorithm 2 and the fast ALS sweep of Section 4 on the host, in float64
NumPy — TEST INFRASTRUCTURE ONLY (the CPU side of the paper's speed-ratio
experiment, Section 5, eq. 5.1).

The parity oracle is ``cp_oracle`` (the definition: explicit unfoldings and
Khatri-Rao products, Algorithm 1).  This module follows the steps of the
paper's fast method instead, so that the two can be timed against each other
on the same machine; it is pinned against ``cp_oracle`` by the tests.

Steps (Section 3.3): with the split n* (Algorithm 2, step 1) the free view
Y_(1:n*) (eq. 2.3, no data movement for a column-major tensor) is contracted
once from the right with the Khatri-Rao product of modes N..n*+1 (eq. 3.10)
and once from the left with that of modes n*..1 (eq. 3.9).  The gradients of
modes n*, ..., 1 then come from the right partial by peeling one mode at a
time (eqs. 3.20, 3.12) and those of modes n*+1, ..., N from the left one
(eqs. 3.22, 3.16).
"""
from __future__ import annotations

import numpy as np

from .cp_oracle import als_order, cost_identity, fit_from_cost, gamma, gram, khatri_rao, n_star, norm2

__all__ = ["cp_gradient_all_fast", "als_sweep_fast"]


def _kr(A, modes):
    """Khatri-Rao product of the listed modes with the FIRST listed mode's row
    index fastest (the row order of the reverse-ordered products of Notation
    2.1); a single row of ones for no modes."""
    if not modes:
        return np.ones((1, A[0].shape[1]))
    return khatri_rao([A[m] for m in reversed(modes)])


def _free_view(Y, s):
    """Y_(1:s) as a J_s x K_s matrix (eq. 2.3)."""
    J = int(np.prod(Y.shape[:s]))
    return np.reshape(Y, (J, -1), order="F")


def _right_partial(Y, A, s):
    """Columns r: vec of Y contracted over modes s+1..N with a_r (eq. 3.10)."""
    return _free_view(Y, s) @ _kr(A, list(range(s, Y.ndim)))


def _left_partial(Y, A, s):
    """Columns r: vec of Y contracted over modes 1..s with a_r (eq. 3.9)."""
    return _free_view(Y, s).T @ _kr(A, list(range(s)))


def _right_grad(Z, A, dims, m):
    """Gradient of 0-based mode m from the right chain tensor over modes 0..m
    (rows ivec(i_0..i_m)): contract modes 0..m-1 with their rank columns (eq. 3.12)."""
    lo = int(np.prod(dims[:m]))
    Zr = Z.reshape(lo, dims[m], -1, order="F")
    return np.einsum("jir,jr->ir", Zr, _kr(A, list(range(m))))


def _right_step(Z, A, dims, m):
    """Chain tensor over modes 0..m-1 from the one over modes 0..m (eq. 3.20)."""
    lo = int(np.prod(dims[:m]))
    return np.einsum("jir,ir->jr", Z.reshape(lo, dims[m], -1, order="F"), A[m])


def _left_grad(Z, A, dims, m):
    """Gradient of 0-based mode m from the left chain tensor over modes m..N-1
    (rows ivec(i_m..i_{N-1})): contract modes m+1..N-1 (eq. 3.16)."""
    Zr = Z.reshape(dims[m], -1, Z.shape[-1], order="F")
    return np.einsum("ikr,kr->ir", Zr, _kr(A, list(range(m + 1, len(dims)))))


def _left_step(Z, A, dims, m):
    """Chain tensor over modes m+1..N-1 from the one over modes m..N-1 (eq. 3.22)."""
    return np.einsum("ikr,ir->kr", Z.reshape(dims[m], -1, Z.shape[-1], order="F"), A[m])


def cp_gradient_all_fast(Y, A, nstar=None):
    """All N CP gradients by Algorithm 2 (1-based ``nstar`` overrides step 1)."""
    dims = Y.shape
    N = len(dims)
    s = n_star(dims) if nstar is None else int(nstar)
    G = [None] * N
    Z = _right_partial(Y, A, s)
    for m in range(s - 1, -1, -1):
        if m < s - 1:
            Z = _right_step(Z, A, dims, m + 1)
        G[m] = _right_grad(Z, A, dims, m)
    Z = _left_partial(Y, A, s)
    for m in range(s, N):
        if m > s:
            Z = _left_step(Z, A, dims, m - 1)
        G[m] = _left_grad(Z, A, dims, m)
    return G


def _solve(G, Gam):
    """eq. 2.14 for a symmetric positive definite Gamma (Cholesky)."""
    L = np.linalg.cholesky(Gam)
    Z = np.linalg.solve(L, G.T)
    return np.linalg.solve(L.T, Z).T


def als_sweep_fast(Y, A, normY2=None):
    """One fast ALS sweep (Section 4): the updates of eq. 2.14 inserted into the
    chains of Algorithm 2, modes n*, ..., 1 from the right partial, then a
    second partial with the updated modes 1..n* and modes n*+1, ..., N.
    Returns ``(A_new, cost, fit)`` like ``cp_oracle.als_sweep``."""
    dims = Y.shape
    N = len(dims)
    s = n_star(dims)
    A = [M.copy() for M in A]
    grams = [gram(M) for M in A]
    Z = _right_partial(Y, A, s)
    for m in range(s - 1, -1, -1):
        if m < s - 1:
            Z = _right_step(Z, A, dims, m + 1)
        A[m] = _solve(_right_grad(Z, A, dims, m), gamma(A, m, grams))
        grams[m] = gram(A[m])
    Z = _left_partial(Y, A, s)
    G = None
    for m in range(s, N):
        if m > s:
            Z = _left_step(Z, A, dims, m - 1)
        G = _left_grad(Z, A, dims, m)
        A[m] = _solve(G, gamma(A, m, grams))
        grams[m] = gram(A[m])
    if normY2 is None:
        normY2 = norm2(Y)
    D = cost_identity(normY2, G, A[N - 1], grams)
    assert als_order(N, s)[-1] == N - 1
    return A, D, fit_from_cost(D, normY2)
