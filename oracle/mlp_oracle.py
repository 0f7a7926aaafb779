"""Float64 reference of the learned-step network and features — test
infrastructure only (see the package header).

The paper gives no design for a learned step (it only names line-search
extrapolation, Section 1); the network, its loss and the features follow the
definitions documented with the library's C ABI, written out plainly here:

  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), z = w3 . h2 + b3,
  sigma = sigma_max * sigmoid(z),
  loss = mean_s (log(1 + sigma_s) - log(1 + target_s))^2,
  params = [W1 (H x F row-major), b1, W2 (H x H), b2, w3, b3].
"""
from __future__ import annotations

import numpy as np

__all__ = ["mlp_unpack", "mlp_nparams", "mlp_forward", "mlp_loss_grad", "adam_step", "step_features",
           "extrapolate"]


def mlp_nparams(F, H):
    return H * F + H + H * H + H + H + 1


def mlp_unpack(p, F, H):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def mlp_forward(p, X, F, H, smax):
    """sigma for every row of X (float64)."""
    W1, b1, W2, b2, w3, b3 = mlp_unpack(p, F, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    z = h2 @ w3 + b3
    return smax / (1.0 + np.exp(-z))


def mlp_loss_grad(p, X, target, F, H, smax):
    """(loss, gradient) by hand-written backpropagation, float64."""
    W1, b1, W2, b2, w3, b3 = mlp_unpack(p, F, H)
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    a1 = X @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    z = h2 @ w3 + b3
    sg = 1.0 / (1.0 + np.exp(-z))
    sigma = smax * sg
    err = np.log1p(sigma) - np.log1p(np.asarray(target, dtype=np.float64))
    loss = float(np.mean(err ** 2))
    dz = (2.0 * err / B) / (1.0 + sigma) * smax * sg * (1.0 - sg)
    gw3 = h2.T @ dz
    gb3 = dz.sum()
    d2 = np.outer(dz, w3) * (1.0 - h2 ** 2)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 ** 2)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def extrapolate(A, A_start, sigma):
    """A + sigma (A - A_start), mode by mode."""
    return [a + sigma * (a - s) for a, s in zip(A, A_start)]


def step_features(A, A_start, D_prev, costs, iteration, last_sigma, last_accept, R):
    """The 12 step features (definitions of include/cpmlp.h), float64.
    costs: history including the newest cost, oldest first; D_prev: the
    previous update per mode or None."""
    c = list(costs)[-5:]
    f = np.zeros(12)
    nc = len(c)
    for k in range(4):
        j = nc - 4 + k
        rel = 1.0
        if 1 <= j < nc and c[j - 1] > 0:
            rel = (c[j - 1] - c[j]) / c[j - 1]
        rel = min(max(rel, 1e-12), 1.0)
        f[k] = np.log10(rel) / 12.0
    N = len(A)
    lr, cs = [], []
    for n in range(N):
        u = np.asarray(A[n], dtype=np.float64) - np.asarray(A_start[n], dtype=np.float64)
        uu, aa = float(np.sum(u * u)), float(np.sum(np.asarray(A[n], dtype=np.float64) ** 2))
        lr.append(np.log10(max(np.sqrt(uu) / (np.sqrt(aa) + 1e-300), 1e-12)))
        if D_prev is None:
            cs.append(0.0)
        else:
            d = np.asarray(D_prev[n], dtype=np.float64)
            dd, ud = float(np.sum(d * d)), float(np.sum(u * d))
            cs.append(ud / np.sqrt(uu * dd) if uu > 0 and dd > 0 else 0.0)
    f[4] = np.mean(lr) / 6.0
    f[5] = np.max(lr) / 6.0
    f[6] = np.mean(cs)
    f[7] = np.min(cs)
    f[8] = R / 20.0
    f[9] = np.log10(iteration + 1.0) / 4.0
    f[10] = np.log1p(last_sigma) / np.log1p(32.0)
    f[11] = float(last_accept)
    return f
