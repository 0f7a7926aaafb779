"""Pins for the float64 network reference: finite differences, closed forms
and a textbook Adam step.  CPU only."""
import numpy as np

from oracle import mlp_oracle as M


def _params(F, H, seed, scale=0.5):
    return np.random.default_rng(seed).standard_normal(M.mlp_nparams(F, H)) * scale


def test_backprop_matches_central_differences():
    F, H, smax = 12, 8, 16.0
    p = _params(F, H, 1)
    g = np.random.default_rng(2)
    X = g.standard_normal((7, F))
    t = np.abs(g.standard_normal(7)) * 3
    loss, grad = M.mlp_loss_grad(p, X, t, F, H, smax)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (M.mlp_loss_grad(p + e, X, t, F, H, smax)[0] - M.mlp_loss_grad(p - e, X, t, F, H, smax)[0]) / (2 * h)
    assert np.max(np.abs(num - grad)) <= 1e-7 * max(1.0, np.max(np.abs(grad)))
    assert abs(loss - np.mean((np.log1p(M.mlp_forward(p, X, F, H, smax)) - np.log1p(t)) ** 2)) < 1e-15


def test_zero_network_gives_half_sigma_max():
    F, H = 12, 32
    p = np.zeros(M.mlp_nparams(F, H))
    X = np.random.default_rng(3).standard_normal((5, F))
    assert np.allclose(M.mlp_forward(p, X, F, H, 16.0), 8.0)


def test_output_bias_only():
    F, H, smax = 4, 3, 10.0
    p = np.zeros(M.mlp_nparams(F, H))
    p[-1] = 2.0                      # b3
    s = M.mlp_forward(p, np.ones((1, F)), F, H, smax)[0]
    assert abs(s - smax / (1 + np.exp(-2.0))) < 1e-14


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = M.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.1)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.1 * np.sign(g), atol=1e-6)


def test_features_simple_case():
    A = [np.array([[2.0, 0.0]]), np.array([[0.0, 3.0]])]
    As = [np.array([[1.0, 0.0]]), np.array([[0.0, 1.0]])]
    D = [np.array([[1.0, 0.0]]), np.array([[0.0, -1.0]])]
    f = M.step_features(A, As, D, [10.0, 5.0, 4.0, 3.9, 3.8], 9, 1.0, 1, 2)
    assert abs(f[0] - np.log10(0.5) / 12) < 1e-15           # 10 -> 5
    assert abs(f[3] - np.log10(0.1 / 3.9) / 12) < 1e-12     # 3.9 -> 3.8
    # update norms: |(1,0)|/|(2,0)| = 0.5, |(0,2)|/|(0,3)| = 2/3
    assert abs(f[4] - (np.log10(0.5) + np.log10(2 / 3)) / 2 / 6) < 1e-14
    assert f[6] == 0.0 and f[7] == -1.0                      # cosines +1 and -1
    assert f[8] == 0.1 and abs(f[9] - 0.25) < 1e-15 and f[11] == 1.0
