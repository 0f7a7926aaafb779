"""Pins for the float64 network reference: finite differences, closed forms
and a textbook Adam step.  CPU only."""
import numpy as np
import pytest

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


def test_features_max_mode_and_last_sigma():
    """f[5] is the largest per-mode update ratio, f[10] the last step size on a
    log(1 + sigma) / log(33) scale; the middle cost decreases f[1], f[2]."""
    A = [np.array([[2.0, 0.0]]), np.array([[0.0, 3.0]])]
    As = [np.array([[1.0, 0.0]]), np.array([[0.0, 1.0]])]
    f = M.step_features(A, As, None, [10.0, 5.0, 4.0, 3.9, 3.8], 9, 1.0, 0, 2)
    assert abs(f[5] - np.log10(2.0 / 3.0) / 6) < 1e-15          # max(log10 0.5, log10 2/3)
    assert abs(f[10] - np.log(2.0) / np.log(33.0)) < 1e-15       # sigma = 1
    assert abs(f[1] - np.log10(0.2) / 12) < 1e-15                # 5 -> 4
    assert abs(f[2] - np.log10(0.025) / 12) < 1e-15              # 4 -> 3.9
    assert f[6] == 0.0 and f[7] == 0.0 and f[11] == 0.0          # no previous update, not accepted
    g = M.step_features(A, As, None, [10.0, 5.0], 0, 0.0, 0, 2)
    assert g[10] == 0.0
    # fewer than five costs: the missing decreases count as 1 (log10 1 = 0)
    assert g[0] == 0.0 and g[1] == 0.0 and g[2] == 0.0 and abs(g[3] - np.log10(0.5) / 12) < 1e-15


def test_extrapolate_endpoints_and_hand_case():
    """A + sigma (A - A_start): sigma = 0 is the plain step, sigma = -1 returns
    to the start, and a hand-worked 1 x 2 case (a sign flip fails all three)."""
    A = [np.array([[1.0, 2.0]]), np.array([[-1.0], [0.5]])]
    As = [np.array([[0.0, 4.0]]), np.array([[3.0], [0.5]])]
    for a, b in zip(M.extrapolate(A, As, 0.0), A):
        assert np.array_equal(a, b)
    for a, b in zip(M.extrapolate(A, As, -1.0), As):
        assert np.array_equal(a, b)
    e = M.extrapolate(A, As, 2.0)
    assert np.array_equal(e[0], np.array([[3.0, -2.0]]))          # (1, 2) + 2 (1, -2)
    assert np.array_equal(e[1], np.array([[-9.0], [0.5]]))        # (-1, .5) + 2 (-4, 0)


def _adam_run(grads, lr=0.1):
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    traj = []
    for t, g in enumerate(grads, start=1):
        p, m, v = M.adam_step(p, np.array([g]), m, v, t, lr)
        traj.append(float(p[0]))
    return traj


def test_adam_constant_gradient_moves_lr_per_step():
    """Adam (Kingma and Ba, Algorithm 1): for a constant gradient the bias
    corrections give m_hat = g and v_hat = g^2 at every t, so each step is
    lr * sign(g).  A wrong bias-correction exponent breaks this from t = 2 on."""
    traj = _adam_run([0.3] * 5)
    assert np.allclose(np.diff([0.0] + traj), -0.1, atol=1e-7, rtol=0)   # eps = 1e-8 shifts it by ~3e-9


def test_adam_alternating_gradient_closed_form():
    """Gradients +g, -g: the second moment stays exactly g^2 after correction,
    the first moment after two steps is -(1 - b1)^2 g, corrected by 1 - b1^2,
    so step 2 moves by +lr (1 - b1) / (1 + b1) = +lr / 19 for b1 = 0.9."""
    traj = _adam_run([2.0, -2.0])
    assert abs(traj[0] - (-0.1)) < 1e-9
    assert abs((traj[1] - traj[0]) - 0.1 / 19.0) < 1e-9


def test_adam_gradient_then_zero_closed_form():
    """Gradients g, 0: after two steps m_hat = b1 / (1 + b1) g and
    v_hat = b2 / (1 + b2) g^2, so step 2 moves by
    -lr (b1 / (1 + b1)) / sqrt(b2 / (1 + b2)); with b1 and b2 swapped the
    step would be a different number, so this pins which beta is which."""
    traj = _adam_run([1.5, 0.0])
    expect = -0.1 * (0.9 / 1.9) / np.sqrt(0.999 / 1.999)
    swapped = -0.1 * (0.999 / 1.999) / np.sqrt(0.9 / 1.9)
    assert abs((traj[1] - traj[0]) - expect) < 1e-9
    assert abs(expect - swapped) > 1e-3


def test_pins_catch_planted_mistakes(monkeypatch):
    """Each pin above fails for a plausible mistake planted in the reference:
    the betas swapped, the bias-correction exponent off by one, and the sign of
    the extrapolation flipped."""
    orig_adam = M.adam_step

    def swapped(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        return orig_adam(p, g, m, v, t, lr, b2, b1, eps)

    def exponent(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        return p - lr * (m / (1 - b1 ** (t + 1))) / (np.sqrt(v / (1 - b2 ** (t + 1))) + eps), m, v

    def flipped(A, A_start, sigma):
        return [a + sigma * (s - a) for a, s in zip(A, A_start)]

    for planted, pin in [(swapped, test_adam_gradient_then_zero_closed_form),
                         (exponent, test_adam_constant_gradient_moves_lr_per_step),
                         (exponent, test_adam_alternating_gradient_closed_form)]:
        monkeypatch.setattr(M, "adam_step", planted)
        with pytest.raises(AssertionError):
            pin()
    monkeypatch.setattr(M, "adam_step", orig_adam)
    monkeypatch.setattr(M, "extrapolate", flipped)
    with pytest.raises(AssertionError):
        test_extrapolate_endpoints_and_hand_case()
