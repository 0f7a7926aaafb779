"""Learned extrapolation step on the GPU: the network's forward pass,
gradients and Adam step against the float64 reference; the step features,
the exact cost of an extrapolated model and the accept-only-if-lower rule;
and the gain of a trained network over plain ALS."""
import numpy as np
import pytest
import torch

import cpgen
import oracle as O
from oracle import mlp_oracle as MO
from gpu_util import exact_factors, exact_tensor, rel_fro, to_device_factors, to_device_y

pytestmark = pytest.mark.gpu

F, H, SMAX = 12, 32, 16.0


def _net(seed=0):
    import paper_1204_1586_amd as P
    g = np.random.default_rng(seed)
    p = (g.standard_normal(MO.mlp_nparams(F, H)) * 0.3).astype(np.float32)
    m = P.cpmlp_create(F, H, SMAX)
    P.cpmlp_set_params(m, p)
    return P, m, p


def test_forward_and_gradient_match_reference():
    P, m, p = _net(1)
    g = np.random.default_rng(2)
    B = 300   # spans several blocks of the gradient kernel and a ragged tail
    X = g.standard_normal((B, F)).astype(np.float32)
    T = (np.abs(g.standard_normal(B)) * 4).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    sig = torch.empty(B, device="cuda")
    P.cpmlp_forward(m, Xd, sig)
    ref = MO.mlp_forward(p, X, F, H, SMAX)
    assert np.max(np.abs(sig.cpu().numpy() - ref) / (np.abs(ref) + 1e-6)) < 1e-5
    grad = torch.empty(P.cpmlp_num_params(m), device="cuda")
    loss = P.cpmlp_gradients(m, Xd, Td, grad)
    lref, gref = MO.mlp_loss_grad(p, X, T, F, H, SMAX)
    assert abs(loss - lref) <= 1e-5 * lref
    gd = grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gd - gref)) <= 1e-4 * np.max(np.abs(gref))
    assert rel_fro(gd, gref) < 1e-5


def test_adam_step_matches_reference():
    P, m, p = _net(3)
    g = np.random.default_rng(4)
    X = g.standard_normal((64, F)).astype(np.float32)
    T = (np.abs(g.standard_normal(64)) * 2).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p64, mm, vv = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t in range(1, 4):
        P.cpmlp_train_step(m, Xd, Td, 1e-2)
        _, gr = MO.mlp_loss_grad(p64, X, T, F, H, SMAX)
        p64, mm, vv = MO.adam_step(p64, gr, mm, vv, t, 1e-2)
        got = P._lib.cpmlp_get_params(m).astype(np.float64)
        assert np.max(np.abs(got - p64)) < 2e-4
        p64 = got   # continue from the device's parameters


def _als_problem(dims=(12, 10, 14, 9), R=4, seed=0):
    import paper_1204_1586_amd as P
    pr = cpgen.make_problem("cp4d_40x70_learned", rep=3000 + seed, dims=dims, rank=R)
    Y = to_device_y(pr["y"], "f32")
    A = to_device_factors(pr["init"], "f32")
    plan = P.cpgrad_plan(dims, R, "f32", "f32")
    P.cpgrad_bind(plan, Y)
    return P, pr, Y, A, plan


def test_features_match_reference():
    P, pr, Y, A, plan = _als_problem()
    feat = torch.empty(P.NFEAT, device="cuda")
    costs, D_prev = [], None
    for k in range(3):
        As = [a.clone() for a in A]
        cost, _ = P.cpals_step(plan, Y, A)
        costs.append(cost)
        P.cpals_features(plan, A, As, costs, k, 0.5 * k, k % 2, feat)
        Ax, Asx = exact_factors(A), exact_factors(As)
        ref = MO.step_features(Ax, Asx, D_prev, costs, k, 0.5 * k, k % 2, pr["R"])
        assert np.allclose(feat.cpu().numpy(), ref, rtol=1e-5, atol=1e-6), (k, feat.cpu().numpy(), ref)
        D_prev = [a - s for a, s in zip(Ax, Asx)]


@pytest.mark.parametrize("sigma", [0.0, 0.7, 4.0])
def test_fit_of_extrapolated_model(sigma):
    P, pr, Y, A, plan = _als_problem(seed=1)
    As = [a.clone() for a in A]
    P.cpals_step(plan, Y, A)
    cost, fit = P.cp_fit_extrapolated(plan, Y, A, As, sigma)
    Yx = exact_tensor(pr["y"], "f32", pr["dims"])
    D = O.cost_explicit(Yx, MO.extrapolate(exact_factors(A), exact_factors(As), sigma))
    scale = max(D, O.norm2(Yx))   # the cost is formed from terms of this size
    assert abs(cost - D) <= 1e-5 * scale, (cost, D)


def test_learned_step_never_worse_than_plain_step():
    """Accept only if the exact cost drops: each learned step's cost is the
    minimum of the plain sweep's cost and the extrapolated model's cost."""
    import paper_1204_1586_amd as P
    from paper_1204_1586_amd import learned
    _, pr, Y, A, plan = _als_problem(seed=2)
    y2 = O.norm2(exact_tensor(pr["y"], "f32", pr["dims"]))
    net = learned.new_network(seed=1)
    feat_costs, last_s, last_a = [], 0.0, 0
    for k in range(12):
        B = [a.clone() for a in A]
        As = [a.clone() for a in A]
        c_plain, _ = P.cpals_step(plan, Y, B)
        # the same model's cost through the other contraction: equal up to float32 rounding of <Y, Yhat>
        c_ext, _ = P.cp_fit_extrapolated(plan, Y, B, As, 0.0)
        assert abs(c_ext - c_plain) <= 1e-6 * y2
        cost, fit, acc, sg = P.cpals_learned_step(plan, net, Y, A, feat_costs, k, last_s, last_a)
        assert cost <= c_plain * (1 + 1e-12)
        if acc:
            assert cost < c_plain
        feat_costs.append(cost)
        last_s, last_a = sg, acc


def test_trained_network_gains_over_plain_als():
    """Train on ALS trajectories of small collinear (congruence 0.9) tensors
    (half plain, half following the labelled extrapolation), then on held-out
    tensors run plain ALS to |delta fit| < 1e-6 and the learned-step ALS until
    it reaches the plain run's final fit (to 1e-6): the learned run must get
    there (no early stall at a worse fit), in fewer sweeps and less wall time
    (each learned sweep pays an extra pass over Y for the exact cost)."""
    import paper_1204_1586_amd as P
    from paper_1204_1586_amd import learned
    dims = (20, 25, 30, 35)
    Xs, Ts = [], []
    for t in range(10):
        pr = cpgen.make_problem("cp4d_40x70_learned", rep=t, dims=dims, rank=8 + t % 5)
        Y = to_device_y(pr["y"], "f32")
        plan = P.cpgrad_plan(dims, pr["R"], "f32", "f32")
        P.cpgrad_bind(plan, Y)
        for i in range(4):
            g = np.random.default_rng([7, t, i])
            A = [torch.tensor(g.standard_normal((I, pr["R"])), dtype=torch.float32).cuda() for I in dims]
            X, T, _ = learned.collect_trajectory(plan, Y, A, 45, label_every=2, follow=(i % 2 == 1))
            Xs.append(X)
            Ts.append(T)
    net = learned.new_network()
    learned.train(net, np.concatenate(Xs), np.concatenate(Ts), epochs=40)
    plain, learn, tp, tl = [], [], 0.0, 0.0
    for t in range(4):
        pr = cpgen.make_problem("cp4d_40x70_learned", rep=10000 + t, dims=dims, rank=8 + 2 * t)
        Y = to_device_y(pr["y"], "f32")
        plan = P.cpgrad_plan(dims, pr["R"], "f32", "f32")
        P.cpgrad_bind(plan, Y)
        A0 = to_device_factors(pr["init"], "f32")
        r0 = learned.run_als(plan, Y, [a.clone() for a in A0], max_sweeps=3000)
        target = r0["fit"] - 1e-6
        r1 = learned.run_als(plan, Y, [a.clone() for a in A0], tol=0.0, max_sweeps=3000, mlp=net, target_fit=target)
        print(f"  held-out {t}: R={pr['R']} plain {r0['sweeps']} sweeps {r0['wall_s'] * 1e3:.1f} ms fit "
              f"{r0['fit']:.7f} | learned {r1['sweeps']} sweeps {r1['wall_s'] * 1e3:.1f} ms fit {r1['fit']:.7f} "
              f"accept {r1['accept_rate']:.2f}", flush=True)
        assert r1["fit"] >= target, (r1["fit"], target)
        plain.append(r0["sweeps"])
        learn.append(r1["sweeps"])
        tp += r0["wall_s"]
        tl += r1["wall_s"]
    print(f"  sweep ratio {np.sum(learn) / np.sum(plain):.3f}, time ratio {tl / tp:.3f}", flush=True)
    assert np.mean(learn) < 0.8 * np.mean(plain)
    assert tl < tp


@pytest.mark.parametrize("sigma", [0.0, 0.5, 3.0, 40.0])
def test_extrapolate_with_host_sigma_accepts_only_if_lower(sigma):
    """cpals_extrapolate: the exact cost of A_new + sigma (A_new - A_prev) against
    the oracle's explicit residual; A_new replaced exactly when that cost is
    below the last sweep's (accept-if-lower), and the returned cost is the
    kept model's."""
    import paper_1204_1586_amd as P
    _, pr, Y, A, plan = _als_problem(seed=3)
    Yx = exact_tensor(pr["y"], "f32", pr["dims"])
    y2 = O.norm2(Yx)
    for _ in range(3):
        P.cpals_step(plan, Y, A)
    A_prev = [a.clone() for a in A]
    c_new, _ = P.cpals_step(plan, Y, A)
    before = exact_factors(A)
    cost, fit, acc = P.cpals_extrapolate(plan, Y, A, A_prev, sigma)
    D_ext = O.cost_explicit(Yx, MO.extrapolate(before, exact_factors(A_prev), sigma))
    after = exact_factors(A)
    print(f"  sigma {sigma}: plain {c_new:.6e} extrapolated {D_ext:.6e} accepted {acc}", flush=True)
    if acc:
        assert D_ext < c_new + 1e-6 * y2
        assert abs(cost - D_ext) <= 1e-5 * y2
        ext = MO.extrapolate(before, exact_factors(A_prev), sigma)
        for a, b in zip(after, ext):
            assert np.allclose(a, b, rtol=1e-6, atol=1e-6)
    else:
        assert D_ext > c_new - 1e-6 * y2
        assert cost == c_new
        for a, b in zip(after, before):
            assert np.array_equal(a, b)
    if sigma == 0.0:
        # the same model: accepting it or not leaves the factors as they were
        # (the two evaluations of its cost differ only by float32 rounding)
        for a, b in zip(after, before):
            assert np.array_equal(a, b)
