"""GPU parity of the further uses of the fast gradients, through the C ABI,
against the float64 oracle on identical seeded inputs:
  cpgrad_e_gradient     the full gradient of eq. 2.13 (without -2), all modes;
  cpgrad_mode_gradient  one mode's gradient by Section 3.2 (direction by
                        J_n <= K_{n-1});
  cpntf_step            the multiplicative nonnegative sweep of eq. 2.18."""
import numpy as np
import pytest
import torch

import cpgen
import oracle as O
from gpu_util import (ENTRY_BOUND, FRO_TOL, check_gradients, exact_factors, exact_tensor, factor_storage,
                      magnitude_gradients, problem, rel_fro, to_device_factors, to_device_y)

pytestmark = pytest.mark.gpu


def _setup(dims, R, storage, mode="native", seed=0):
    import paper_1204_1586_amd as P
    pr = problem(dims, R, storage, seed=seed)
    fst = factor_storage(storage)
    Y = to_device_y(pr["y"], storage)
    A = to_device_factors(pr["init"], fst)
    plan = P.cpgrad_plan(dims, R, storage, fst, mode)
    return P, pr, Y, A, plan


@pytest.mark.parametrize("dims,R,storage", [((20, 20, 20), 3, "f64"), ((9, 8, 7, 6), 5, "f64"),
                                            ((20, 30, 40, 50), 16, "f32"), ((6, 5, 4, 6, 5, 4, 6), 10, "f32"),
                                            ((4, 65, 300), 5, "f32"), ((9, 70, 130), 33, "f32")])
def test_e_gradient_matches_oracle(dims, R, storage):
    """E^(n) = G^(n) - A^(n) Gamma^(n): every entry within the rounding bound of
    its two parts, |dE| <= c (Gabs + |A^(n)| |Gamma^(n)|), and the Frobenius error
    within the form's tolerance of ||G|| + ||A Gamma||."""
    print(f"[e_gradient] dims={dims} R={R} storage={storage}", flush=True)
    P, pr, Y, A, plan = _setup(dims, R, storage)
    E = [torch.empty_like(M) for M in A]
    P.cpgrad_e_gradient(plan, Y, A, E)
    torch.cuda.synchronize()
    Yx = exact_tensor(pr["y"], storage, dims)
    Ax = exact_factors(A)
    ref = O.e_gradient_all(Yx, Ax)
    gabs = magnitude_gradients(Yx, Ax)
    for n in range(len(dims)):
        Gam = O.gamma(Ax, n)
        scale = gabs[n] + np.abs(Ax[n]) @ np.abs(Gam)
        d = np.abs(E[n].cpu().double().numpy() - ref[n])
        assert np.all(d <= ENTRY_BOUND[storage] * scale + 1e-300), (n, float(np.max(d / scale)))
        fro = np.linalg.norm(d) / (np.linalg.norm(O.mttkrp(Yx, Ax, n)) + np.linalg.norm(Ax[n] @ Gam))
        assert fro <= FRO_TOL[storage], (n, fro)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_e_gradient_vanishes_at_exact_model(storage):
    """Y = [[A]] (no noise): the full gradient of eq. 2.13 is zero, so E is
    rounding error of the size of the gradient's own rounding."""
    import paper_1204_1586_amd as P
    dims, R = (12, 10, 14, 9), 4
    g = np.random.default_rng(21)
    truth = [g.standard_normal((I, R)) for I in dims]
    y = cpgen.noisy_cp_tensor(truth, None, g, storage)
    fst = factor_storage(storage)
    Y = to_device_y(y, storage)
    A = to_device_factors(truth, fst)
    E = [torch.empty_like(M) for M in A]
    plan = P.cpgrad_plan(dims, R, storage, fst)
    P.cpgrad_e_gradient(plan, Y, A, E)
    torch.cuda.synchronize()
    Ax = exact_factors(A)
    Yx = exact_tensor(y, storage, dims)
    for n in range(4):
        G = O.mttkrp(Yx, Ax, n)
        rel = float(torch.linalg.norm(E[n].double()).item() / np.linalg.norm(G))
        # float32: Y itself was rounded to float32, so [[A]] fits it only to u_32 ||Y||
        assert rel <= FRO_TOL[storage], (n, rel)


@pytest.mark.parametrize("dims,R,storage", [((20, 30, 40, 50), 16, "f32"), ((6, 5, 4, 6, 5, 4, 6), 10, "f32"),
                                            ((9, 8, 7, 6, 5), 4, "f64"), ((4, 65, 300), 5, "f32"),
                                            ((100, 77), 5, "f32"), ((8, 10, 8, 6, 4), 8, "bf16")])
def test_mode_gradient_matches_oracle_and_picks_the_cheaper_side(dims, R, storage):
    """Each mode's gradient from one pass over Y, element by element, and the
    direction taken is Section 3.2's: right to left iff J_n <= K_{n-1} (mode 1
    always right to left, mode N always left to right)."""
    mode = "bf16_refined" if storage == "bf16" else "native"
    print(f"[mode_gradient] dims={dims} R={R} storage={storage}", flush=True)
    P, pr, Y, A, plan = _setup(dims, R, storage, mode)
    N = len(dims)
    Yx = exact_tensor(pr["y"], storage, dims)
    Ax = exact_factors(A)
    ref = O.cp_gradient_all(Yx, Ax)
    gabs = magnitude_gradients(Yx, Ax)
    got = []
    for n in range(1, N + 1):
        G = torch.empty_like(A[n - 1])
        d = P.cpgrad_mode_gradient(plan, Y, A, n, G)
        J = int(np.prod(dims[:n]))
        Km1 = int(np.prod(dims[n - 1:]))
        want_right = n == 1 or (n <= N - 1 and J <= Km1)
        if storage != "bf16":
            assert d == (0 if want_right else 1), (n, d)
        torch.cuda.synchronize()
        got.append(G.cpu().double().numpy())
    form = "bf16_refined" if storage == "bf16" else storage
    check_gradients(got, ref, gabs, form, label=f"{dims}")


def _ntf_setup(dims, R, storage, rep):
    import paper_1204_1586_amd as P
    pr = cpgen.make_nonnegative_problem(dims, R, rep=rep, storage=storage)
    Y = to_device_y(pr["y"], storage)
    A = to_device_factors(pr["init"], storage)
    plan = P.cpgrad_plan(dims, R, storage, storage)
    P.cpgrad_bind(plan, Y)
    return P, pr, Y, A, plan


@pytest.mark.parametrize("dims,R,storage", [((20, 30, 40, 50), 8, "f32"), ((10, 12, 9, 11, 8), 5, "f64"),
                                            ((6, 5, 4, 6, 5, 4, 6), 6, "f32"), ((30, 40, 50), 20, "f32")])
def test_ntf_sweep_matches_oracle(dims, R, storage):
    """One sweep of eq. 2.18 from the same nonnegative start.  With nonnegative
    data and factors every sum has nonnegative terms, so each gradient entry
    is accurate to c G(i,r) (c = the rounding bound) and each update
    A G / (A Gamma) to about 2c relatively; errors of the modes updated
    earlier in the sweep feed the later ones: tol = 2 N c per entry."""
    print(f"[ntf] dims={dims} R={R} storage={storage}", flush=True)
    P, pr, Y, A, plan = _ntf_setup(dims, R, storage, rep=1)
    A0 = exact_factors(A)
    cost, fit = P.cpntf_step(plan, Y, A)
    Yx = exact_tensor(pr["y"], storage, dims)
    A_ref, D_ref, fit_ref = O.ntf_sweep(Yx, A0)
    A_gpu = exact_factors(A)
    tol = 2 * len(dims) * ENTRY_BOUND[storage]
    worst = 0.0
    for n in range(len(dims)):
        assert np.all(A_gpu[n] >= 0)
        rel = np.abs(A_gpu[n] - A_ref[n]) / np.maximum(np.abs(A_ref[n]), 1e-300)
        worst = max(worst, float(rel.max()))
        assert np.all(rel <= tol), (n, float(rel.max()))
    D = O.cost_explicit(Yx, A_gpu)
    print(f"  max entry rel err {worst:.1e} (tol {tol:.1e}); cost vs explicit {abs(cost - D) / O.norm2(Yx):.1e}; "
          f"fit vs oracle {abs(fit - fit_ref):.1e}", flush=True)
    assert abs(cost - D) <= tol * O.norm2(Yx)
    assert abs(fit - fit_ref) <= tol


def test_ntf_sweeps_never_raise_the_cost_64_4():
    """Eight multiplicative sweeps on a 64^4 nonnegative float32 tensor, rank
    10: the cost never rises (to float32 rounding of the cost identity) and the
    factors stay nonnegative."""
    dims, R = (64, 64, 64, 64), 10
    print(f"[ntf x8] dims={dims} R={R}", flush=True)
    P, pr, Y, A, plan = _ntf_setup(dims, R, "f32", rep=2)
    y2 = float(np.sum(pr["y"].astype(np.float64) ** 2))
    costs = [P.cpntf_step(plan, Y, A)[0] for _ in range(8)]
    print("  costs/||Y||^2: " + " ".join(f"{c / y2:.6e}" for c in costs), flush=True)
    for a, b in zip(costs, costs[1:]):
        assert b <= a + 1e-6 * y2
    assert all(float(M.min()) >= 0.0 for M in A)
    assert costs[-1] < 0.9 * costs[0]   # the multiplicative rule descends slowly (measured 0.76 after 8 sweeps)
