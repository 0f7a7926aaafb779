"""Learned extrapolation step for CP_ALS: data collection, training and the
ALS driver.  All arithmetic runs in the library's kernels (ALS sweeps, step
features, exact costs of extrapolated models, the network's forward pass,
gradients and Adam updates); this module only sequences the calls and keeps
the per-sweep bookkeeping (cost history, stopping test, statistics).

Training data come from ALS trajectories: after sweep k from A_start to A, the
label is the step size sigma* in SIGMA_GRID that minimises the exact cost of
A + sigma (A - A_start) (sigma = 0 is the plain step).  Half of the
trajectories are plain ALS; the other half take the labelled extrapolation
whenever it lowers the cost (accept-if-lower, as the learned step does at
inference), so the network also sees the states that extrapolated runs visit.

Usage (trains on seeded synthetic tensors and writes the parameters):
    python -m paper_1204_1586_amd.learned --tensors 200 --inits 10 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import _lib as L

SIGMA_GRID = (0.0, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0)
SIGMA_MAX = 64.0
N_HIDDEN = 32


def init_params(seed=0, n_in=L.NFEAT, n_hidden=N_HIDDEN):
    """Seeded initial parameters: scaled Gaussian weights, zero hidden biases,
    output bias -3 (initial proposal sigma_max * sigmoid(-3), about 0.76)."""
    g = np.random.default_rng(np.random.SeedSequence([1204, 1586, 77, seed]))
    W1 = g.standard_normal((n_hidden, n_in)) / np.sqrt(n_in)
    W2 = g.standard_normal((n_hidden, n_hidden)) / np.sqrt(n_hidden)
    w3 = g.standard_normal(n_hidden) / np.sqrt(n_hidden) * 0.1
    p = np.concatenate([W1.ravel(), np.zeros(n_hidden), W2.ravel(), np.zeros(n_hidden), w3, [-3.0]])
    return p.astype(np.float32)


def new_network(params=None, seed=0):
    m = L.cpmlp_create(L.NFEAT, N_HIDDEN, SIGMA_MAX)
    L.cpmlp_set_params(m, init_params(seed) if params is None else params)
    return m


def collect_trajectory(plan, Y, A, sweeps, label_every=3, grid=SIGMA_GRID, follow=False):
    """ALS from A (updated in place) for `sweeps` sweeps; every `label_every`
    sweeps one (features, best sigma) pair.  With `follow`, the labelled
    extrapolation is then taken (it lowers the exact cost by construction).
    Returns (X, T, fits)."""
    feat = torch.empty(L.NFEAT, dtype=torch.float32, device="cuda")
    X, T, fits, costs = [], [], [], []
    last_sigma, last_acc = 0.0, 0
    for k in range(sweeps):
        A_start = [a.clone() for a in A]
        cost, fit = L.cpals_step(plan, Y, A)
        costs.append(cost)
        fits.append(fit)
        L.cpals_features(plan, A, A_start, costs, k, last_sigma, last_acc, feat)
        last_sigma, last_acc = 0.0, 0
        if k >= 2 and k % label_every == 0:
            best_s, best_c = 0.0, cost
            for s in grid[1:]:
                c, _ = L.cp_fit_extrapolated(plan, Y, A, A_start, s)
                if np.isfinite(c) and c < best_c:
                    best_s, best_c = s, c
            X.append(feat.cpu().numpy().copy())
            T.append(best_s)
            last_sigma, last_acc = best_s, int(best_s > 0)
            if follow and best_s > 0:
                # the plan's last cost is the sweep's (cp_fit_extrapolated keeps it)
                L.cp_fit(plan, Y, A)
                c, f, acc = L.cpals_extrapolate(plan, Y, A, A_start, best_s)
                costs[-1], fits[-1] = c, f
                last_acc = acc
    return (np.array(X, dtype=np.float32).reshape(-1, L.NFEAT), np.array(T, dtype=np.float32), fits)


def train(mlp, X, T, epochs=30, batch=256, lr=3e-3, seed=0, log=None):
    """Adam on (X, T) with the library's training kernels; returns per-epoch loss."""
    g = np.random.default_rng(seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).cuda()
    n = Xd.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(n)).cuda()
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            xb, tb = Xd[idx].contiguous(), Td[idx].contiguous()
            tot += L.cpmlp_train_step(mlp, xb, tb, lr) * xb.shape[0]
        hist.append(tot / n)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def run_als(plan, Y, A, tol=1e-6, max_sweeps=5000, mlp=None, target_fit=None):
    """ALS from A (updated in place) until |fit_k - fit_{k-1}| < tol (or, with
    target_fit, until the fit reaches it); with a network, each sweep is a
    learned-extrapolation step.  Returns statistics."""
    costs, fits = [], []
    last_sigma, last_acc, accepted, proposals = 0.0, 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(max_sweeps):
        if mlp is None:
            cost, fit = L.cpals_step(plan, Y, A)
        else:
            cost, fit, acc, sg = L.cpals_learned_step(plan, mlp, Y, A, costs, k, last_sigma, last_acc)
            proposals += 1
            accepted += acc
            last_sigma, last_acc = sg, acc
        costs.append(cost)
        fits.append(fit)
        if target_fit is not None and fit >= target_fit:
            break
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    wall = time.perf_counter() - t0
    return {"sweeps": len(fits), "fit": fits[-1], "wall_s": wall, "converged": len(fits) < max_sweeps,
            "accept_rate": (accepted / proposals) if proposals else None,
            "fallback_rate": (1 - accepted / proposals) if proposals else None}


def _problem(w, rep, dims=None, rank=None):
    import cpgen
    return cpgen.make_problem(w, rep=rep, dims=dims, rank=rank)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cp4d_40x70_learned")
    ap.add_argument("--dims", default=None, help="override dims, e.g. 20,25,30,35")
    ap.add_argument("--tensors", type=int, default=200)
    ap.add_argument("--inits", type=int, default=10)
    ap.add_argument("--sweeps", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--label-every", type=int, default=2)
    ap.add_argument("--out", default="learned_step.npz")
    args = ap.parse_args()
    import cpgen
    dims = tuple(int(x) for x in args.dims.split(",")) if args.dims else None
    Xs, Ts = [], []
    t0 = time.time()
    for t in range(args.tensors):
        pr = cpgen.make_problem(args.workload, rep=t, dims=dims)
        Y = torch.from_numpy(pr["y"]).cuda()
        plan = L.cpgrad_plan(pr["dims"], pr["R"], "f32", "f32")
        L.cpgrad_bind(plan, Y)
        for i in range(args.inits):
            g = np.random.default_rng(np.random.SeedSequence([1204, 1586, 5, t, i]))
            A = [torch.tensor(g.standard_normal((I, pr["R"])), dtype=torch.float32).cuda() for I in pr["dims"]]
            X, T, _ = collect_trajectory(plan, Y, A, args.sweeps, label_every=args.label_every,
                                         follow=(i % 2 == 1))
            Xs.append(X)
            Ts.append(T)
        print(f"tensor {t + 1}/{args.tensors} R={pr['R']} samples={sum(len(x) for x in Xs)} "
              f"{time.time() - t0:.0f}s", flush=True)
    X, T = np.concatenate(Xs), np.concatenate(Ts)
    mlp = new_network()
    hist = train(mlp, X, T, epochs=args.epochs, log=lambda s: print(s, flush=True))
    np.savez(args.out, params=L.cpmlp_get_params(mlp), loss=np.array(hist), n_samples=len(T),
             trajectories=args.tensors * args.inits, sigma_hist=np.bincount(
                 np.searchsorted(np.array(SIGMA_GRID), T), minlength=len(SIGMA_GRID)))
    print(json.dumps({"samples": int(len(T)), "trajectories": args.tensors * args.inits,
                      "final_loss": hist[-1]}), flush=True)


if __name__ == "__main__":
    main()
