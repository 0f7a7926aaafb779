"""Allocation-free all-mode gradient (cpgrad_all_modes_noalloc) against the
planned entry point (cpgrad_all_modes) on the same inputs: two calls in a row
through the shared static scratch array, the second on a smaller tensor, then
a shape whose workspace exceeds the array, which must be refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import exact_factors, exact_tensor, problem, rel_fro, to_device_factors, to_device_y

pytestmark = pytest.mark.gpu


def _planned(dims, R, Y, A):
    import paper_1204_1586_amd as P
    G = [torch.empty_like(M) for M in A]
    plan = P.cpgrad_plan(dims, R, "f32", "f32")
    P.cpgrad_all_modes(plan, Y, A, G)
    torch.cuda.synchronize()
    info = P.cpgrad_plan_info(plan)
    return [g.cpu().double().numpy() for g in G], info["workspace_bytes"]


def test_noalloc_matches_planned_twice_then_smaller():
    import paper_1204_1586_amd as P
    for seed, (dims, R) in enumerate([((64, 64, 64, 64), 16), ((20, 30, 40, 50), 7)]):
        print(f"[noalloc] dims={dims} R={R}", flush=True)
        pr = problem(dims, R, "f32", seed=seed + 70)
        Y = to_device_y(pr["y"], "f32")
        A = to_device_factors(pr["init"], "f32")
        G = [torch.full_like(M, float("nan")) for M in A]
        P.cpgrad_all_modes_noalloc(dims, R, Y, A, G)
        torch.cuda.synchronize()
        got = [g.cpu().double().numpy() for g in G]
        ref, ws = _planned(dims, R, Y, A)
        assert ws <= P.NOALLOC_SCRATCH_BYTES
        for n in range(len(dims)):
            # same kernels, same tiling, fixed-order reductions: identical bits
            assert np.array_equal(got[n], ref[n]), (dims, n, float(np.max(np.abs(got[n] - ref[n]))))
        if np.prod(dims) <= 2_000_000:
            orc = O.cp_gradient_all(exact_tensor(pr["y"], "f32", dims), exact_factors(A))
            for n in range(len(dims)):
                assert rel_fro(got[n], orc[n]) <= 1e-5, (n, rel_fro(got[n], orc[n]))


def test_noalloc_refuses_shape_beyond_scratch():
    import paper_1204_1586_amd as P
    dims, R = (64, 64, 64, 64), 64      # split partials alone need 2 x 16 MiB
    Y = torch.zeros(dims, dtype=torch.float32, device="cuda")
    A = [torch.zeros(d, R, dtype=torch.float32, device="cuda") for d in dims]
    G = [torch.zeros_like(M) for M in A]
    with pytest.raises(P.CpgError) as e:
        P.cpgrad_all_modes_noalloc(dims, R, Y, A, G)
    assert e.value.status == -7
    torch.cuda.synchronize()
    assert all(float(g.abs().max()) == 0.0 for g in G)
