"""C-ABI library on the host: it loads, exports every function the header
declares, rejects bad arguments before touching a device, and its host-only
planner agrees with the paper's n* rule and with an independent flop tally.
No GPU needed (no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1204_1586_amd as P

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include")


def _declared():
    text = "".join(open(os.path.join(INCLUDE, h)).read() for h in sorted(os.listdir(INCLUDE)) if h.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_functions_are_all_exported():
    names = _declared()
    assert "cpgrad_all_modes" in names and "cpals_step" in names and "cp_fit" in names
    lib = ctypes.CDLL(P.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.EXPORTS) == names


def _plan_status(N, dims, R, ydt=1, fdt=1, mode=0):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * max(1, len(dims)))(*dims)
    return P.LIB.cpgrad_plan(ctypes.byref(h), N, arr, R, ydt, fdt, mode, None)


@pytest.mark.parametrize("N,dims,R", [
    (1, [5], 3), (17, [2] * 17, 3), (3, [4, 5, 6], 0), (3, [4, 5, 6], 65), (3, [4, 0, 6], 3),
    (3, [4, -1, 6], 3), (4, [2 ** 20, 2 ** 20, 2 ** 20, 2 ** 20], 3),
])
def test_plan_rejects_bad_shapes(N, dims, R):
    assert _plan_status(N, dims, R) == -1


def test_plan_rejects_bad_types():
    assert _plan_status(3, [4, 5, 6], 3, ydt=7) == -1
    assert _plan_status(3, [4, 5, 6], 3, mode=9) == -1
    assert _plan_status(3, [4, 5, 6], 3, ydt=0, fdt=1) == -5      # f64 tensor with f32 factors
    assert _plan_status(3, [4, 5, 6], 3, ydt=2, fdt=1, mode=0) == -5  # bf16 tensor needs a bf16 mode
    assert _plan_status(3, [4, 5, 6], 3, ydt=1, fdt=2) == -5
    assert P.LIB.cpgrad_plan(None, 3, (ctypes.c_int64 * 3)(4, 5, 6), 3, 1, 1, 0, None) == -1


def test_null_handles_are_rejected():
    assert P.LIB.cpgrad_all_modes(None, None, None, None) == -1
    assert P.LIB.cpals_step(None, None, None, None, None) == -1
    assert P.LIB.cp_fit(None, None, None, None, None) == -1
    assert P.LIB.cpgrad_bind(None, None) == -1
    assert P.LIB.cpgrad_set_option(None, 1, 0) == -1
    assert P.LIB.cpgrad_plan_info(None, None, None, None, None) == -1
    assert P.LIB.cpgrad_destroy(None) == 0


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert P.LIB.cpgrad_status_string(s).decode().startswith("CPG_")


@pytest.mark.parametrize("dims", [(20, 20, 20), (64,) * 4, (10,) * 7, (48,) * 5, (40, 50, 60, 70), (100, 2, 2),
                                  (2, 3, 100), (7, 5), (3, 1, 4, 1, 5)])
def test_query_n_star_matches_oracle(dims):
    assert P.cpgrad_query(dims, 3)["n_star"] == O.n_star(dims)


def test_query_force_n_star():
    dims = (6, 5, 4, 3, 2)
    for ns in range(1, 5):
        assert P.cpgrad_query(dims, 3, force_nstar=ns)["n_star"] == ns
    with pytest.raises(P.CpgError):
        P.cpgrad_query(dims, 3, force_nstar=5)


def _tally(dims, R, ns):
    """Independent count of Algorithm 2's multiply-adds: the two big
    contractions (Y once per side), then one pass over each chain tensor per
    chain step and per gradient (eqs. 3.12, 3.16, 3.20, 3.22)."""
    N = len(dims)
    J = [int(np.prod(dims[:n])) for n in range(N + 1)]
    K = [int(np.prod(dims[n:])) for n in range(N + 1)]
    mac = 2 * J[N] * R
    right_sizes = [J[n] for n in range(ns, 0, -1)]               # R^(n) tensors, n = n*..1
    mac += sum(right_sizes) * R + sum(right_sizes[:-1]) * R       # gradients + chain steps
    left_sizes = [K[n - 1] for n in range(ns + 1, N + 1)]        # L^(n) tensors, n = n*+1..N
    mac += sum(left_sizes) * R + sum(left_sizes[:-1]) * R
    return 2 * mac


@pytest.mark.parametrize("dims,R", [((64,) * 4, 16), ((10,) * 7, 10), ((48,) * 5, 32), ((40, 50, 60, 70), 20),
                                    ((20, 20, 20), 3)])
def test_query_flops(dims, R):
    q = P.cpgrad_query(dims, R)
    assert q["alg_flops"] == _tally(dims, R, O.n_star(dims))
    # the O(R prod I_n) claim (Section 1, Table 4.1): at most a few % above 4 R J_N
    assert q["alg_flops"] <= 4 * R * np.prod(dims) * 1.2


def test_noalloc_rejects_bad_arguments_before_any_device_call():
    dims = (ctypes.c_int64 * 3)(4, 5, 6)
    vp = ctypes.c_void_p
    ptrs = (vp * 3)(16, 32, 48)
    f = P.LIB.cpgrad_all_modes_noalloc
    assert f(3, dims, 3, 1, 1, 0, None, ptrs, ptrs, None) == -1                 # NULL Y
    assert f(3, dims, 3, 1, 1, 0, vp(16), None, ptrs, None) == -1               # NULL A
    assert f(3, dims, 3, 1, 1, 0, vp(17), ptrs, ptrs, None) == -1               # misaligned Y
    assert f(1, dims, 3, 1, 1, 0, vp(16), ptrs, ptrs, None) == -1               # N < 2
    assert f(3, dims, 0, 1, 1, 0, vp(16), ptrs, ptrs, None) == -1               # R < 1
    assert f(3, dims, 3, 0, 1, 0, vp(16), ptrs, ptrs, None) == -5               # f64 tensor, f32 factors
    nulls = (vp * 3)(16, None, 48)
    assert f(3, dims, 3, 1, 1, 0, vp(16), nulls, ptrs, None) == -1             # a NULL factor
    assert P.LIB.cpgrad_status_string(-7).decode().startswith("CPG_ERR_SCRATCH")


def test_reduced_precision_mode_is_refused_where_matrix_cores_cannot_run():
    """A bf16 mode never falls back silently to the full-precision kernel: a
    split whose row count J = I_1...I_n* is not a multiple of 8 is refused
    before any device call."""
    assert _plan_status(3, [5, 6, 7], 3, ydt=1, fdt=1, mode=1) == -5        # n* = 1, J = 5
    assert _plan_status(3, [5, 6, 7], 3, ydt=2, fdt=1, mode=2) == -5
    dims = (ctypes.c_int64 * 3)(5, 6, 7)
    vp = ctypes.c_void_p
    ptrs = (vp * 3)(16, 32, 48)
    assert P.LIB.cpgrad_all_modes_noalloc(3, dims, 3, 1, 1, 2, vp(16), ptrs, ptrs, None) == -5
