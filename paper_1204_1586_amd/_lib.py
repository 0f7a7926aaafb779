"""ctypes binding of libcpgrad (include/cpgrad.h): argument marshalling only.

Every call takes torch tensors that live on the GPU, checks their type,
shape and contiguity, and passes raw device pointers to the C ABI.  No step
of the computation runs here; if the shared library is missing the import of
this module raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcpgrad.so")

CPG_F64, CPG_F32, CPG_BF16, CPG_F16 = 0, 1, 2, 3
CPG_MODE_NATIVE, CPG_MODE_BF16, CPG_MODE_BF16_REFINED = 0, 1, 2
CPG_MODE_F16_SCALED, CPG_MODE_F16_SCALED_REFINED = 3, 4
CPG_OPT_FORCE_NSTAR, CPG_OPT_KERNEL, CPG_OPT_PROFILE, CPG_OPT_MFMA_COLS = 1, 2, 3, 4
MAX_MODES, MAX_RANK = 16, 64

STATUS = {0: "CPG_OK", -1: "CPG_ERR_INVALID", -2: "CPG_ERR_NOMEM", -3: "CPG_ERR_HIP", -4: "CPG_ERR_NOT_SPD",
          -5: "CPG_ERR_UNSUPPORTED", -6: "CPG_ERR_NONFINITE", -7: "CPG_ERR_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 32 << 20

DTYPES = {"f64": CPG_F64, "f32": CPG_F32, "bf16": CPG_BF16, "f16": CPG_F16}
MODES = {"native": CPG_MODE_NATIVE, "bf16": CPG_MODE_BF16, "bf16_refined": CPG_MODE_BF16_REFINED,
         "f16_scaled": CPG_MODE_F16_SCALED, "f16_scaled_refined": CPG_MODE_F16_SCALED_REFINED}
TORCH_DTYPE = {CPG_F64: torch.float64, CPG_F32: torch.float32, CPG_BF16: torch.bfloat16, CPG_F16: torch.float16}

EXPORTS = ["cpgrad_plan", "cpgrad_plan_info", "cpgrad_query", "cpgrad_set_option", "cpgrad_profile_read",
           "cpgrad_bind", "cpgrad_all_modes", "cpals_step", "cp_fit", "cpgrad_last_fit", "cpgrad_destroy",
           "cpgrad_status_string", "cpgrad_version",
           "cpmlp_create", "cpmlp_num_params", "cpmlp_set_params", "cpmlp_get_params", "cpmlp_forward",
           "cpmlp_gradients", "cpmlp_train_step", "cpmlp_destroy", "cpals_features", "cp_fit_extrapolated",
           "cpals_learned_step", "cpgrad_all_modes_noalloc", "cpgrad_plan_path", "cpgrad_e_gradient",
           "cpgrad_mode_gradient", "cpntf_step", "cpals_extrapolate"]
NFEAT = 12


class CpgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1204_1586_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "cpgrad_plan": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, vp]),
        "cpgrad_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t),
                                            dp, dp]),
        "cpgrad_plan_path": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "cpgrad_query": (ctypes.c_int, [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), dp, dp]),
        "cpgrad_set_option": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int64]),
        "cpgrad_profile_read": (ctypes.c_int, [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64)]),
        "cpgrad_bind": (ctypes.c_int, [vp, vp]),
        "cpgrad_all_modes": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "cpgrad_all_modes_noalloc": (ctypes.c_int, [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                     ctypes.c_int, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]),
        "cpals_step": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), dp, dp]),
        "cpntf_step": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), dp, dp]),
        "cpgrad_e_gradient": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "cpgrad_mode_gradient": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), ctypes.c_int, vp,
                                                ctypes.POINTER(ctypes.c_int)]),
        "cp_fit": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), dp, dp]),
        "cpgrad_last_fit": (ctypes.c_int, [vp, dp, dp]),
        "cpgrad_destroy": (ctypes.c_int, [vp]),
        "cpgrad_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "cpgrad_version": (ctypes.c_char_p, []),
        "cpmlp_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_float, vp]),
        "cpmlp_num_params": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64)]),
        "cpmlp_set_params": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
        "cpmlp_get_params": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
        "cpmlp_forward": (ctypes.c_int, [vp, vp, ctypes.c_int, vp]),
        "cpmlp_gradients": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp, dp]),
        "cpmlp_train_step": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_float, dp]),
        "cpmlp_destroy": (ctypes.c_int, [vp]),
        "cpals_features": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_float, ctypes.c_int, vp]),
        "cp_fit_extrapolated": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double, dp,
                                               dp]),
        "cpals_extrapolate": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int), dp, dp]),
        "cpals_learned_step": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(vp), dp, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_float, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(status, where):
    if status != 0:
        raise CpgError(status, where)


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


class Plan:
    """Owns a cpgrad_plan_t; the library's plan lives until destroy()/GC."""

    def __init__(self, handle, dims, R, ydt, fdt, mode, stream):
        self.handle = handle
        self.dims = tuple(dims)
        self.R = R
        self.ydt, self.fdt, self.mode = ydt, fdt, mode
        self.stream = stream
        self.bound = None
        self._memo = {}   # call name -> (argument identities, tensors kept alive, marshalled pointers)

    @property
    def N(self):
        return len(self.dims)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            LIB.cpgrad_destroy(h)
            self.handle = None


def _check_y(plan, Y):
    if not (isinstance(Y, torch.Tensor) and Y.is_cuda and Y.is_contiguous()):
        raise ValueError("Y must be a contiguous CUDA tensor")
    if Y.dtype != TORCH_DTYPE[plan.ydt]:
        raise ValueError(f"Y dtype {Y.dtype} does not match the plan ({TORCH_DTYPE[plan.ydt]})")
    n = 1
    for d in plan.dims:
        n *= d
    if Y.numel() != n:
        raise ValueError(f"Y has {Y.numel()} entries, the plan expects {n}")


def _check_factors(plan, A, what="A"):
    if len(A) != plan.N:
        raise ValueError(f"{what} must hold {plan.N} tensors")
    for n, M in enumerate(A):
        if not (isinstance(M, torch.Tensor) and M.is_cuda and M.is_contiguous()):
            raise ValueError(f"{what}[{n}] must be a contiguous CUDA tensor")
        if tuple(M.shape) != (plan.dims[n], plan.R) or M.dtype != TORCH_DTYPE[plan.fdt]:
            raise ValueError(f"{what}[{n}] must be ({plan.dims[n]}, {plan.R}) {TORCH_DTYPE[plan.fdt]}")


def cpgrad_plan(dims, R, y_dtype="f32", factor_dtype=None, mode="native", stream=None):
    """Create a plan (see cpgrad_plan in include/cpgrad.h).  dims[0] = I_1 is the
    fastest mode; ``stream`` defaults to torch's current stream."""
    ydt = DTYPES[y_dtype] if isinstance(y_dtype, str) else int(y_dtype)
    if factor_dtype is None:
        factor_dtype = "f64" if ydt == CPG_F64 else "f32"
    fdt = DTYPES[factor_dtype] if isinstance(factor_dtype, str) else int(factor_dtype)
    md = MODES[mode] if isinstance(mode, str) else int(mode)
    if stream is None:
        stream = torch.cuda.current_stream()
    dims = [int(d) for d in dims]
    arr = (ctypes.c_int64 * len(dims))(*dims)
    h = ctypes.c_void_p()
    _check(LIB.cpgrad_plan(ctypes.byref(h), len(dims), arr, int(R), ydt, fdt, md,
                           ctypes.c_void_p(stream.cuda_stream)), "cpgrad_plan")
    return Plan(h, dims, int(R), ydt, fdt, md, stream)


def cpgrad_plan_info(plan):
    """Returns dict(n_star, workspace_bytes, alg_flops, alg_bytes)."""
    ns, ws = ctypes.c_int(), ctypes.c_size_t()
    fl, by = ctypes.c_double(), ctypes.c_double()
    _check(LIB.cpgrad_plan_info(plan.handle, ctypes.byref(ns), ctypes.byref(ws), ctypes.byref(fl),
                                ctypes.byref(by)), "cpgrad_plan_info")
    return {"n_star": ns.value, "workspace_bytes": ws.value, "alg_flops": fl.value, "alg_bytes": by.value}


def cpgrad_plan_path(plan):
    """dict(kernel: 1 generic / 2 float32 MFMA / 3 bf16 MFMA, fused_reduction: bool)."""
    k, f = ctypes.c_int(), ctypes.c_int()
    _check(LIB.cpgrad_plan_path(plan.handle, ctypes.byref(k), ctypes.byref(f)), "cpgrad_plan_path")
    return {"kernel": k.value, "fused_reduction": bool(f.value)}


def cpgrad_query(dims, R, y_dtype="f32", factor_dtype=None, force_nstar=0):
    """Host-only: dict(n_star, alg_flops, alg_bytes) for a shape (no device needed)."""
    ydt = DTYPES[y_dtype] if isinstance(y_dtype, str) else int(y_dtype)
    if factor_dtype is None:
        factor_dtype = "f64" if ydt == CPG_F64 else "f32"
    fdt = DTYPES[factor_dtype] if isinstance(factor_dtype, str) else int(factor_dtype)
    dims = [int(d) for d in dims]
    arr = (ctypes.c_int64 * max(1, len(dims)))(*dims)
    ns, fl, by = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(LIB.cpgrad_query(len(dims), arr, int(R), ydt, fdt, int(force_nstar), ctypes.byref(ns), ctypes.byref(fl),
                            ctypes.byref(by)), "cpgrad_query")
    return {"n_star": ns.value, "alg_flops": fl.value, "alg_bytes": by.value}


def cpgrad_set_option(plan, option, value):
    _check(LIB.cpgrad_set_option(plan.handle, int(option), int(value)), "cpgrad_set_option")


def cpgrad_profile_read(plan, roles=0):
    """(total_ms, launches) of the big-contraction launches timed since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(LIB.cpgrad_profile_read(plan.handle, int(roles), ctypes.byref(ms), ctypes.byref(n)),
           "cpgrad_profile_read")
    return ms.value, n.value


def cpgrad_bind(plan, Y):
    _check_y(plan, Y)
    _check(LIB.cpgrad_bind(plan.handle, ctypes.c_void_p(Y.data_ptr())), "cpgrad_bind")
    plan.bound = Y


def _marshal(plan, name, Y, lists, checks):
    """Validated, marshalled pointers for (Y, *lists).  A repeat call with the
    very same tensor objects at the same device addresses reuses the last
    result (the memo holds those tensors, so their identities cannot be reused
    while it does; storage moved by resize_ or set_ is validated again)."""
    key = (id(Y), Y.data_ptr()) + tuple(x for ts in lists for t in ts for x in (id(t), t.data_ptr()))
    m = plan._memo.get(name)
    if m is not None and m[0] == key:
        return m[2]
    checks()
    out = (ctypes.c_void_p(Y.data_ptr()),) + tuple(_ptrs(ts) for ts in lists)
    plan._memo[name] = (key, (Y,) + tuple(tuple(ts) for ts in lists), out)
    return out


def cpgrad_all_modes(plan, Y, A, G):
    """G[n] <- Y_(n) (⊙_{k≠n} A^(k)) for all n (asynchronous)."""
    def checks():
        _check_y(plan, Y)
        _check_factors(plan, A)
        _check_factors(plan, G, "G")
    y, a, g = _marshal(plan, "all_modes", Y, (A, G), checks)
    _check(LIB.cpgrad_all_modes(plan.handle, y, a, g), "cpgrad_all_modes")


def cpgrad_all_modes_noalloc(dims, R, Y, A, G, y_dtype="f32", factor_dtype=None, mode="native", stream=None):
    """cpgrad_all_modes without a plan: every intermediate lives in the library's
    static device scratch array (no device allocation; asynchronous)."""
    ydt = DTYPES[y_dtype] if isinstance(y_dtype, str) else int(y_dtype)
    if factor_dtype is None:
        factor_dtype = "f64" if ydt == CPG_F64 else "f32"
    fdt = DTYPES[factor_dtype] if isinstance(factor_dtype, str) else int(factor_dtype)
    md = MODES[mode] if isinstance(mode, str) else int(mode)
    if stream is None:
        stream = torch.cuda.current_stream()
    shape = Plan(None, dims, R, ydt, fdt, md, stream)   # argument checks only (owns no library plan)
    _check_y(shape, Y)
    _check_factors(shape, A)
    _check_factors(shape, G, "G")
    dims = [int(d) for d in dims]
    arr = (ctypes.c_int64 * len(dims))(*dims)
    _check(LIB.cpgrad_all_modes_noalloc(len(dims), arr, int(R), ydt, fdt, md, ctypes.c_void_p(Y.data_ptr()),
                                        _ptrs(A), _ptrs(G), ctypes.c_void_p(stream.cuda_stream)),
           "cpgrad_all_modes_noalloc")


def cpgrad_e_gradient(plan, Y, A, E):
    """E[n] <- Y_(n)(⊙_{k≠n} A^(k)) - A^(n) Gamma^(n) for all n (eq. 2.13 without -2; asynchronous)."""
    _check_y(plan, Y)
    _check_factors(plan, A)
    _check_factors(plan, E, "E")
    _check(LIB.cpgrad_e_gradient(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), _ptrs(E)),
           "cpgrad_e_gradient")


def cpgrad_mode_gradient(plan, Y, A, n, G):
    """G <- Y_(n)(⊙_{k≠n} A^(k)) for one mode n (1-based) by Section 3.2; returns
    the direction taken (0 right-to-left, 1 left-to-right)."""
    _check_y(plan, Y)
    _check_factors(plan, A)
    if not (1 <= int(n) <= plan.N):
        raise ValueError(f"mode {n} outside [1, {plan.N}]")
    if not (isinstance(G, torch.Tensor) and G.is_cuda and G.is_contiguous() and
            tuple(G.shape) == (plan.dims[n - 1], plan.R) and G.dtype == TORCH_DTYPE[plan.fdt]):
        raise ValueError(f"G must be a contiguous ({plan.dims[n - 1]}, {plan.R}) {TORCH_DTYPE[plan.fdt]} CUDA tensor")
    d = ctypes.c_int()
    _check(LIB.cpgrad_mode_gradient(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), int(n),
                                    ctypes.c_void_p(G.data_ptr()), ctypes.byref(d)), "cpgrad_mode_gradient")
    return d.value


def cpntf_step(plan, Y, A, sync=True):
    """One multiplicative nonnegative sweep (eq. 2.18), A updated in place.
    Returns (cost, fit) if sync, else None."""
    _check_y(plan, Y)
    _check_factors(plan, A)
    if sync:
        c, f = ctypes.c_double(), ctypes.c_double()
        _check(LIB.cpntf_step(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), ctypes.byref(c),
                              ctypes.byref(f)), "cpntf_step")
        return c.value, f.value
    _check(LIB.cpntf_step(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), None, None), "cpntf_step")
    return None


def cpals_step(plan, Y, A, sync=True):
    """One CP_ALS sweep, A updated in place.  Returns (cost, fit) if sync, else None."""
    def checks():
        _check_y(plan, Y)
        _check_factors(plan, A)
    y, a = _marshal(plan, "als", Y, (A,), checks)
    if sync:
        c, f = ctypes.c_double(), ctypes.c_double()
        _check(LIB.cpals_step(plan.handle, y, a, ctypes.byref(c), ctypes.byref(f)), "cpals_step")
        return c.value, f.value
    _check(LIB.cpals_step(plan.handle, y, a, None, None), "cpals_step")
    return None


def cp_fit(plan, Y, A):
    """(cost, fit) of [[A]] against the bound Y."""
    _check_y(plan, Y)
    _check_factors(plan, A)
    c, f = ctypes.c_double(), ctypes.c_double()
    _check(LIB.cp_fit(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), ctypes.byref(c), ctypes.byref(f)),
           "cp_fit")
    return c.value, f.value


def cpgrad_last_fit(plan):
    c, f = ctypes.c_double(), ctypes.c_double()
    _check(LIB.cpgrad_last_fit(plan.handle, ctypes.byref(c), ctypes.byref(f)), "cpgrad_last_fit")
    return c.value, f.value


def cpgrad_destroy(plan):
    if plan.handle:
        _check(LIB.cpgrad_destroy(plan.handle), "cpgrad_destroy")
        plan.handle = None


def cpgrad_version():
    return LIB.cpgrad_version().decode()


# ---------------------------------------------------------------------------
# learned extrapolation step (include/cpmlp.h)
# ---------------------------------------------------------------------------

class Mlp:
    """Owns a cpmlp_t (the step-size network)."""

    def __init__(self, handle, n_in, n_hidden, sigma_max, stream):
        self.handle = handle
        self.n_in, self.n_hidden, self.sigma_max = n_in, n_hidden, sigma_max
        self.stream = stream

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            LIB.cpmlp_destroy(h)
            self.handle = None


def cpmlp_create(n_in, n_hidden, sigma_max, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    _check(LIB.cpmlp_create(ctypes.byref(h), int(n_in), int(n_hidden), float(sigma_max),
                            ctypes.c_void_p(stream.cuda_stream)), "cpmlp_create")
    return Mlp(h, int(n_in), int(n_hidden), float(sigma_max), stream)


def cpmlp_num_params(m):
    n = ctypes.c_int64()
    _check(LIB.cpmlp_num_params(m.handle, ctypes.byref(n)), "cpmlp_num_params")
    return n.value


def cpmlp_set_params(m, params):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(LIB.cpmlp_set_params(m.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
           "cpmlp_set_params")


def cpmlp_get_params(m):
    import numpy as np
    a = np.empty(cpmlp_num_params(m), dtype=np.float32)
    _check(LIB.cpmlp_get_params(m.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
           "cpmlp_get_params")
    return a


def _f32(t, shape=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype == torch.float32):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def cpmlp_forward(m, X, sigma):
    B = X.shape[0]
    _check(LIB.cpmlp_forward(m.handle, _f32(X, (B, m.n_in)), B, _f32(sigma, (B,))), "cpmlp_forward")


def cpmlp_gradients(m, X, target, grad):
    B = X.shape[0]
    loss = ctypes.c_double()
    _check(LIB.cpmlp_gradients(m.handle, _f32(X, (B, m.n_in)), _f32(target, (B,)), B,
                               _f32(grad, (cpmlp_num_params(m),)), ctypes.byref(loss)), "cpmlp_gradients")
    return loss.value


def cpmlp_train_step(m, X, target, lr):
    B = X.shape[0]
    loss = ctypes.c_double()
    _check(LIB.cpmlp_train_step(m.handle, _f32(X, (B, m.n_in)), _f32(target, (B,)), B, float(lr),
                                ctypes.byref(loss)), "cpmlp_train_step")
    return loss.value


def cpmlp_destroy(m):
    if m.handle:
        _check(LIB.cpmlp_destroy(m.handle), "cpmlp_destroy")
        m.handle = None


def _costs(costs):
    arr = (ctypes.c_double * max(1, len(costs)))(*[float(c) for c in costs])
    return arr, len(costs)


def cpals_features(plan, A, A_start, costs, iteration, last_sigma, last_accept, feat):
    _check_factors(plan, A)
    _check_factors(plan, A_start, "A_start")
    arr, nc = _costs(costs)
    _check(LIB.cpals_features(plan.handle, _ptrs(A), _ptrs(A_start), arr, nc, int(iteration), float(last_sigma),
                              int(last_accept), _f32(feat, (NFEAT,))), "cpals_features")


def cp_fit_extrapolated(plan, Y, A, A_start, sigma):
    _check_y(plan, Y)
    _check_factors(plan, A)
    _check_factors(plan, A_start, "A_start")
    c, f = ctypes.c_double(), ctypes.c_double()
    _check(LIB.cp_fit_extrapolated(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), _ptrs(A_start),
                                   float(sigma), ctypes.byref(c), ctypes.byref(f)), "cp_fit_extrapolated")
    return c.value, f.value


def cpals_extrapolate(plan, Y, A_new, A_prev, sigma):
    """Keep A_new + sigma (A_new - A_prev) in A_new only if its exact cost is
    below the plan's last cost (that of A_new); returns (cost, fit, accepted)."""
    _check_y(plan, Y)
    _check_factors(plan, A_new, "A_new")
    _check_factors(plan, A_prev, "A_prev")
    c, f, acc = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    _check(LIB.cpals_extrapolate(plan.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A_new), _ptrs(A_prev),
                                 float(sigma), ctypes.byref(acc), ctypes.byref(c), ctypes.byref(f)),
           "cpals_extrapolate")
    return c.value, f.value, acc.value


def cpals_learned_step(plan, mlp, Y, A, costs, iteration, last_sigma, last_accept):
    """One learned-extrapolation ALS step; returns (cost, fit, accepted, sigma)."""
    _check_y(plan, Y)
    _check_factors(plan, A)
    arr, nc = _costs(costs)
    c, f = ctypes.c_double(), ctypes.c_double()
    acc, sg = ctypes.c_int(), ctypes.c_float()
    _check(LIB.cpals_learned_step(plan.handle, mlp.handle, ctypes.c_void_p(Y.data_ptr()), _ptrs(A), arr, nc,
                                  int(iteration), float(last_sigma), int(last_accept), ctypes.byref(c),
                                  ctypes.byref(f), ctypes.byref(acc), ctypes.byref(sg)), "cpals_learned_step")
    return c.value, f.value, acc.value, sg.value
