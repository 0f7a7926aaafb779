"""Benchmark of the fast all-mode CP gradient and the fast CP_ALS sweep on one GPU.

One step = one all-mode gradient (Algorithm 2: the fused contraction pass
over Y plus both peel-off chains) followed by one CP_ALS sweep (Section 4:
two passes over Y, the per-mode Cholesky updates of eq. 2.14 and the float64
cost of eq. 2.12), on the 4-D 64x64x64x64 float32 tensor of rank 16 with
20 dB noise (synthetic, seeded).  Inputs are resident in HBM before timing.

Prints one JSON line: value = all-mode CP-gradient GFLOP/s (algorithmic
flops of Algorithm 2 / time of the all-mode call), plus ALS sweeps per second,
the roofline of the dominant kernel (the fused contraction, timed with HIP
events on its stream) and the oracle timed on the host's cores.  In the timed
region the K gradients run back to back and then the K sweeps, each phase
bracketed by one HIP event pair (no host event records between calls).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "all-mode CP-gradient GFLOP/s & ALS iters/s, plain FP32 vs BF16-refined at 1e-6 fit"
WORKLOAD = "cp4d_64_r16_f32"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter calibration)")
    ap.add_argument("--quick", action="store_true", help="only the main step timing (no comparisons)")
    ap.add_argument("--mode", choices=("native", "bf16_refined"), default="native",
                    help="contraction form of the timed step for a float32 tensor (the JSON line's "
                         "headline is the native form; bf16_refined is for profiling that kernel)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1204_1586_amd", "weights",
                                                      "learned_step_cp4d_40x70.npz"))
    ap.add_argument("--configs", default="all", choices=("all", "none"),
                    help="also measure the 3-D, 7-D, 48^5 and 40x50x60x70 workloads (extra keys of the line)")
    ap.add_argument("--learned-tensors", type=int, default=50,
                    help="held-out 40x50x60x70 tensors for the learned-step comparison")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, budget_s, dtype="float64"):
    """The oracle as it stands (NumPy, Algorithm 1 per mode) on the same
    tensor: whole all-mode gradients, repeated while the budget lasts.  With
    dtype float32 the same code runs on float32 inputs (like-for-like with the
    float32 device path)."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = os.cpu_count()
    dt_ = np.float64 if dtype == "float64" else np.float32
    Y = np.asarray(pr["y"], dtype=dt_).reshape(tuple(pr["dims"]), order="F")
    A = [np.asarray(M, dtype=dt_) for M in pr["init"]]
    t0 = time.perf_counter()
    reps = 0
    while True:
        O.cp_gradient_all(Y, A)
        reps += 1
        if time.perf_counter() - t0 > budget_s * 0.5 or reps >= 5:
            break
    dt = (time.perf_counter() - t0) / reps
    return dt, reps, cores


def als_to_fit(P, plan, Y, A0, tol=1e-6, max_sweeps=1000):
    """Plain ALS from A0 until |fit_k - fit_{k-1}| < tol: sweeps and wall time."""
    import torch
    from paper_1204_1586_amd import learned
    A = [a.clone() for a in A0]
    r = learned.run_als(plan, Y, A, tol=tol, max_sweeps=max_sweeps)
    return {"sweeps": r["sweeps"], "wall_s": round(r["wall_s"], 4), "fit": r["fit"], "converged": r["converged"]}


def time_step(P, plan, Y, A0, steps, warmup):
    """ms of one all-mode gradient and of one ALS sweep (HIP events on the plan's stream)."""
    import torch
    A = [a.clone() for a in A0]
    G = [torch.empty_like(a) for a in A]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        P.cpgrad_all_modes(plan, Y, A, G)
        P.cpals_step(plan, Y, A, sync=False)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(stream)
    for _ in range(steps):
        P.cpgrad_all_modes(plan, Y, A, G)
    e[1].record(stream)
    for _ in range(steps):
        P.cpals_step(plan, Y, A, sync=False)
    e[2].record(stream)
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]) / steps, e[1].elapsed_time(e[2]) / steps


def learned_comparison(P, weights, n_tensors=3, max_sweeps=3000):
    """Plain FP32 ALS to |delta fit| < 1e-6 vs learned-step ALS run until it
    reaches the plain run's final fit (to 1e-6), on held-out 4-D 40x50x60x70
    collinear tensors (same seeds and initial factors)."""
    import numpy as np
    import torch
    import cpgen
    from paper_1204_1586_amd import learned
    d = np.load(weights)
    net = learned.new_network(params=d["params"])
    rows = []
    for t in range(n_tensors):
        pr = cpgen.make_problem("cp4d_40x70_learned", rep=10000 + t)
        Y = torch.from_numpy(pr["y"]).cuda()
        plan = P.cpgrad_plan(pr["dims"], pr["R"], "f32", "f32")
        P.cpgrad_bind(plan, Y)
        A0 = [torch.tensor(M, dtype=torch.float32).cuda() for M in pr["init"]]
        r0 = learned.run_als(plan, Y, [a.clone() for a in A0], max_sweeps=max_sweeps)
        # the learned run goes on until it reaches the plain run's final fit (to 1e-6)
        r1 = learned.run_als(plan, Y, [a.clone() for a in A0], tol=0.0, max_sweeps=max_sweeps, mlp=net,
                             target_fit=r0["fit"] - 1e-6)
        rows.append({"rep": 10000 + t, "R": pr["R"], "plain_sweeps": r0["sweeps"], "plain_s": round(r0["wall_s"], 4),
                     "plain_fit": r0["fit"], "learned_sweeps": r1["sweeps"], "learned_s": round(r1["wall_s"], 4),
                     "learned_fit": r1["fit"], "fallback_rate": round(r1["fallback_rate"], 4)})
    tot0 = sum(r["plain_sweeps"] for r in rows)
    tot1 = sum(r["learned_sweeps"] for r in rows)
    return {"tensors": rows, "trained_on_trajectories": int(d["trajectories"]),
            "sweep_ratio": round(tot1 / tot0, 4),
            "time_ratio": round(sum(r["learned_s"] for r in rows) / sum(r["plain_s"] for r in rows), 4)}


def device_y(pr, storage=None):
    import numpy as np
    import torch
    st = storage or pr["storage"]
    if st == "bf16":
        return torch.from_numpy(pr["y"].view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(pr["y"]).cuda()


def time_form(P, dims, R, Y, A0, ydt, mode, reps=20, sweeps=20):
    """One form of the contraction on a resident tensor: all-mode call and ALS
    sweep (HIP events, back to back), the fused contraction alone (events
    attached to its launches), algorithmic rates and the dominant kernel's
    HBM roofline fraction."""
    import torch
    fdt = "f64" if ydt == "f64" else "f32"
    plan = P.cpgrad_plan(dims, R, ydt, fdt, mode)
    info = P.cpgrad_plan_info(plan)
    A = [a.clone() for a in A0]
    G = [torch.empty_like(a) for a in A]
    P.cpgrad_bind(plan, Y)
    s = torch.cuda.current_stream()
    for _ in range(3):
        P.cpgrad_all_modes(plan, Y, A, G)
        P.cpals_step(plan, Y, A, sync=False)
    for a, a0 in zip(A, A0):
        a.copy_(a0)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record(s)
    for _ in range(reps):
        P.cpgrad_all_modes(plan, Y, A, G)
    e[1].record(s)
    for _ in range(sweeps):
        P.cpals_step(plan, Y, A, sync=False)
    e[2].record(s)
    torch.cuda.synchronize()
    P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 1)
    for _ in range(reps):
        P.cpgrad_all_modes(plan, Y, A0, G)
    fused_ms, n = P.cpgrad_profile_read(plan, 3)
    P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 0)
    grad_ms = e[0].elapsed_time(e[1]) / reps
    als_ms = e[1].elapsed_time(e[2]) / sweeps
    k_ms = fused_ms / max(n, 1)
    ybytes = Y.numel() * Y.element_size()
    fbytes = sum(M.numel() * M.element_size() for M in A0)
    path = P.cpgrad_plan_path(plan)
    P.cpgrad_all_modes(plan, Y, A0, G)
    torch.cuda.synchronize()
    return plan, [g.double() for g in G], {
        "all_mode_gradient_us": round(grad_ms * 1e3, 2), "gflops": round(info["alg_flops"] / (grad_ms * 1e-3) / 1e9, 1),
        "als_sweep_us": round(als_ms * 1e3, 2), "als_iters_per_s": round(1e3 / als_ms, 1),
        "fused_contraction_us": round(k_ms * 1e3, 2),
        "fused_hbm_gbs": round((ybytes + fbytes) / (k_ms * 1e-3) / 1e9, 1),
        "fused_frac_hbm": round((ybytes + fbytes) / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "fused_mfma_tflops": round(info["alg_flops"] * 0.999 / (k_ms * 1e-3) / 1e12, 1),
        "contraction_kernel": {1: "vector ALU", 2: "fp32 MFMA", 3: "bf16 MFMA", 4: "scaled fp16 MFMA"}[path["kernel"]],
        "n_star": info["n_star"]}


def rel_errors(G, ref):
    import torch
    return [float(torch.linalg.norm(g - r) / torch.linalg.norm(r)) for g, r in zip(G, ref)]


def measure_configs(P, args):
    """The other workloads, one entry each (the headline line stays the 64^4
    float32 one): rates, the fused contraction's roofline fraction, per-mode
    errors of the reduced-precision forms against the library's own float64
    path on the same values, and for the 48^5 bf16 tensor ALS to
    |delta fit| < 1e-6 in three forms from the same start."""
    import cpgen
    import torch
    from paper_1204_1586_amd import learned
    out = {}
    tdt = {"f64": torch.float64, "f32": torch.float32}
    # 3-D, float64 (latency-bound: times only)
    pr = cpgen.make_problem("cp3d_20_r3_f64", rep=0)
    Y = device_y(pr)
    A0 = [torch.tensor(M, dtype=torch.float64).cuda() for M in pr["init"]]
    _, _, r = time_form(P, pr["dims"], pr["R"], Y, A0, "f64", "native")
    out["cp3d_20_r3_f64"] = {k: r[k] for k in ("all_mode_gradient_us", "als_sweep_us", "als_iters_per_s")}
    print(f"[configs] 3-D done", file=sys.stderr, flush=True)
    # 7-D float32: three forms, errors against the float64 path
    pr = cpgen.make_problem("cp7d_10_r10_f32", rep=0)
    Y = device_y(pr)
    A0 = [torch.tensor(M, dtype=torch.float32).cuda() for M in pr["init"]]
    _, ref, r64 = time_form(P, pr["dims"], pr["R"], Y.double(), [a.double() for a in A0], "f64", "native", reps=5,
                            sweeps=5)
    c3 = {"float64_vector_alu": {k: r64[k] for k in ("all_mode_gradient_us", "gflops")}}
    for mode in ("native", "bf16", "bf16_refined", "f16_scaled", "f16_scaled_refined"):
        _, G, r = time_form(P, pr["dims"], pr["R"], Y, A0, "f32", mode)
        r["rel_err_vs_f64_per_mode"] = [float(f"{x:.3e}") for x in rel_errors(G, ref)]
        c3["f32" if mode == "native" else mode] = r
    out["cp7d_10_r10_f32"] = c3
    print(f"[configs] 7-D done", file=sys.stderr, flush=True)
    # 40x50x60x70 collinear (the learned-step shape), float32, two ranks
    c5 = {}
    for rep in (10000, 10001):
        pr = cpgen.make_problem("cp4d_40x70_learned", rep=rep)
        Y = device_y(pr)
        A0 = [torch.tensor(M, dtype=torch.float32).cuda() for M in pr["init"]]
        _, _, r = time_form(P, pr["dims"], pr["R"], Y, A0, "f32", "native")
        c5[f"R{pr['R']}"] = r
    out["cp4d_40x70_learned"] = c5
    print(f"[configs] 40x70 done", file=sys.stderr, flush=True)
    # 48^5 stored bf16, rank 32, congruence 0.5
    pr = cpgen.make_problem("cp5d_48_r32_bf16", rep=0)
    Yb = device_y(pr)
    del pr["y"]
    A0 = [torch.tensor(M, dtype=torch.float32).cuda() for M in pr["init"]]
    dims, R = pr["dims"], pr["R"]
    Yf = Yb.float()
    _, ref, r64 = time_form(P, dims, R, Yf.double(), [a.double() for a in A0], "f64", "native", reps=2, sweeps=1)
    torch.cuda.empty_cache()
    c4 = {"float64_vector_alu": {k: r64[k] for k in ("all_mode_gradient_us", "gflops")}, "als_to_fit_1e-6": {}}
    for name, Yx, ydt, mode in (("f32_on_upcast_y", Yf, "f32", "native"), ("bf16_refined", Yb, "bf16", "bf16_refined"),
                                ("f16_scaled_refined", Yb, "bf16", "f16_scaled_refined")):
        plan, G, r = time_form(P, dims, R, Yx, A0, ydt, mode, reps=10, sweeps=10)
        r["rel_err_vs_f64_per_mode"] = [float(f"{x:.3e}") for x in rel_errors(G, ref)]
        c4[name] = r
        A = [a.clone() for a in A0]
        res = learned.run_als(plan, Yx, A, tol=1e-6, max_sweeps=5000)
        c4["als_to_fit_1e-6"][name] = {"sweeps": res["sweeps"], "wall_s": round(res["wall_s"], 4),
                                       "ms_per_sweep_incl_readback": round(res["wall_s"] * 1e3 / res["sweeps"], 4),
                                       "fit": res["fit"], "converged": res["converged"]}
        print(f"[configs] 48^5 {name} done", file=sys.stderr, flush=True)
    out["cp5d_48_r32_bf16"] = c4
    del Yf, Yb
    torch.cuda.empty_cache()
    return out


def cold_cache_fused(P, plan, Y, A, G, reps=10):
    """The fused contraction with the 256 MB Infinity Cache scrubbed before
    each launch (a 512 MB device write), median of `reps` launches."""
    import torch
    scrub = torch.empty(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    ts = []
    for k in range(reps):
        scrub.fill_(float(k))
        P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 1)
        P.cpgrad_all_modes(plan, Y, A, G)
        ms, n = P.cpgrad_profile_read(plan, 3)
        ts.append(ms / max(n, 1))
    P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 0)
    del scrub
    ts.sort()
    return ts[len(ts) // 2]


def als_rate_with_readback(P, plan, Y, A0, sweeps=50):
    """Sweeps per second when every sweep returns its cost and fit to the host
    (what the |delta fit| stopping rule needs)."""
    import torch
    A = [a.clone() for a in A0]
    for _ in range(3):
        P.cpals_step(plan, Y, A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        P.cpals_step(plan, Y, A)
    return sweeps / (time.perf_counter() - t0)


# HBM traffic of the fused contraction comes from rocprofv3 counters taken
# outside this script (FETCH_SIZE and WRITE_SIZE runs, scaled by the same
# counters on a plain copy of known size) and recorded in a profile summary,
# together with a hash of the sources the kernel is built from.  It is
# reported only while those sources are unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_cp4d_64_r16_f32.md")
CONTRACTION_SOURCES = ("paper_1204_1586_amd/csrc/k_contract_mfma.hip", "paper_1204_1586_amd/csrc/cpg_device.h",
                       "paper_1204_1586_amd/csrc/cpg_internal.h", "paper_1204_1586_amd/csrc/cpg_fastdiv.h",
                       "include/cpgrad.h")


def contraction_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in CONTRACTION_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(workload):
    """(bytes per launch, record) of the fused contraction, or (None, reason)."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            line = next(l for l in f if l.startswith("traffic-record:"))
        rec = json.loads(line.split(":", 1)[1])
    except (OSError, StopIteration, ValueError):
        return None, "no traffic record"
    if rec.get("workload") != workload:
        return None, "record is for another workload"
    if rec.get("source_sha256") != contraction_source_hash():
        return None, "kernel sources changed since the counters were taken"
    b = (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024
    return int(round(b)), rec


def calib_copy():
    import torch
    n = 64 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": a.numel() * 4, "calib_copy_bytes_written": b.numel() * 4,
                      "launches": 20}))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the slab split of Y over GPUs is described in DESIGN.md, not built).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calib_copy:
        calib_copy()
        return

    import cpgen
    import paper_1204_1586_amd as P

    w = cpgen.WORKLOADS[args.workload]
    pr = cpgen.make_problem(w, rep=0)
    dims, R = pr["dims"], pr["R"]
    fst = "f64" if pr["storage"] == "f64" else "f32"
    tdt = torch.float64 if fst == "f64" else torch.float32
    if pr["storage"] == "bf16":
        Y = torch.from_numpy(pr["y"].view(np.int16)).view(torch.bfloat16).cuda()
        mode = "bf16_refined"
    else:
        Y = torch.from_numpy(pr["y"]).cuda()
        mode = args.mode
    A0 = [torch.tensor(M, dtype=tdt).cuda() for M in pr["init"]]
    A = [M.clone() for M in A0]
    G = [torch.empty_like(M) for M in A]
    plan = P.cpgrad_plan(dims, R, pr["storage"], fst, mode)
    info = P.cpgrad_plan_info(plan)
    P.cpgrad_bind(plan, Y)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        P.cpgrad_all_modes(plan, Y, A, G)
        P.cpals_step(plan, Y, A, sync=False)
    torch.cuda.synchronize()
    # restart the sweeps from the seeded initial factors so the timed sweeps are reproducible
    for a, a0 in zip(A, A0):
        a.copy_(a0)
    # Timed region: K steps, each = one all-mode gradient + one ALS sweep.  The
    # K gradients run back to back and then the K sweeps (same work, no host
    # event records between calls); one HIP event pair brackets each phase.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(args.steps):
        P.cpgrad_all_modes(plan, Y, A, G)
    ev[1].record(stream)
    for s in range(args.steps):
        P.cpals_step(plan, Y, A, sync=False)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cost, fit = P.cpgrad_last_fit(plan)
    # the dominant kernel alone: the fused contraction bracketed by HIP events on the plan's stream
    P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 1)
    for s in range(args.steps):
        P.cpgrad_all_modes(plan, Y, A, G)
    torch.cuda.synchronize()
    fused_ms, fused_n = P.cpgrad_profile_read(plan, 3)
    P.cpgrad_set_option(plan, P.CPG_OPT_PROFILE, 0)

    grad_ms = ev[0].elapsed_time(ev[1]) / args.steps
    als_ms = ev[1].elapsed_time(ev[2]) / args.steps
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gflops = info["alg_flops"] / (grad_ms * 1e-3) / 1e9

    # roofline of the dominant kernel: the fused contraction (one pass over Y)
    ybytes = Y.numel() * Y.element_size()
    fbytes = sum(M.numel() * M.element_size() for M in A)
    alg_bytes_launch = ybytes + fbytes
    k_ms = fused_ms / max(fused_n, 1)
    achieved = alg_bytes_launch / (k_ms * 1e-3) / 1e9
    traffic, rec = recorded_traffic(w.name) if mode == "native" else (None, "counters cover the float32 kernel")
    traffic_note = (os.path.relpath(TRAFFIC_PROFILE, ROOT) if traffic is not None else rec)
    out = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("bf16" if mode == "bf16_refined" else "f32") if pr["storage"] == "f32" else pr["storage"],
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(dims), "rank": R, "snr_db": w.snr_db,
                   "storage": pr["storage"], "mode": mode, "n_star": info["n_star"],
                   "step": "cpgrad_all_modes + cpals_step"},
        "all_mode_gradient_ms": round(grad_ms, 5),
        "als_iters_per_s": round(1e3 / als_ms, 2),
        "als_sweep_ms": round(als_ms, 5),
        "fit_after_timed_sweeps": fit,
        "alg_flops_all_modes": info["alg_flops"],
        "roofline": {"bound": "hbm", "kernel": "fused contraction (both partials, one pass over Y)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM read + write, counter-scaled)",
                     "traffic_note": traffic_note,
                     "avg_launch_ms": round(k_ms, 6), "launches": fused_n,
                     "alg_bytes_per_launch": alg_bytes_launch},
    }
    if not args.quick and pr["storage"] == "f32":
        # the same tensor through the bf16 matrix cores with the same-pass refinement
        planb = P.cpgrad_plan(dims, R, "f32", "f32", "bf16_refined")
        P.cpgrad_bind(planb, Y)
        gb_ms, ab_ms = time_step(P, planb, Y, A0, args.steps, args.warmup)
        out["bf16_refined"] = {"all_mode_gradient_ms": round(gb_ms, 5),
                               "value": round(info["alg_flops"] / (gb_ms * 1e-3) / 1e9, 3),
                               "als_iters_per_s": round(1e3 / ab_ms, 2)}
        # plain FP32 vs BF16-refined ALS to |delta fit| < 1e-6 from the same start
        out["fit_1e-6"] = {"f32": als_to_fit(P, plan, Y, A0), "bf16_refined": als_to_fit(P, planb, Y, A0)}
        if os.path.exists(args.weights):
            out["learned_step"] = learned_comparison(P, args.weights, n_tensors=args.learned_tensors)
    if not args.quick:
        out["als_iters_per_s_with_readback"] = round(als_rate_with_readback(P, plan, Y, A0), 1)
        cold = cold_cache_fused(P, plan, Y, A0, G)
        out["fused_contraction_cold_cache"] = {
            "avg_launch_ms": round(cold, 6), "achieved": round(alg_bytes_launch / (cold * 1e-3) / 1e9, 1),
            "frac": round(alg_bytes_launch / (cold * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "median of 10 launches, each after a 512 MB device write that evicts the 256 MB Infinity Cache"}
    if not args.quick and args.configs == "all":
        out["configs"] = measure_configs(P, args)
    if not args.no_cpu_baseline:
        dt, reps, cores = cpu_baseline(pr, args.cpu_budget_s)
        dt32, reps32, _ = cpu_baseline(pr, args.cpu_budget_s, "float32")
        out["cpu_baseline"] = {"value": round(info["alg_flops"] / dt / 1e9, 4), "unit": "GFLOP/s", "cores": cores,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"{reps} whole all-mode gradient(s) of the same tensor by the float64 "
                                         f"oracle (Algorithm 1 per mode), {dt:.3f} s each; GFLOP/s counts Algorithm "
                                         f"2's flops (the unit of the GPU figure) over the oracle's time",
                               "float32_inputs": {"value": round(info["alg_flops"] / dt32 / 1e9, 4),
                                                  "sample": f"{reps32} all-mode gradient(s), the same oracle code on "
                                                            f"float32 arrays, {dt32:.3f} s each"}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
