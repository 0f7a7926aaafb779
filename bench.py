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
    return ap.parse_args()


def cpu_baseline(pr, budget_s):
    """The oracle as it stands (float64 NumPy, Algorithm 1 per mode) on the same
    tensor: whole all-mode gradients, repeated while the budget lasts."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        cores = os.cpu_count()
    Y = O.as_tensor(pr["y"].astype(np.float64), pr["dims"])
    A = [np.asarray(M, dtype=np.float64) for M in pr["init"]]
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
    """Plain FP32 ALS vs learned-step ALS to |delta fit| < 1e-6 on held-out
    4-D 40x50x60x70 collinear tensors (same seeds and initial factors)."""
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
        r1 = learned.run_als(plan, Y, [a.clone() for a in A0], max_sweeps=max_sweeps, mlp=net)
        rows.append({"rep": 10000 + t, "R": pr["R"], "plain_sweeps": r0["sweeps"], "plain_s": round(r0["wall_s"], 4),
                     "plain_fit": r0["fit"], "learned_sweeps": r1["sweeps"], "learned_s": round(r1["wall_s"], 4),
                     "learned_fit": r1["fit"], "fallback_rate": round(r1["fallback_rate"], 4)})
    tot0 = sum(r["plain_sweeps"] for r in rows)
    tot1 = sum(r["learned_sweeps"] for r in rows)
    return {"tensors": rows, "trained_on_trajectories": int(d["trajectories"]),
            "sweep_ratio": round(tot1 / tot0, 4),
            "time_ratio": round(sum(r["learned_s"] for r in rows) / sum(r["plain_s"] for r in rows), 4)}


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
            out["learned_step"] = learned_comparison(P, args.weights)
    if not args.no_cpu_baseline:
        dt, reps, cores = cpu_baseline(pr, args.cpu_budget_s)
        out["cpu_baseline"] = {"value": round(info["alg_flops"] / dt / 1e9, 4), "unit": "GFLOP/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{reps} whole all-mode gradient(s) of the same tensor by the float64 "
                                         f"oracle (Algorithm 1 per mode), {dt:.3f} s each"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
