#!/usr/bin/env python3
"""Benchmark of the batched operator rotation on one MI355X.

Workload: dense shared-U rotation out_b = U^T (O_b (x) I_d) U with m = m' =
1024, d = 4 (the Hubbard site), 64 symmetric Gaussian operators scaled by
1/sqrt(m), U the Q factor of a seeded 4096 x 1024 Gaussian.  Inputs are
synthetic (seeded) and resident in HBM before timing starts.  One step = one
rotation of the whole batch (stage 1 and stage 2 for every operator).

Prints ONE JSON line (rank 0) with operator rotations/s, the roofline of the
dominant kernel (timed with HIP events on its launch stream) and the oracle's
CPU throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "operator rotations/s + % MFMA peak, m=1024 d=4, FP32 vs split-BF16 @1e-5"
PEAK_TFLOPS = {"fp32": 157.3, "split_bf16": 2516.6, "fp64": 78.6}  # dense matrix-core peaks
WORKLOAD = "dense_m1024_n64"
# dense shared-U workloads timed by bench_dense: the headline, the 512-state
# batch of 200 operators and the latency-bound 64-state FP64 batch
DENSE = (WORKLOAD, "dense_m512_n200", "dense_m64_f64")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split-bf16", action="store_true",
                    help="with --precision fp32, skip the split-BF16 measurement")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip timing the plain FP64 GPU rotation (speedup denominator)")
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[*DENSE, "blocked_1024_n400", "uneven_1000", "differentiated_m1024_n64",
                             "site_m1024_n64", "measure_m1024", "density_m1024", "superblock_m1024"],
                    help="default: the headline dense workload; the others time the quantum-number "
                         "blocked batch or the uneven sweep plan")
    ap.add_argument("--symmetric", action="store_true",
                    help="time the dense workload with the symmetric-output stage 2 (upper triangle)")
    ap.add_argument("--no-symmetric", action="store_true",
                    help="skip the symmetric-output figures of the dense workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def flops_per_op(m, d, mp, symmetric=False):
    """Algorithmic flops of one rotation: stage 1 (2 m^2 d m') plus stage 2,
    2 m d m'^2 in general or m d m'(m'+1) when only the upper triangle of the
    symmetric output is formed."""
    s2 = m * d * mp * (mp + 1) if symmetric else 2.0 * m * d * mp * mp
    return 2.0 * m * m * d * mp + s2


def time_steps(rot, U, O, out, ws, d, precision, steps, warmup, profile, symmetric=False):
    """Total ms of `steps` rotations (events on the launch stream around the
    whole loop), the per-step times (one event per step boundary) and the
    kernel timings of librot's profiler."""
    import torch
    for _ in range(warmup):
        rot.rotate(U, O, d, precision, out=out, workspace=ws, symmetric_O=symmetric)
    torch.cuda.synchronize()
    if profile:
        rot.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        rot.rotate(U, O, d, precision, out=out, workspace=ws, symmetric_O=symmetric)
        ev[i + 1].record()
    torch.cuda.synchronize()
    kernels = rot.profile_read() if profile else {}
    if profile:
        rot.profile_enable(False)
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]), kernels, per_step


def recorded_traffic(kernel_kind):
    """HBM bytes per launch from the rocprofv3 counter runs recorded in
    profiles/hbm_traffic.txt, or None when the kernel source has changed since
    (its sha256 no longer matches) or no record exists."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        kind, src, sha, rd, wr = line.split()
        if kind != kernel_kind:
            continue
        cur = hashlib.sha256(open(os.path.join(root, src), "rb").read()).hexdigest()[:16]
        return int(rd) + int(wr) if cur == sha else None
    return None


def measure(rot, U, O, out, d, precision, steps, warmup, symmetric=False):
    """Time `steps` rotations of the batch; returns the figures for one precision.
    symmetric: the operators are symmetric and stage 2 forms only the upper
    output triangle, counted with its own (smaller) algorithmic flops."""
    import torch
    n, m, _ = O.shape
    mp = U.shape[1]
    p = rot._problem(U, O, out, d)
    prec = rot.precision_code(precision)
    ws = torch.empty(rot.rot_workspace_size([p], prec), dtype=torch.uint8, device=U.device)
    ms, kernels, per_step = time_steps(rot, U, O, out, ws, d, precision, steps, warmup, True, symmetric)
    del ws
    ops_per_s = n * steps / (ms / 1e3)
    F = flops_per_op(m, d, mp, symmetric)
    tflops = F * ops_per_s / 1e12
    peak = PEAK_TFLOPS[precision]
    exec_factor = 3.0 if precision == "split_bf16" else 1.0
    per_launch_flops = {"stage1": n * 2.0 * m * m * d * mp, "stage2": n * 2.0 * m * d * mp * mp,
                        "stage2sym": n * 1.0 * m * d * mp * (mp + 1),
                        "small": n * (2.0 * m * m * d * mp + 2.0 * m * d * mp * mp)}  # both stages, one launch
    stage_kernels = {k: v for k, v in kernels.items() if k.split("_")[0] in per_launch_flops}
    dom_name, (dom_count, dom_ms) = max(stage_kernels.items(), key=lambda kv: kv[1][1])
    dom_avg_ms = dom_ms / dom_count
    achieved = per_launch_flops[dom_name.split("_")[0]] * exec_factor / (dom_avg_ms / 1e3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": recorded_traffic(dom_name),
                "kernel": dom_name, "avg_ms": round(dom_avg_ms, 4)}
    per_step.sort()
    return {"ops_per_s": ops_per_s, "ms_per_step": ms / steps, "tflops": tflops,
            "ms_per_step_median": per_step[len(per_step) // 2], "ms_per_step_min": per_step[0],
            "pct_mfma_peak": 100 * tflops * exec_factor / peak,
            "kernels_ms_avg": {k: round(v[1] / v[0], 4) for k, v in kernels.items()},
            "roofline": roofline}


def base_record(args, value, unit, ms_per_step, config, dtype="f32"):
    return {"metric": METRIC, "value": round(value, 2), "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def bench_blocked(args, rot, torch, workloads):
    """Quantum-number blocked batch: m = m' = 1024 in (N_up, N_dn) sectors, 400
    operators (200 conserving, 100 + 100 shifting)."""
    case = workloads.blocked_case()
    pk = workloads.pack_blocked(case)
    dev = torch.device("cuda:0")
    U_blk = torch.from_numpy(pk.U_blk).float().to(dev)
    O_blk = torch.from_numpy(pk.O_blk).float().to(dev)
    out_blk = torch.empty(pk.out_size, device=dev)
    p, keep = rot.blocked_problem(pk.site_qn, pk.old, pk.new, pk.shift, U_blk, pk.U_off, O_blk, pk.O_off,
                                  pk.out_off, out_blk)
    ws = torch.empty(max(256, rot.rot_blocked_workspace_size(p)), dtype=torch.uint8, device=dev)
    run = lambda: rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(),
                                        torch.cuda.current_stream().cuda_stream)
    # algorithmic work: the block GEMMs that the sector structure requires
    old = {s.qn: s for s in case.old}
    new = {s.qn: s for s in case.new}
    flops = 0.0
    bytes_alg = sum(v.size for b in case.O_blocks for v in b.values()) * 4 + pk.U_blk.size * 4
    for delta, blocks in zip(case.shifts, case.O_blocks):
        for sec in case.new:
            t = (sec.qn[0] + delta[0], sec.qn[1] + delta[1])
            if t not in new:
                continue
            MT = sum(old[(t[0] - a, t[1] - b)].dim for a, b in case.site_qn if (t[0] - a, t[1] - b) in old)
            for a, b in case.site_qn:
                qs, qt = (sec.qn[0] - a, sec.qn[1] - b), (t[0] - a, t[1] - b)
                if qs in old and qt in old:
                    flops += 2.0 * old[qt].dim * old[qs].dim * sec.dim
            flops += 2.0 * new[t].dim * MT * sec.dim
            bytes_alg += new[t].dim * sec.dim * 4
    # cold first call: builds the work-lists and times the execution paths
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - c0) * 1e3
    for _ in range(max(1, args.warmup)):
        run()
    torch.cuda.synchronize()
    # direct calls, with librot's per-kernel profiler
    rot.profile_enable(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        run()
    t1.record()
    torch.cuda.synchronize()
    kernels = rot.profile_read()
    rot.profile_enable(False)
    direct_ms = t0.elapsed_time(t1) / args.steps
    # the timed figure: replays of ten calls captured in one hipGraph (one
    # graph launch spread over ten batches), per batch
    reps = 10
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            run()
    for _ in range(max(1, args.warmup)):
        graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for i in range(args.steps):
        graph.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per_step = sorted(ev[i].elapsed_time(ev[i + 1]) / reps for i in range(args.steps))
    ms = ev[0].elapsed_time(ev[args.steps]) / args.steps / reps
    del graph
    n = len(case.shifts)
    tflops = flops / (ms / 1e3) / 1e12
    rec = base_record(args, n / (ms / 1e3), "operator rotations/s", ms,
                      {"workload": "blocked_1024_n400", "m": case.m, "mp": case.mp, "d": case.d,
                       "sectors": len(case.old), "sector_dims": [min(s.dim for s in case.old),
                                                                 max(s.dim for s in case.old)],
                       "n_ops": n, "precision": "fp32"})
    dom, (cnt, tot) = max(kernels.items(), key=lambda kv: kv[1][1])
    rec.update({"timing": "hipGraph replays of ten calls, per call", "ms_per_step_median": round(per_step[len(per_step) // 2], 4),
                "ms_per_step_min": round(per_step[0], 4), "direct_call_ms_per_step": round(direct_ms, 4),
                "cold_first_call_ms": round(cold_ms, 2),
                "gflop_per_step": round(flops / 1e9, 3), "tflops": round(tflops, 2),
                "pct_fp32_mfma_peak": round(100 * tflops / 157.3, 2),
                "algorithmic_gb_per_s": round(bytes_alg / (ms / 1e3) / 1e9, 1),
                "kernels_ms_avg": {k: round(v[1] / v[0], 4) for k, v in kernels.items()},
                "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 157.3, "unit": "TFLOP/s",
                             "frac": round(tflops / 157.3, 4), "traffic": None, "kernel": "blocked (both stages)",
                             "note": "small sector GEMMs (4..76): latency/occupancy bound"}})
    del keep
    return rec


def bench_uneven(args, rot, torch, workloads):
    """1000 rotations, m uniform in {128,...,2048}, d = 4, m' = m, 8 operators
    each, one plan (grouped persistent launches, tuned, hipGraph replay)."""
    sizes = workloads.uneven_sizes(1000)
    data = workloads.uneven_case_gpu(sizes, d=4, ops_per_rot=8, cfg=4)
    groups = [(U, O, torch.empty((8, U.shape[1], U.shape[1]), device=U.device), 4) for U, O in data]
    torch.cuda.synchronize()
    # plan creation with an empty tuning cache (times the candidates per size
    # class and writes ROT_TUNE_CACHE), then again with the cache warm
    cache = os.environ.get("ROT_TUNE_CACHE")
    cache_entries = None
    c0 = time.perf_counter()
    plan = rot.Plan(groups, workspace_bytes=32 << 30)  # size classes, tuning, graph capture
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - c0
    tuned_now = sum(1 for c in plan.describe()["classes"] if c["tuned_now"])
    plan.close()
    c0 = time.perf_counter()
    plan = rot.Plan(groups, workspace_bytes=32 << 30)
    torch.cuda.synchronize()
    plan_warm_s = time.perf_counter() - c0
    if cache and os.path.exists(cache):
        cache_entries = sum(1 for line in open(cache) if line.strip() and not line.startswith("#"))
    flops = sum(8 * flops_per_op(m, 4, m) for m in sizes)
    c0 = time.perf_counter()
    plan.execute()
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - c0) * 1e3
    for _ in range(max(1, args.warmup)):
        plan.execute()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        plan.execute()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    tflops = flops / (ms / 1e3) / 1e12
    rec = base_record(args, 8000 / (ms / 1e3), "operator rotations/s", ms,
                      {"workload": "uneven_1000", "rotations": 1000, "ops_per_rotation": 8, "d": 4,
                       "m_classes": [128, 256, 512, 1024, 2048], "precision": "fp32"})
    rec.update({"timing": "hipGraph replays of the plan", "plan_create_s": round(plan_s, 2),
                "plan_create_warm_cache_s": round(plan_warm_s, 2), "classes_tuned_on_first_create": tuned_now,
                "tune_cache_file": cache, "tune_cache_entries": cache_entries,
                "cold_first_execute_ms": round(cold_ms, 1),
                "tflop_per_step": round(flops / 1e12, 2), "tflops": round(tflops, 2),
                "pct_fp32_mfma_peak": round(100 * tflops / 157.3, 2), "plan": plan.describe(),
                "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 157.3, "unit": "TFLOP/s",
                             "frac": round(tflops / 157.3, 4), "traffic": None, "kernel": "plan graph (all launches)"}})
    plan.close()
    return rec


def bench_differentiated(args, rot, torch, workloads):
    """Forward + FP64 pair loss + adjoint (nothing stored) through
    torch.autograd, m = m' = 1024, d = 4, 64 symmetric operators; the forward
    and adjoint in FP32 (the line's value) and in split-BF16."""
    case = workloads.named_dense(WORKLOAD)
    psi = torch.from_numpy(workloads.psi_vector(case.mp, workloads.rng(5, 2))).cuda()
    U = torch.from_numpy(case.U).float().cuda().requires_grad_(True)
    O = torch.from_numpy(case.O).float().cuda().requires_grad_(True)
    n, m, mp, d = 64, 1024, 1024, 4
    f_fwd = n * flops_per_op(m, d, mp)
    # backward per symmetric operator: P = U dOut and (P + Q) = U (dOut + dOut^T)
    # (2 md mp^2 each), dO = P_r U_r^T and dU_r += O (P + Q)_r (2 m^2 d mp each)
    f_bwd = n * (4.0 * m * d * mp * mp + 4.0 * m * m * d * mp)

    def run(precision):
        def step():
            U.grad = None
            O.grad = None
            X = rot.RotateFn.apply(U, O, 4, precision, True)
            L = rot.PairLossFn.apply(X, psi)
            L.backward()
            return L

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        rot.profile_enable(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            step()
        t1.record()
        torch.cuda.synchronize()
        kernels = rot.profile_read()
        rot.profile_enable(False)
        ms = t0.elapsed_time(t1) / args.steps
        tflops = (f_fwd + f_bwd) / (ms / 1e3) / 1e12
        return ms, tflops, kernels

    ms, tflops, kernels = run("fp32")
    rec = base_record(args, n / (ms / 1e3), "operator rotations/s (forward + loss + adjoint)", ms,
                      {"workload": "differentiated_m1024_n64", "m": m, "d": d, "mp": mp, "n_ops": n,
                       "precision": "fp32 forward/adjoint, fp64 loss"})
    rec.update({"tflop_per_step": round((f_fwd + f_bwd) / 1e12, 3), "tflops": round(tflops, 2),
                "pct_fp32_mfma_peak": round(100 * tflops / 157.3, 2),
                "kernels_ms_avg": {k: round(v[1] / v[0], 4) for k, v in kernels.items()},
                "kernels_ms_total_per_step": {k: round(v[1] / args.steps, 4) for k, v in kernels.items()}})
    ms_b, tflops_b, kernels_b = run("split_bf16")
    rec["split_bf16"] = {"value": round(n / (ms_b / 1e3), 2), "unit": "operator rotations/s (forward + loss + adjoint)",
                         "ms_per_step": round(ms_b, 4), "tflops_fp32_equivalent": round(tflops_b, 2),
                         "pct_bf16_mfma_peak_executed": round(100 * 3 * tflops_b / 2516.6, 2),
                         "speedup_vs_fp32": round(ms / ms_b, 3),
                         "kernels_ms_total_per_step": {k: round(v[1] / args.steps, 4) for k, v in kernels_b.items()}}
    return rec


def timed_loop(torch, fn, steps, warmup):
    """ms per call of fn over `steps` calls (events on the current stream)."""
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


C_UP = ((0.0, 1.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 1.0), (0.0, 0.0, 0.0, 0.0))
C_DN = ((0.0, 0.0, 1.0, 0.0), (0.0, 0.0, 0.0, -1.0), (0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0))
N_SITE = ((0.0, 0.0, 0.0, 0.0), (0.0, 1.0, 0.0, 0.0), (0.0, 0.0, 1.0, 0.0), (0.0, 0.0, 0.0, 2.0))
SZ_SITE = ((0.0, 0.0, 0.0, 0.0), (0.0, 0.5, 0.0, 0.0), (0.0, 0.0, -0.5, 0.0), (0.0, 0.0, 0.0, 0.0))


def bench_site(args, rot, torch, workloads):
    """Blocking with the added site (m = m' = 1024, d = 4, FP32): the 64
    block-site products X_b (x) c_up of one step, and the new site's own
    operators I_B (x) n_a, I_B (x) S^z_a, P_B (x) c_up, P_B (x) c_dn."""
    import numpy as np
    case = workloads.named_dense(WORKLOAD)
    U = torch.from_numpy(case.U).float().cuda()
    X = torch.from_numpy(case.O).float().cuda()
    parity = torch.from_numpy(np.where(np.arange(case.m) % 2 == 0, 1.0, -1.0)).float().cuda()
    n = X.shape[0]
    import ctypes
    S = np.ascontiguousarray(C_UP, dtype=np.float64)
    p = rot.RotSiteProblem(case.m, 4, case.mp, n, rot.ROT_BLOCK_DENSE, U.data_ptr(),
                           S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), X.data_ptr(), case.m * case.m,
                           1 << 40, case.mp * case.mp)
    ws = torch.empty(rot.rot_site_workspace_size([p], rot.ROT_FP32), dtype=torch.uint8, device=U.device)
    rot.profile_enable(True)
    ms_dense = timed_loop(torch, lambda: rot.rotate_site(U, X, C_UP, "fp32", workspace=ws), args.steps, args.warmup)
    kernels = rot.profile_read()
    rot.profile_enable(False)

    def new_site():
        rot.rotate_site(U, None, N_SITE, "fp32", workspace=ws)
        rot.rotate_site(U, None, SZ_SITE, "fp32", workspace=ws)
        rot.rotate_site(U, parity, C_UP, "fp32", workspace=ws)
        rot.rotate_site(U, parity, C_DN, "fp32", workspace=ws)

    ms_new = timed_loop(torch, new_site, args.steps, args.warmup)
    F = flops_per_op(case.m, 4, case.mp)
    tflops = n * F / (ms_dense / 1e3) / 1e12
    stage = {k: v for k, v in kernels.items() if k.startswith("site_stage")}
    dom, (cnt, tot) = max(stage.items(), key=lambda kv: kv[1][1])
    achieved = n * F / 2 / (tot / cnt / 1e3) / 1e12
    rec = base_record(args, n / (ms_dense / 1e3), "operator rotations/s (block-site products)", ms_dense,
                      {"workload": "site_m1024_n64", "m": case.m, "d": 4, "mp": case.mp, "n_ops": n,
                       "site_operator": "c_up", "precision": "fp32"})
    rec.update({"tflops": round(tflops, 2), "pct_fp32_mfma_peak": round(100 * tflops / 157.3, 2),
                "new_site_operators_ms": round(ms_new, 4), "new_site_operators": 4,
                "kernels_ms_avg": {k: round(v[1] / v[0], 4) for k, v in kernels.items()},
                "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": 157.3, "unit": "TFLOP/s",
                             "frac": round(achieved / 157.3, 4), "traffic": None, "kernel": dom,
                             "avg_ms": round(tot / cnt, 4)}})
    return rec


def bench_measure(args, rot, torch, workloads):
    """Superblock measurements in FP64: block B of m = 1024 states with site
    a (d = 4), site a~ and block B~ (dR = 4, mR = 1024), a seeded unit state
    psi (4096 x 4096); one-point values of the 64 stored operators of the
    headline batch (FP32), and the 8 x 8 products of operators of the two
    blocks (FP64)."""
    import numpy as np
    case = workloads.named_dense(WORKLOAD)
    m, d, mR, dR = case.m, 4, 1024, 4
    g = torch.Generator(device="cuda")
    g.manual_seed(5662 * 100 + 7)
    psi = torch.randn((m * d, dR * mR), generator=g, dtype=torch.float64, device="cuda")
    psi /= psi.norm()
    Z32 = torch.from_numpy(case.O).float().cuda()
    ZL = Z32[:8].double().contiguous()
    WR = Z32[8:16].double().contiguous()
    n = Z32.shape[0]
    ms_one = timed_loop(torch, lambda: rot.expect_block(psi, Z32, d), args.steps, args.warmup)
    rot.profile_enable(True)
    ms_cross = timed_loop(torch, lambda: rot.expect_cross(psi, ZL, WR, d, dR), max(2, args.steps // 4), 1)
    kernels = rot.profile_read()
    rot.profile_enable(False)
    mp = dR * mR
    f_one = 2.0 * m * m * d * dR * mR + 2.0 * n * m * m
    f_cross = 8 * (2.0 * m * m * d * mp + 2.0 * m * d * mp * mp) + 2.0 * 8 * 8 * mR * mR
    t_one = f_one / (ms_one / 1e3) / 1e12
    t_cross = f_cross / (ms_cross / 1e3) / 1e12
    rec = base_record(args, n / (ms_one / 1e3), "stored operators measured/s (one-point, FP64)", ms_one,
                      {"workload": "measure_m1024", "m": m, "d": d, "mR": mR, "dR": dR, "n_stored": n,
                       "cross_pairs": "8 x 8", "precision": "fp64 state and reductions"}, dtype="f64")
    rec.update({"one_point_tflops_fp64": round(t_one, 2), "cross_block_ms": round(ms_cross, 3),
                "cross_block_tflops_fp64": round(t_cross, 2),
                "kernels_ms_avg": {k: round(v[1] / v[0], 4) for k, v in kernels.items()},
                "roofline": {"bound": "mfma", "achieved": round(t_cross, 2), "peak": 78.6, "unit": "TFLOP/s",
                             "frac": round(t_cross / 78.6, 4), "traffic": None,
                             "kernel": "cross-block products (FP64 rotation by psi, pair product)"}})
    return rec


def bench_density(args, rot, torch, workloads):
    """Density matrix to kept basis (FP64): the enlarged block [B a] of the
    1024-state sector grid, 47 sectors of 4..246 states (3939 states), a
    superblock state of decaying weights, m' = 1024 kept.  Each step is one
    rot_density_basis call (rho per sector, Jacobi, sort, selection), host
    synchronisations per sweep included."""
    import time

    import numpy as np
    case = workloads.density_case()
    psi = [torch.from_numpy(p).cuda() for p in case.psi]
    secs, outs = [], []
    for p in psi:
        n, r = p.shape
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        V = torch.empty((n, n), dtype=torch.float64, device="cuda")
        secs.append(rot.RotDmSector(n, r, p.data_ptr(), r, w.data_ptr(), V.data_ptr(), n))
        outs.append((w, V))
    kept = torch.empty(len(secs), dtype=torch.int32, device="cuda")
    eps = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(rot.density_workspace_size(secs), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        rot.rot_density_basis(secs, case.m_keep, kept.data_ptr(), eps.data_ptr(), ws.data_ptr(), ws.numel(),
                              stream)

    ms = timed_loop(torch, step, args.steps, args.warmup)
    rot.profile_enable(True)
    calls = 2
    for _ in range(calls):
        step()
    torch.cuda.synchronize()
    kernels = rot.profile_read()
    rot.profile_enable(False)
    rounds = kernels.get("dm_jacobi_pairs", (0, 0.0))[0] / calls

    def torch_eigh():
        for p in psi:
            torch.linalg.eigh(p @ p.T)

    ms_torch = timed_loop(torch, torch_eigh, max(2, args.steps // 4), 1)
    t0 = time.perf_counter()
    import oracle.density as odm
    ref = odm.density_basis(case.psi, case.m_keep)
    ms_cpu = (time.perf_counter() - t0) * 1e3
    n_states = sum(p.shape[0] for p in case.psi)
    rec = base_record(args, 1e3 / ms, "density-matrix steps/s (3939 states, 47 sectors)", ms,
                      {"workload": "density_m1024", "sectors": len(psi), "states": n_states,
                       "largest_sector": max(p.shape[0] for p in case.psi), "m_keep": case.m_keep,
                       "weights": "Schmidt form, log-uniform over 16 decades"}, dtype="f64")
    rec.update({"jacobi_rounds_per_call": rounds, "eps_rho": float(eps.cpu()[0]),
                "eps_rho_oracle": ref["eps"],
                "kernels_ms_per_call": {k: round(v[1] / calls, 4) for k, v in kernels.items()},
                "torch_gpu_eigh_ms": round(ms_torch, 3), "speedup_vs_torch_gpu_eigh": round(ms_torch / ms, 2),
                "cpu_baseline": {"value": round(1e3 / ms_cpu, 3), "unit": "density-matrix steps/s",
                                 "cores": os.cpu_count(), "kind": "oracle",
                                 "sample": "the whole workload once (numpy: rho, LAPACK eigh, selection)"},
                "kept_total": int(kept.sum().item()), "kept_matches_oracle":
                    bool(np.array_equal(kept.cpu().numpy(), ref["kept"]))})
    return rec


def bench_superblock(args, rot, torch, workloads):
    """Superblock Hamiltonian times a state (FP64): blocks B and B~ of 1024
    states in the Gaussian sector grid (45 sectors each), Hubbard-structured
    terms (block Hamiltonians, four shifting block operators per side paired
    with the site fermions, site-site hopping and interaction), the state in
    the 60 system sectors of total numbers (25, 25).  Each step is one
    rot_sb_apply."""
    import time

    import numpy as np
    case = workloads.superblock_random(1024, cfg=8)
    H = rot.SuperblockH(case.site_qn, case.left, case.right, case.target, case.left_ops, case.right_ops,
                        case.terms)
    psi = torch.from_numpy(np.random.default_rng(96).standard_normal(H.total)).cuda()
    out = torch.empty_like(psi)
    ms = timed_loop(torch, lambda: H.apply(psi, out), args.steps, args.warmup)
    # the same products replayed from a captured graph: device time without host gaps
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    reps = 10
    with torch.cuda.stream(stream):
        H.apply(psi, out)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            for _ in range(reps):
                H.apply(psi, out)
    torch.cuda.current_stream().wait_stream(stream)
    ms_graph = timed_loop(torch, graph.replay, max(2, args.steps // 2), 1) / reps
    rot.profile_enable(True)
    for _ in range(5):
        H.apply(psi, out)
    torch.cuda.synchronize()
    kernels = rot.profile_read()
    rot.profile_enable(False)
    cnt, tot = kernels["sb_matvec"]
    avg_ms = tot / cnt
    tflops = H.flops / (avg_ms / 1e3) / 1e12
    # dense reference on the GPU: the same terms on the dense Kronecker layout, torch FP64
    L, R = workloads.superblock_dense_ops(case)
    Ld = [torch.from_numpy(x).cuda() for x in L]
    Rd = [torch.from_numpy(x).cuda() for x in R]
    D = torch.from_numpy(workloads.superblock_to_dense(case, psi.cpu().numpy())).cuda().reshape(1024, 4, 4, 1024)

    def dense_step():
        acc = torch.zeros_like(D)
        for coef, lo, sa, sat, ro in case.terms:
            Y = D
            if lo >= 0:
                Y = torch.tensordot(Ld[lo], Y, dims=([1], [0]))
            if sa is not None:
                Y = torch.einsum("sk,iktj->istj", torch.from_numpy(np.asarray(sa)).cuda(), Y)
            if sat is not None:
                Y = torch.einsum("tk,iskj->istj", torch.from_numpy(np.asarray(sat)).cuda(), Y)
            if ro >= 0:
                Y = torch.tensordot(Y, Rd[ro], dims=([3], [1]))
            acc += coef * Y
        return acc

    ms_dense = timed_loop(torch, dense_step, 3, 1)
    t0 = time.perf_counter()
    from oracle import superblock as osb
    terms = [(coef, L[lo] if lo >= 0 else None, sa, sat, R[ro] if ro >= 0 else None)
             for coef, lo, sa, sat, ro in case.terms]
    osb.matvec(terms, D.reshape(4096, 4096).cpu().numpy(), 1024, 4, 1024)
    ms_cpu = (time.perf_counter() - t0) * 1e3
    rec = base_record(args, 1e3 / ms, "superblock products H psi per second", ms,
                      {"workload": "superblock_m1024", "m": 1024, "mR": 1024, "d": 4, "target": list(case.target),
                       "system_sectors": len(H.blocks), "state_length": H.total, "terms": len(case.terms)},
                      dtype="f64")
    rec.update({"flops_per_product": H.flops, "tflops_fp64": round(tflops, 2),
                "graph_replay_ms_per_product": round(ms_graph, 4),
                "kernels_ms_avg": {"sb_matvec": round(avg_ms, 4)},
                "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 78.6, "unit": "TFLOP/s",
                             "frac": round(tflops / 78.6, 4), "traffic": None, "kernel": "sb_tile_kernel",
                             "avg_ms": round(avg_ms, 4)},
                "torch_dense_fp64_ms": round(ms_dense, 3), "speedup_vs_torch_dense": round(ms_dense / ms, 2),
                "cpu_baseline": {"value": round(1e3 / ms_cpu, 4), "unit": "superblock products H psi per second",
                                 "cores": os.cpu_count(), "kind": "oracle",
                                 "sample": "one product on the dense Kronecker layout (numpy, BLAS contractions)"}})
    H.close()
    return rec


def bench_dense(args, rot, torch, workloads, name):
    """The dense shared-U workloads: `name` is the headline batch (m = m' =
    1024, 64 operators), the 512-state batch of 200 operators, or the
    64-state FP64 batch of 32 operators (launch-latency bound: also timed as
    hipGraph replays, with its algorithmic bytes per second)."""
    import numpy as np
    dev = torch.device("cuda:0")
    case = workloads.named_dense(name)
    m, d, mp, n = case.m, case.d, case.mp, case.O.shape[0]
    precision = "fp64" if name == "dense_m64_f64" else args.precision
    dt = torch.float64 if precision == "fp64" else torch.float32
    U = torch.from_numpy(case.U).to(dt).to(dev)
    O = torch.from_numpy(case.O).to(dt).to(dev)
    out = torch.empty((n, mp, mp), dtype=dt, device=dev)
    # operators whose outputs are compared with the oracle's (the CPU leg's sample)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    n_ref = n if name != WORKLOAD else max(1, min(n, nthreads))
    outputs = {}
    main_run = measure(rot, U, O, out, d, precision, args.steps, args.warmup, args.symmetric)
    outputs[precision] = out[:n_ref].double().cpu().numpy()

    result = base_record(args, main_run["ops_per_s"], "operator rotations/s", main_run["ms_per_step"],
                         {"workload": name, "m": m, "d": d, "mp": mp, "n_ops": n, "precision": precision,
                          "operators": "symmetric Gaussian / sqrt(m)" if name != "dense_m64_f64"
                          else "symmetric Gaussian",
                          "output": "upper triangle mirrored" if args.symmetric else "full",
                          "U": f"QR of seeded {m * d}x{mp} Gaussian"},
                         dtype={"fp32": "f32", "fp64": "f64", "split_bf16": "bf16x3+f32acc"}[precision])
    result["metric"] = METRIC
    result.update({
        "ms_per_step_median": round(main_run["ms_per_step_median"], 4),
        "ms_per_step_min": round(main_run["ms_per_step_min"], 4),
        "tflops": round(main_run["tflops"], 2),
        "pct_mfma_peak": round(main_run["pct_mfma_peak"], 2),
        "kernels_ms_avg": main_run["kernels_ms_avg"],
        "roofline": main_run["roofline"],
    })

    if name == "dense_m64_f64":
        # latency bound: per-batch time, graph replays, algorithmic bytes/s
        nbytes = 8.0 * (m * d * mp + n * m * m + n * mp * mp)
        p = rot._problem(U, O, out, d)
        ws = torch.empty(rot.rot_workspace_size([p], rot.ROT_FP64), dtype=torch.uint8, device=dev)
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        # ten calls per graph, so that one graph launch is spread over ten batches
        reps = 10
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            rot.rotate(U, O, d, "fp64", out=out, workspace=ws)
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=stream):
                for _ in range(reps):
                    rot.rotate(U, O, d, "fp64", out=out, workspace=ws)
        torch.cuda.current_stream().wait_stream(stream)
        ms_graph = timed_loop(torch, graph.replay, max(args.steps // reps, 10), args.warmup) / reps
        us = main_run["ms_per_step"] * 1e3
        result["unit"] = "operator rotations/s"
        result.update({"us_per_batch": round(us, 2), "us_per_batch_graph_replay": round(ms_graph * 1e3, 2),
                       "graph_calls_per_replay": reps,
                       "algorithmic_bytes_per_batch": nbytes,
                       "algorithmic_gb_per_s": round(nbytes / (main_run["ms_per_step"] / 1e3) / 1e9, 2),
                       "algorithmic_gb_per_s_graph": round(nbytes / (ms_graph / 1e3) / 1e9, 2)})
        result["roofline"] = {"bound": "hbm", "achieved": result["algorithmic_gb_per_s_graph"],
                              "peak": 8000.0, "unit": "GB/s",
                              "frac": round(result["algorithmic_gb_per_s_graph"] / 8000.0, 5), "traffic": None,
                              "kernel": "whole batch (one launch, rotate_small_f64_kernel)",
                              "note": "134 MFLOP and 2.23 MB per batch in one launch of 128 workgroups (both "
                                      "stages, operator by operator, 16 output columns each); direct calls are "
                                      "bound by the host (argument marshalling and launch), graph replays by "
                                      "the per-workgroup chain of 8 dependent products, not by bandwidth or "
                                      "matrix throughput"}
        del graph

    if precision == "fp32" and not args.no_split_bf16:
        b = measure(rot, U, O, out, d, "split_bf16", args.steps, args.warmup, args.symmetric)
        outputs["split_bf16"] = out[:n_ref].double().cpu().numpy()
        result["split_bf16"] = {"value": round(b["ops_per_s"], 2), "unit": "operator rotations/s",
                                "ms_per_step": round(b["ms_per_step"], 4),
                                "ms_per_step_median": round(b["ms_per_step_median"], 4),
                                "ms_per_step_min": round(b["ms_per_step_min"], 4),
                                "tflops_fp32_equivalent": round(b["tflops"], 2),
                                "pct_bf16_mfma_peak": round(b["pct_mfma_peak"], 2),
                                "speedup_vs_fp32": round(b["ops_per_s"] / main_run["ops_per_s"], 3),
                                "kernels_ms_avg": b["kernels_ms_avg"], "roofline": b["roofline"]}

    if precision == "fp32" and name == WORKLOAD and not (args.no_split_bf16 or args.symmetric or args.no_symmetric):
        # the headline operators are symmetric, so the symmetric-output path applies to them
        sym = {}
        for prec in ("fp32", "split_bf16"):
            r = measure(rot, U, O, out, d, prec, args.steps, args.warmup, symmetric=True)
            outputs[prec + "_symmetric_output"] = out[:n_ref].double().cpu().numpy()
            sym[prec] = {"value": round(r["ops_per_s"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                         "ms_per_step_median": round(r["ms_per_step_median"], 4),
                         "tflops_algorithmic": round(r["tflops"], 2),
                         "kernels_ms_avg": r["kernels_ms_avg"]}
        sym["unit"] = "operator rotations/s"
        sym["flops_per_op"] = flops_per_op(m, d, mp, True)
        result["symmetric_output"] = sym

    if not args.no_fp64_reference and precision != "fp64":
        U64, O64 = U.double(), O.double()
        out64 = torch.empty((n, mp, mp), dtype=torch.float64, device=dev)
        r64 = measure(rot, U64, O64, out64, d, "fp64", max(2, args.steps // 5), 1)
        result["fp64_gpu_ops_per_s"] = round(r64["ops_per_s"], 2)
        result["speedup_vs_fp64_gpu"] = round(main_run["ops_per_s"] / r64["ops_per_s"], 3)
        del U64, O64, out64
        naive = torch_fp64_naive(torch, U, O, d)
        result["torch_fp64_kron_ops_per_s"] = round(naive, 2)
        result["speedup_vs_torch_fp64_kron"] = round(main_run["ops_per_s"] / naive, 2)

    if not args.no_cpu_baseline:
        # the headline batch: one operator per host thread; the smaller
        # configurations run the oracle on the whole batch
        rec, ref = cpu_baseline(case, n, n_sample=n_ref, one_thread=name == WORKLOAD)
        result["cpu_baseline"] = rec
        result["error"] = {k: parity_error(v, ref) for k, v in outputs.items()}
        result["error"]["reference"] = (f"oracle (FP64, explicit kron) on the first {n_ref} of {n} operators; "
                                        "relative Frobenius error per operator")
        result["error"]["bound"] = 1e-12 if precision == "fp64" else 1e-5
    return result


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, n_total, n_sample=None, one_thread=True):
    """The oracle, as it stands, on a bounded sample: one operator per host
    thread (at most the whole batch; n_sample overrides), all threads of this
    process; then one operator on one thread.  Returns the record and the
    oracle's outputs for the sampled operators (the parity reference)."""
    import oracle
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    n_s = max(1, min(n_total, nthreads if n_sample is None else n_sample))
    t0 = time.perf_counter()
    ref = oracle.rotate(case.U, case.O[:n_s], case.d, nthreads=nthreads)
    dt = time.perf_counter() - t0
    rec = {"value": n_s / dt, "unit": "operator rotations/s", "cores": min(nthreads, n_s),
           "kind": "oracle",
           "sample": f"{n_s} of {n_total} operators (m={case.m}, d={case.d}, m'={case.mp}), FP64, explicit kron, "
                     f"{dt:.1f} s wall", "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    if one_thread:
        t0 = time.perf_counter()
        oracle.rotate(case.U, case.O[:1], case.d, nthreads=1)
        dt1 = time.perf_counter() - t0
        rec["sample"] += f"; then 1 operator on 1 thread, {dt1:.1f} s"
        rec["value_1thread"] = 1.0 / dt1
    return rec, ref


def parity_error(got, ref):
    """Max and median over operators of ||got_b - ref_b||_F / ||ref_b||_F."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    err = np.sqrt(((got - ref) ** 2).sum((1, 2))) / np.sqrt((ref ** 2).sum((1, 2)))
    return {"max": float(err.max()), "median": float(np.median(err)), "operators": int(err.size)}


def torch_fp64_naive(torch, U, O, d, sample=8, reps=3):
    """Operators/s of the naive PyTorch FP64 rotation (explicit kron(O_b, I_d),
    then two batched matmuls) on the GPU, for a sample of the batch: a
    reported reference point, not part of the library."""
    U64 = U.double()
    Ut64 = U64.t().contiguous()
    O64 = O[:sample].double()
    eye = torch.eye(d, dtype=torch.float64, device=U.device)
    n, m, _ = O64.shape

    def step():
        A = (O64[:, :, None, :, None] * eye[None, None, :, None, :]).reshape(n, m * d, m * d)
        return torch.matmul(Ut64, torch.matmul(A, U64))

    step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        step()
    t1.record()
    torch.cuda.synchronize()
    return n * reps / (t0.elapsed_time(t1) / 1e3)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the rotation shards by "
              "operators across GPUs but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "uneven_1000" and not os.environ.get("ROT_TUNE_CACHE"):
        # a fresh tuning cache file for this run (written by the first plan, read by the second)
        import tempfile
        os.environ["ROT_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="rot_tune_"), "tune_cache.txt")
    import torch

    import paper_0909_5662_amd as rot
    import workloads

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = 1 << 28  # 1 GiB of float32
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}))
        return

    if args.workload not in DENSE:
        fn = {"blocked_1024_n400": bench_blocked, "uneven_1000": bench_uneven,
              "differentiated_m1024_n64": bench_differentiated, "site_m1024_n64": bench_site,
              "measure_m1024": bench_measure, "density_m1024": bench_density,
              "superblock_m1024": bench_superblock}[args.workload]
        print(json.dumps(fn(args, rot, torch, workloads)), flush=True)
        return

    print(json.dumps(bench_dense(args, rot, torch, workloads, args.workload)), flush=True)


if __name__ == "__main__":
    main()
