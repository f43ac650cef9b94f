"""Benchmark of the CppFlow refinement path on one MI355X.

A step is one pass of the whole path over one request: batched FK over the
K x T candidates, the layered-graph search with its back-tracking and seed
gather, the LM iterations (linearise, FP64 block solve with refinement,
trial, accept) and the pose-error report.  Inputs are resident in HBM before
the timed region starts (the plan is uploaded once; every step restarts from
the search).

Default workload: T=300 waypoints, K=256 candidates (sigma 0.1 rad, 25%
branch-offset candidates), 50 LM iterations, seed-0 7-DOF DH robot.

Prints one JSON line.  `value` is waypoint-LM-iterations per second of the
mixed-precision path (FP32 kinematics, FP64 solve); the all-FP64 path on the
same GPU is reported beside it.  The `serving` object is the other half of
the metric: a short seeded request stream (Poisson arrivals at 200/s,
T ~ U{50..2000}, K in {128, 256, 512}, 30 LM iterations) served by
cpf_submit/cpf_poll (continuous batching, mixed precision) and by the
all-FP64 path one request at a time, with p50/p99 latency, open loop and as
a closed-loop burst.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, FP32 unpacked and FP64
PEAK_HBM_GBS = 8000.0

# Algorithmic flops of one LM waypoint-iteration (derivation in the design notes):
# linearise 964 (FK + J + residual + J^T J + J^T r), trial 436 (FK + residual),
# FP64 solve 1160, FP64 refinement 330, FP64 clamp / predicted reduction 42.
LM_FLOPS_PER_WAYPOINT_ITER = 964 + 436 + 1160 + 330 + 42
# One search pair (t, k', k): 7 sub + 7 abs-max + add + max + 2 compares.
DP_OPS_PER_PAIR = 18


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--workload", default="T300_K256",
                    choices=["T300_K256", "T1000_K512", "batch64", "batchopt", "schedule", "research",
                             "collision", "prismatic", "serve"],
                    help="T300_K256: the headline single-request line; the others are the "
                         "additional measured workloads in paper_2309_09102_amd/workloads.py")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: stream length (s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-chip", action="store_true",
                    help="skip the leg that runs the same request 256 times in one batch launch "
                         "(one plan per compute unit)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the short serving comparison (continuous batching, mixed precision, "
                         "vs all-FP64 one request at a time) that the default line carries")
    ap.add_argument("--serving-seconds", type=float, default=5.0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy three times: the known-size "
                         "reference that scales the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def calibrate_copy():
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": a.numel() * 8,
                      "bytes_written": a.numel() * 8, "repeats": 3}))


def kernel_sources_sha(files):
    """Hash of the sources a kernel is built from; counter figures taken from a
    different build of the kernel are not reported."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2309_09102_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, summary="hbm_traffic_T300_K256.json"):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("sources_sha") != kernel_sources_sha(k["sources"]):
        return None
    return k["bytes_per_launch"]


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); plans are "
              "independent, so several GPUs would shard whole requests with no collective.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload != "T300_K256":
        from paper_2309_09102_amd import workloads
        if args.workload == "T1000_K512":
            out = workloads.run_precision(iters=args.iters)
        elif args.workload == "batch64":
            out = workloads.run_batch64(iters=30)
        elif args.workload == "batchopt":
            out = workloads.run_batchopt()
        elif args.workload == "schedule":
            out = workloads.run_schedule()
        elif args.workload == "research":
            out = workloads.run_research()
        elif args.workload == "collision":
            out = workloads.run_collision()
        elif args.workload == "prismatic":
            out = workloads.run_prismatic()
        else:
            out = workloads.run_serve(duration_s=args.duration)
        print(json.dumps(out))
        return

    import torch
    from paper_2309_09102_amd import cpf, synth

    dev = torch.device("cuda:0")
    prob = synth.config2()
    T, K, iters = prob.T, prob.K, args.iters
    ctx = cpf.Context(0)

    # Targets FK(q*) by the library's FP64 FK on the device (input preparation).
    q_star = torch.tensor(prob.q_star.T.copy(), dtype=torch.float64, device=dev)
    pose, _ = ctx.fk_batch(prob.robot, q_star)
    torch.cuda.synchronize()
    prob = prob.with_targets(pose.cpu().numpy().T)

    cand_soa = torch.tensor(prob.cand.reshape(-1, 7).T.copy(), dtype=torch.float32, device=dev)

    def run_arm(prec):
        opts = cpf.make_opts(prec=prec, iters=iters)
        plan = ctx.plan(prob.robot, prob.targets, prob.cand, opts=opts)

        def step():
            ctx.fk_batch(prob.robot, cand_soa)          # batched FK over the K x T candidates
            # search, back-track, seed, LM iterations and report in one stream
            _, _, xi, rep = plan.solve(want_xi=False)
            return xi, rep

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, rep = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = {k: ctx.kernel_stats(k) for k in ("fk", "dp", "lm", "eval")}
        ctx.profile(False)
        xi, _ = plan.lm_refine(0)
        plan.free()
        return (t1 - t0) / args.steps, stats, rep, xi

    sec_mixed, st_mixed, rep_mixed, xi_mixed = run_arm("mixed")
    sec_fp64, st_fp64, rep_fp64, xi_fp64 = run_arm("fp64")

    work = T * iters
    value = work / sec_mixed

    def avg_ms(stats, k):
        ms, n = stats[k]
        return ms / max(n, 1)

    lm_ms = avg_ms(st_mixed, "lm")
    dp_ms = avg_ms(st_mixed, "dp")
    lm_flops = LM_FLOPS_PER_WAYPOINT_ITER * T * iters
    dp_flops = DP_OPS_PER_PAIR * (T - 1) * K * K
    if lm_ms >= dp_ms:
        dom, dom_ms, dom_flops = "lm_kernel<float, false, false, false>", lm_ms, lm_flops
    else:
        dom, dom_ms, dom_flops = "dp_kernel", dp_ms, dp_flops
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS, "traffic": measured_traffic(dom),
                "avg_launch_ms": dom_ms}

    out = {
        "metric": "waypoint-LM-iters/sec",
        "value": value,
        "unit": "waypoint-LM-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 kinematics + f64 solve",
        "data": "synthetic (seeded DH robot, sum-of-sinusoid path, noisy candidate plans)",
        "config": {"workload": f"single request T={T} K={K}, {iters} LM iterations",
                   "T": T, "K": K, "lm_iters": iters, "parallelism": "single GPU"},
        "fp64_path": {"value": work / sec_fp64, "ms_per_step": sec_fp64 * 1e3,
                      "speedup_mixed_over_fp64": sec_fp64 / sec_mixed},
        "kernels_ms": {"mixed": {k: avg_ms(st_mixed, k) for k in st_mixed},
                       "fp64": {k: avg_ms(st_fp64, k) for k in st_fp64}},
        "report": {"mixed": rep_mixed, "fp64": rep_fp64},
        "roofline": roofline,
    }

    if not args.no_full_chip:
        # The same request 256 times in one batch launch, one plan per
        # compute unit: what the LM kernel does with the chip full, beside
        # the single request of `value`, which leaves 255 compute units idle.
        n_plans = 256
        opts = cpf.make_opts(iters=iters)
        items = [(prob.robot, prob.targets, prob.cand)] * n_plans
        ctx.solve_batch(items[:8], opts)                          # warm-up
        ctx.profile(True)
        t0 = time.perf_counter()
        res = ctx.solve_batch(items, opts)
        t1 = time.perf_counter()
        lm_b = ctx.kernel_stats("lm")[0]
        dp_b = ctx.kernel_stats("dp")[0]
        ctx.profile(False)
        ach_b = LM_FLOPS_PER_WAYPOINT_ITER * T * iters * n_plans / (lm_b * 1e-3) / 1e12
        # bytes past the L2 for the 256-plan launch (FETCH_SIZE + WRITE_SIZE,
        # scaled by a copy of known size), from the committed counter summary
        tr_b = measured_traffic("lm_kernel<float, false, false, false>", "hbm_traffic_full_chip_T300_K256.json")
        gbs_b = tr_b / (lm_b * 1e-3) / 1e9 if tr_b else None
        out["full_chip"] = {
            "plans": n_plans, "lm_kernel_ms": lm_b, "search_ms": dp_b, "wall_ms": (t1 - t0) * 1e3,
            "waypoint_lm_iters_per_s": T * iters * n_plans / (lm_b * 1e-3),
            "lm_achieved_tflops": ach_b, "lm_frac": ach_b / PEAK_ALU_TFLOPS,
            "lm_traffic": tr_b, "lm_traffic_GBps": gbs_b,
            "lm_traffic_frac": gbs_b / PEAK_HBM_GBS if gbs_b else None,
            "results_identical": bool(all(np.array_equal(r["xi"], res[0]["xi"]) for r in res)),
            "note": "wall_ms includes uploading the 256 requests from host memory"}

    if not args.no_serving:
        # The serving half of the metric: the same seeded request stream
        # (Poisson 200/s, T ~ U{50..2000}, K in {128, 256, 512}, 30 LM
        # iterations) served by continuous batching in mixed precision and
        # one request at a time by the all-FP64 path, open loop and as a
        # closed-loop burst; latencies are submit -> result.
        from paper_2309_09102_amd import workloads
        sv = workloads.run_serve(duration_s=args.serving_seconds, burst=240,
                                 fp64_budget_s=args.serving_seconds)
        keep = ("throughput", "p50_ms", "p99_ms", "wall_s", "requests", "requests_served",
                "requests_offered", "statuses")
        out["serving"] = {k: ({kk: vv for kk, vv in v.items() if kk in keep} if isinstance(v, dict) else v)
                          for k, v in sv.items()}

    if not args.no_cpu_baseline:
        import oracle
        threads = 1
        t0 = time.perf_counter()
        n = 0
        ref = None
        while True:
            ref = oracle.plan(prob.robot, prob.cand, prob.targets, iters)
            n += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = (time.perf_counter() - t0) / n
        out["cpu_baseline"] = {"value": work / dt, "unit": "waypoint-LM-iters/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{n} full runs of the same request (search + {iters} LM "
                                         f"iterations), FP64 C oracle, 1 thread, "
                                         f"{platform.processor() or platform.machine()}"}
        ep_m, er_m = oracle.pose_compare(prob.robot, xi_mixed, ref["xi"])
        ep_d, er_d = oracle.pose_compare(prob.robot, xi_fp64, ref["xi"])
        out["pose_err_vs_oracle"] = {"mixed": [ep_m, er_m], "fp64": [ep_d, er_d],
                                     "unit": ["m", "rad"]}
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
