"""Benchmark of the CppFlow refinement path on one MI355X.

Headline (the metric's own workload): the serving stream.  Requests arrive
as a Poisson stream at 200 per second; each has T ~ U{50..2000} waypoints,
K in {128, 256, 512} candidate plans (sigma ~ U[0.02, 0.15], branch-offset
fraction ~ U[0, 0.3]) on the seed-0 7-DOF DH robot and asks for the search
plus 30 LM iterations.  Every request is distinct (seeded), and the inputs
of all of them are resident in HBM before the stream starts.  A step is one
second of the arrival stream (about 200 requests, each a whole pass of the
path: staging, search with its lists and back-tracking, 30 LM iterations,
report); --warmup W serves the first W seconds untimed, --steps K times the
next K seconds.  `value` is waypoint-LM-iterations per second of the
continuously batched mixed-precision server (FP32 Jacobian, FP64 residual,
cost and solve) on that open-loop schedule (submit of the first timed
request to completion of the last); p50/p99 latency is submit -> result.
Beside it: the same requests all at once (saturation), the all-FP64 arm
continuously batched, and the plain all-FP64 path one request at a time on
the same schedule.

The line also carries the roofline of the kernel with the most device time
in the timed stream, the oracle's throughput on the host's cores
(cpu_baseline) with the served results' pose errors against it, and, as
context, the single T=300/K=256 request, the same request 256 times in one
launch (chip full) and the 64-problem ragged batch.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HIP maps a process's streams onto a pool of hardware queues (4 by default),
# and streams that share a queue run one after the other.  The server keeps
# three streams busy at once (LM ticks and two search lanes) in a process
# that also holds torch's streams, so with four queues two of them can land
# on one queue (measured: open-loop p50 16.1 ms and p99 36 ms against 12.4
# and 24 ms with eight).  The pool size is read when HIP starts, so it is
# raised here, before anything imports torch.
def _hw_queues() -> int:
    try:
        return int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
    except ValueError:
        return 0


if _hw_queues() < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

PEAK_ALU_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, FP32 unpacked and FP64
PEAK_HBM_GBS = 8000.0

# Algorithmic operations of one LM waypoint-iteration.  The survey's count
# of the method (FK, Jacobian and residual of the linearisation and of the
# trial, 7x7 Cholesky, block elimination, sweeps and refinement) is about
# 1.3k + 0.6k; this build's own tally of the same steps (derivation in the
# design notes) is 2,932 because it counts the block solve's products in
# full.  `frac` uses the smaller count; `frac_own_count` the larger.
LM_OPS_SURVEY = 1900
LM_OPS_OWN = 964 + 436 + 1160 + 330 + 42
# One search pair (t, k', k): 7 sub + 7 abs-max + add + max + 2 compares.
DP_OPS_PER_PAIR = 18


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="seconds of the arrival stream timed (about 200 requests each)")
    ap.add_argument("--warmup", type=int, default=5, help="seconds of the arrival stream served untimed")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--iters", type=int, default=30, help="LM iterations per request")
    ap.add_argument("--workload", default="serve",
                    choices=["serve", "T300_K256", "T1000_K512", "batch64", "batchopt", "schedule", "research",
                             "collision", "prismatic", "lm_phases"],
                    help="serve: the headline line; the others print the additional measured workloads "
                         "of paper_2309_09102_amd/workloads.py")
    ap.add_argument("--fp64-budget", type=float, default=None,
                    help="seconds after which the one-at-a-time FP64 arm starts no further request "
                         "(default: the timed stream's length)")
    ap.add_argument("--open-loop-only", action="store_true",
                    help="serve only the mixed open-loop stream (for counter runs: every search and LM "
                         "dispatch then belongs to the warm-up and timed requests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context-legs", action="store_true",
                    help="skip the single-request, chip-full and 64-problem legs")
    ap.add_argument("--cpu-seconds", type=float, default=30.0,
                    help="wall budget of the oracle on the sampled stream requests (all host cores)")
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


def measured_traffic(kernel, summary):
    """Record of `kernel` in a committed counter summary (HBM bytes per
    launch and per unit of work), or None when the kernel's sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("sources_sha") != kernel_sources_sha(k["sources"]):
        return None
    return k


def cpu_info():
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def oracle_threads():
    """Host threads for the oracle: the cores this process may use, at most
    16 (the GPU machine's share)."""
    return max(1, min(16, cpu_info()[1]))


# ---- the serving headline ----------------------------------------------------

def roofline_of(summary, raw, iters):
    """Roofline object of the kernel with the most device time in the timed
    open-loop stream: algorithmic operations of all its launches over their
    summed duration."""
    ks = summary["mixed_open"]["kernels"]
    timed = raw["timed"]
    lm_units = sum(T for _, T, _ in timed) * iters
    pairs = sum((T - 1) * K * K for _, T, K in timed)
    cand = {"lm": ("lm_kernel<float, false, false, false> (tick graph)", lm_units * LM_OPS_SURVEY,
                   lm_units * LM_OPS_OWN, f"{lm_units} waypoint-LM-iterations x {LM_OPS_SURVEY} ops"),
            "dp_lists": ("dp_topm_kernel", pairs * DP_OPS_PER_PAIR, pairs * DP_OPS_PER_PAIR,
                         f"{pairs} search pairs x {DP_OPS_PER_PAIR} FP64 ops"),
            "dp": ("dp_kernel<512, 2>", None, None, "stage recursion (one workgroup per plan)")}
    dom = max(("lm", "dp_lists", "dp"), key=lambda k: ks[k]["ms"])
    name, flops, flops_own, unit = cand[dom]
    ms, n = ks[dom]["ms"], ks[dom]["launches"]
    roof = {"bound": "alu", "kernel": name, "unit": "TFLOP/s", "peak": PEAK_ALU_TFLOPS,
            "launches": n, "avg_launch_ms": ms / max(n, 1), "work": unit,
            "device_ms": {k: v["ms"] for k, v in ks.items()}}
    if flops is not None:
        ach = flops / (ms * 1e-3) / 1e12
        roof.update({"achieved": ach, "frac": ach / PEAK_ALU_TFLOPS,
                     "frac_own_count": flops_own / (ms * 1e-3) / 1e12 / PEAK_ALU_TFLOPS})
    rec = measured_traffic("serving:" + dom, "hbm_traffic_serving.json")
    if rec is not None:
        per_unit = rec["bytes_per_unit"]
        units = lm_units if dom == "lm" else pairs
        roof["traffic"] = per_unit * units / max(n, 1)
        roof["traffic_GBps"] = per_unit * units / (ms * 1e-3) / 1e9
    else:
        roof["traffic"] = None
    return roof


# ---- the oracle leg (cpu_baseline) -------------------------------------------

def _parallel(fn, items, threads, deadline=None):
    """fn over items on `threads` host threads (the C oracle runs outside the
    interpreter lock); items not started before `deadline` are skipped.
    Returns (results in item order, None where skipped), wall seconds."""
    from concurrent.futures import ThreadPoolExecutor

    def run(x):
        if deadline is not None and time.perf_counter() > deadline:
            return None
        return fn(x)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(run, items))
    return res, time.perf_counter() - t0


def cpu_baseline_leg(args, summary, raw, ctx_results):
    """The FP64 C oracle on the host: the sampled serving requests on all
    cores (throughput, and the served results' errors against it), configs
    1-3 on one core, the 64-problem batch on all cores."""
    import oracle
    from paper_2309_09102_amd import synth
    model, avail = cpu_info()
    threads = oracle_threads()
    iters = args.iters
    timed = raw["timed"]
    # every 20th timed request and the 20 longest
    idx = [timed[k][0] for k in range(0, len(timed), 20)]
    longest = sorted(timed, key=lambda x: -x[1])[:20]
    idx = sorted(set(idx) | {i for i, _, _ in longest})
    served = raw["mixed_open"]["xi"]
    fp64 = raw["fp64_one_at_a_time_open"]["xi"]
    gpu_tg = raw.get("targets", {})

    def solve(i):
        p = synth.config5_request(i)
        p = p.with_targets(oracle.fk(p.robot, p.q_star))
        t0 = time.perf_counter()
        ref = oracle.plan(p.robot, p.cand, p.targets, iters)
        dt = time.perf_counter() - t0
        rec = {"i": i, "T": p.T, "K": p.K, "sec": dt,
               "targets_equal": bool(i in gpu_tg and np.array_equal(gpu_tg[i], p.targets))}
        c_ref = oracle.cost(p.robot, ref["xi"], p.targets)
        for arm, xs in (("mixed_served", served), ("fp64_one_at_a_time", fp64)):
            if i in xs:
                ep, er = oracle.pose_compare(p.robot, xs[i], ref["xi"])
                c = oracle.cost(p.robot, xs[i], p.targets)
                rec[arm] = [ep, er, abs(c - c_ref) / max(c_ref, 1e-12)]
        return rec

    deadline = time.perf_counter() + args.cpu_seconds
    recs, wall = _parallel(solve, idx, threads, deadline)
    done = [r for r in recs if r is not None]
    work = sum(r["T"] for r in done) * iters

    def dist(arm):
        v = np.array([r[arm] for r in done if arm in r])
        if not len(v):
            return None
        return {"n": int(len(v)), "pos_m": {"p50": float(np.median(v[:, 0])), "p99": float(np.percentile(v[:, 0], 99)),
                                            "max": float(v[:, 0].max())},
                "rot_rad": {"p50": float(np.median(v[:, 1])), "p99": float(np.percentile(v[:, 1], 99)),
                            "max": float(v[:, 1].max())},
                "rel_cost_gap": {"p50": float(np.median(v[:, 2])), "max": float(v[:, 2].max())},
                "within_1e-5_m_rad": bool(v[:, 0].max() <= 1e-5 and v[:, 1].max() <= 1e-5),
                "within_1e-6_cost": bool(v[:, 2].max() <= 1e-6)}

    cb = {"value": work / wall, "unit": "waypoint-LM-iters/s", "cores": threads, "kind": "oracle",
          "sample": (f"{len(done)} of {len(idx)} sampled serving-stream requests (every 20th timed request "
                     f"and the 20 longest; search + {iters} LM iterations each), FP64 C oracle on "
                     f"{threads} host threads, {wall:.1f} s wall"),
          "cpu_model": model, "host_cores_available": avail}
    pose = {"mixed_served": dist("mixed_served"), "fp64_one_at_a_time": dist("fp64_one_at_a_time"),
            "sampled_requests": len(done),
            "targets_bitwise_equal": int(sum(r["targets_equal"] for r in done)),
            "note": "oracle targets from its own FP64 FK of q*, rounded to float32 like the GPU's"}

    # configs 1-3 on one core (median of a few runs), config 4 on all cores
    def one_core(p, it, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.plan(p.robot, p.cand, p.targets, it)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    c1 = synth.config1()
    c1 = c1.with_targets(oracle.fk(c1.robot, c1.q_star))
    t1 = one_core(c1, 20, 5)
    cfg = {"config1": {"T": 50, "K": 16, "lm_iters": 20, "cores": 1, "latency_ms": t1 * 1e3,
                       "waypoint_lm_iters_per_s": 50 * 20 / t1}}
    c2 = synth.config2()
    c2 = c2.with_targets(oracle.fk(c2.robot, c2.q_star))
    t2 = one_core(c2, 50, 3)
    cfg["config2"] = {"T": 300, "K": 256, "lm_iters": 50, "cores": 1, "latency_ms": t2 * 1e3,
                      "waypoint_lm_iters_per_s": 300 * 50 / t2}
    if ctx_results.get("config2_xi"):
        ref2 = oracle.plan(c2.robot, c2.cand, c2.targets, 50)
        c_ref = oracle.cost(c2.robot, ref2["xi"], c2.targets)
        cfg["config2"]["gpu_err_vs_oracle"] = {
            arm: list(oracle.pose_compare(c2.robot, xi, ref2["xi"])) +
            [abs(oracle.cost(c2.robot, xi, c2.targets) - c_ref) / c_ref]
            for arm, xi in ctx_results["config2_xi"].items()}
    c3 = synth.config3()
    c3 = c3.with_targets(oracle.fk(c3.robot, c3.q_star))
    t0 = time.perf_counter()
    ref3 = oracle.plan(c3.robot, c3.cand, c3.targets, 50)
    t3 = time.perf_counter() - t0
    cfg["config3"] = {"T": 1000, "K": 512, "lm_iters": 50, "cores": 1, "latency_ms": t3 * 1e3,
                      "waypoint_lm_iters_per_s": 1000 * 50 / t3}
    if "config3_xi" in ctx_results:
        cfg["config3"]["gpu_pose_err_vs_oracle"] = {
            arm: list(oracle.pose_compare(c3.robot, xi, ref3["xi"])) for arm, xi in ctx_results["config3_xi"].items()}
    if "batch64_probs" in ctx_results:
        probs = [p.with_targets(oracle.fk(p.robot, p.q_star)) for p in ctx_results["batch64_probs"]]
        _, w4 = _parallel(lambda p: oracle.plan(p.robot, p.cand, p.targets, 30), probs, threads)
        cfg["config4"] = {"problems": len(probs), "lm_iters": 30, "cores": threads, "wall_s": w4,
                          "waypoint_lm_iters_per_s": sum(p.T for p in probs) * 30 / w4}
    cb["configs"] = cfg
    return cb, pose


# ---- context legs --------------------------------------------------------------

def context_legs(args, out, ctx_results):
    """The single T=300/K=256 request (mixed and FP64, each step a fresh full
    search + 50 LM iterations + report on resident inputs), the same request
    256 times in one launch, the T=1000/K=512 precision study and the
    64-problem ragged batch."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2309_09102_amd import cpf, synth, workloads
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)

    def targets_of(p):
        q = torch.tensor(p.q_star.T.copy(), dtype=torch.float64, device=dev)
        pose, _ = ctx.fk_batch(p.robot, q)
        torch.cuda.synchronize()
        return p.with_targets(pose.cpu().numpy().T)

    ctx_results["config2_xi"] = {}
    out["single_request"] = workloads.run_single(ctx=ctx, iters=50, xi_out=ctx_results["config2_xi"])
    prob = targets_of(synth.config2())
    T, iters = prob.T, 50

    # the same request 256 times in one launch: one plan per compute unit
    n_plans = 256
    opts = cpf.make_opts(iters=iters)
    items = [(prob.robot, prob.targets, prob.cand)] * n_plans
    ctx.solve_batch(items[:8], opts)
    ctx.profile(True)
    res = ctx.solve_batch(items, opts)
    lm_b = ctx.kernel_stats("lm")[0]
    sr_b = ctx.kernel_stats("dp")[0] + ctx.kernel_stats("dp_lists")[0]
    ctx.profile(False)
    rec = measured_traffic("lm_kernel<float, false, false, false>", "hbm_traffic_full_chip_T300_K256.json")
    tr = rec["bytes_per_launch"] if rec else None
    out["full_chip"] = {"plans": n_plans, "lm_kernel_ms": lm_b, "search_ms": sr_b,
                        "waypoint_lm_iters_per_s": T * iters * n_plans / (lm_b * 1e-3),
                        "lm_frac": T * iters * n_plans * LM_OPS_SURVEY / (lm_b * 1e-3) / 1e12 / PEAK_ALU_TFLOPS,
                        "lm_traffic": tr, "lm_traffic_GBps": tr / (lm_b * 1e-3) / 1e9 if tr else None,
                        "results_identical": bool(all(np.array_equal(r["xi"], res[0]["xi"]) for r in res))}
    # the all-FP64 arm of the same 256 plans (the precision comparison at full chip)
    o64 = cpf.make_opts(iters=iters, prec="fp64")
    ctx.solve_batch(items[:8], o64)
    ctx.profile(True)
    res64 = ctx.solve_batch(items, o64)
    lm64 = ctx.kernel_stats("lm")[0]
    ctx.profile(False)
    out["full_chip"]["fp64"] = {"lm_kernel_ms": lm64, "waypoint_lm_iters_per_s": T * iters * n_plans / (lm64 * 1e-3),
                                "results_identical": bool(all(np.array_equal(r["xi"], res64[0]["xi"]) for r in res64))}

    # precision study T=1000, K=512 (pose errors against the oracle in the cpu_baseline leg)
    p3 = targets_of(synth.config3())
    xs = {}
    prec_study = {}
    for prec in ("mixed", "fp64"):
        with ctx.plan(p3.robot, p3.targets, p3.cand, opts=cpf.make_opts(prec=prec, iters=50)) as plan:
            plan.solve(want_xi=False)
            t0 = time.perf_counter()
            _, _, xi, rep = plan.solve(want_xi=True)
            dt = time.perf_counter() - t0
        xs[prec] = xi
        prec_study[prec] = {"latency_ms": dt * 1e3, "waypoint_lm_iters_per_s": 1000 * 50 / dt}
    out["precision_study_T1000_K512"] = prec_study
    ctx_results["config3_xi"] = xs

    # 64 ragged problems in one launch of each kernel
    with ThreadPoolExecutor(max_workers=8) as ex:
        probs = list(ex.map(synth.config4_problem, range(64)))
    ctx_results["batch64_probs"] = probs
    probs_t = [targets_of(p) for p in probs]
    o4 = cpf.make_opts(iters=30)
    items = [(p.robot, p.targets, p.cand) for p in probs_t]
    ctx.solve_batch(items[:2], o4)
    ctx.profile(True)
    t0 = time.perf_counter()
    ctx.solve_batch(items, o4)
    t1 = time.perf_counter()
    st = {k: ctx.kernel_stats(k)[0] for k in ("dp_lists", "dp", "lm", "eval")}
    ctx.profile(False)
    work = sum(p.T for p in probs_t) * 30
    dev_ms = sum(st.values())
    lm_frac = work * LM_OPS_SURVEY / (st["lm"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS
    pairs = sum((p.T - 1) * p.K * p.K for p in probs_t)
    out["batch64"] = {"problems": 64, "lm_iters": 30, "device_ms": dev_ms, "kernels_ms": st,
                      "waypoint_lm_iters_per_s_device": work / (dev_ms * 1e-3),
                      "waypoint_lm_iters_per_s_end_to_end": work / (t1 - t0),
                      "lm_frac": lm_frac,
                      "lists_frac": pairs * DP_OPS_PER_PAIR / (st["dp_lists"] * 1e-3) / 1e12 / PEAK_ALU_TFLOPS}
    ctx.close()


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

    if args.workload != "serve":
        from paper_2309_09102_amd import workloads
        fn = {"T300_K256": workloads.run_single, "T1000_K512": workloads.run_precision,
              "batch64": lambda: workloads.run_batch64(iters=30), "batchopt": workloads.run_batchopt,
              "schedule": workloads.run_schedule, "research": workloads.run_research,
              "collision": workloads.run_collision, "prismatic": workloads.run_prismatic,
              "lm_phases": workloads.run_lm_phases}[args.workload]
        print(json.dumps(fn()))
        return

    import torch  # noqa: F401
    from paper_2309_09102_amd import workloads

    summary, raw = workloads.run_serve(duration_s=float(args.steps), warmup_s=float(args.warmup),
                                       rate_hz=args.rate, iters=args.iters, fp64_budget_s=args.fp64_budget,
                                       keep_xi="sample", open_loop_only=args.open_loop_only)
    mo = summary["mixed_open"]
    if args.open_loop_only:
        print(json.dumps({"open_loop_only": True, "summary": summary, "roofline": roofline_of(summary, raw, args.iters)}))
        return
    out = {
        "metric": "waypoint-LM-iters/sec",
        "value": mo["throughput"],
        "unit": "waypoint-LM-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mo["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 residuals/cost/solve, f32 Jacobian",
        "data": "synthetic (seeded DH robot, sum-of-sinusoid paths, noisy candidate plans; every request distinct)",
        "config": {"workload": (f"serving stream: Poisson {args.rate:.0f} req/s for {args.steps} s "
                                f"({summary['requests']} distinct requests, inputs resident in HBM), "
                                f"T ~ U{{50..2000}}, K in {{128, 256, 512}}, {args.iters} LM iterations, "
                                "continuous batching, mixed precision"),
                   "rate_hz": args.rate, "duration_s": args.steps, "requests": summary["requests"],
                   "lm_iters": args.iters, "slots": summary["slots"], "iters_per_tick": summary["iters_per_tick"],
                   "tick_budget": summary["tick_budget"],
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": mo["p50_ms"], "p99": mo["p99_ms"], "max": mo["max_ms"]},
        "offered_load": summary["offered_load"],
        "saturation": summary["mixed_closed"],
        "saturation_host_inputs": summary.get("mixed_closed_host_inputs"),
        "fp64_batched_closed": summary["fp64_closed"],
        "fp64_one_at_a_time": summary["fp64_one_at_a_time_open"],
        "speedup_vs_fp64_one_at_a_time": {"open_loop": summary["speedup_open"],
                                          "saturation": summary["speedup_closed_vs_one_at_a_time"]},
        "speedup_mixed_vs_fp64_batched": summary["speedup_mixed_vs_fp64_batched"],
        "serving_kernels_ms": mo["kernels"],
        "input_prep_s": summary["input_prep_s"],
        "input_bytes_resident": summary["input_bytes_resident"],
    }
    out["roofline"] = roofline_of(summary, raw, args.iters)

    ctx_results = {}
    if not args.no_context_legs:
        context_legs(args, out, ctx_results)
    if not args.no_cpu_baseline:
        cb, pose = cpu_baseline_leg(args, summary, raw, ctx_results)
        out["cpu_baseline"] = cb
        out["pose_err_vs_oracle"] = pose
    print(json.dumps(out))


if __name__ == "__main__":
    main()
