"""Additional measured workloads of the refinement path (bench.py --workload).

  batch64    64 independent problems of uneven size (T ~ U{100..1000},
             K ~ U{64..512}, a fresh robot each), search + 30 LM iterations,
             FP32 kinematics with FP64 solve, one launch of each kernel.
  T1000_K512 one request with T=1000, K=512, 50 LM iterations; the mixed arm
             (FP32 kinematics + FP64 solve + one FP64 refinement step) and the
             all-FP64 arm (their agreement with the oracle is a GPU test).
  batchopt   the 5 smoothest candidates of the T=300, K=256 request optimised
             directly without the search, 50 LM iterations each.
  schedule   the T=300, K=256 request refined for 50 iterations by the
             alternating schedule with anytime validity (both precisions),
             beside the weighted objective.
  research   the T=300, K=256 request searched, 256 more candidates appended
             and the search repeated, against a fresh plan over all 512.
  collision  the T=300, K=256 request with link capsules and six cuboid
             obstacles: the collision checker over all candidates, the search
             with the collision penalty and the LM with collision residuals,
             beside the request without geometry.
  serve      Poisson arrivals (200 requests/s) of requests with T ~ U{50..2000},
             K in {128, 256, 512}, sigma ~ U[0.02, 0.15], offset fraction
             ~ U[0, 0.3] and 30 LM iterations, served by cpf_submit/cpf_poll
             (continuous batching, mixed precision), and the same arrival
             schedule served one request at a time by the all-FP64 path;
             then a closed-loop burst (saturation) both ways.  Requests are
             drawn from a pool of distinct seeded problems that the stream
             cycles through (the pool keeps host memory bounded).

Every mode prints one JSON object; inputs are synthetic and seeded.
"""
from __future__ import annotations

import json
import threading
import time

import numpy as np


def _targets(ctx, prob, torch, dev):
    q = torch.tensor(prob.q_star.T.copy(), dtype=torch.float64, device=dev)
    pose, _ = ctx.fk_batch(prob.robot, q)
    torch.cuda.synchronize()
    return prob.with_targets(pose.cpu().numpy().T)


def run_batch64(n=64, iters=30):
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    probs = [_targets(ctx, synth.config4_problem(i), torch, dev) for i in range(n)]
    opts = cpf.make_opts(iters=iters, prec="mixed")
    items = [(p.robot, p.targets, p.cand) for p in probs]
    ctx.solve_batch(items[:2], opts)                  # warm-up (code objects)
    ctx.profile(True)
    t0 = time.perf_counter()
    res = ctx.solve_batch(items, opts)
    t1 = time.perf_counter()
    st = {k: ctx.kernel_stats(k) for k in ("dp", "lm", "eval")}
    ctx.profile(False)
    work = sum(p.T for p in probs) * iters
    dev_ms = sum(v[0] for v in st.values())
    out = {"mode": "batch64", "problems": n, "lm_iters": iters,
           "waypoint_lm_iters": work,
           "value_end_to_end": work / (t1 - t0), "value_device": work / (dev_ms * 1e-3),
           "unit": "waypoint-LM-iters/s", "wall_s": t1 - t0,
           "kernels_ms": {k: v[0] for k, v in st.items()},
           "statuses": sorted(set(int(r["status"]) for r in res))}
    ctx.close()
    return out


def run_precision(iters=50):
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    p = _targets(ctx, synth.config3(), torch, dev)
    out = {"mode": "T1000_K512", "T": p.T, "K": p.K, "lm_iters": iters, "arms": {}}
    for arm, prec in (("A_mixed", "mixed"), ("B_fp64", "fp64")):
        plan = ctx.plan(p.robot, p.targets, p.cand, opts=cpf.make_opts(prec=prec))
        plan.dp_search()
        plan.lm_refine(1)                              # warm-up
        ctx.profile(True)
        t0 = time.perf_counter()
        plan.dp_search()
        _, rep = plan.lm_refine(iters, want_xi=False)
        t1 = time.perf_counter()
        st = {k: ctx.kernel_stats(k) for k in ("dp", "lm")}
        ctx.profile(False)
        plan.free()
        out["arms"][arm] = {"latency_ms": (t1 - t0) * 1e3,
                            "waypoint_lm_iters_per_s": p.T * iters / (t1 - t0),
                            "kernels_ms": {k: v[0] for k, v in st.items()},
                            "pose_err_vs_targets": [rep["max_pos_err_m"], rep["max_rot_err_rad"]]}
    ctx.close()
    return out


def run_batchopt(M=5, iters=50):
    """The M smoothest of the T=300, K=256 request's candidates optimised
    directly (no search), both precisions."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    p = _targets(ctx, synth.config2(), torch, dev)
    out = {"mode": "batchopt", "T": p.T, "K": p.K, "M": M, "lm_iters": iters, "arms": {}}
    for arm, prec in (("mixed", "mixed"), ("fp64", "fp64")):
        o = cpf.make_opts(iters=iters, prec=prec)
        ctx.batchopt(p.robot, p.targets, p.cand, M, opts=o)           # warm-up
        reps = []
        t0 = time.perf_counter()
        for _ in range(3):
            idx, res = ctx.batchopt(p.robot, p.targets, p.cand, M, opts=o)
        dt = (time.perf_counter() - t0) / 3
        costs = [r["report"]["cost"] for r in res]
        out["arms"][arm] = {"latency_ms": dt * 1e3,
                            "waypoint_lm_iters_per_s": M * p.T * iters / dt,
                            "candidates": idx, "final_cost": costs,
                            "best": idx[int(np.argmin(costs))],
                            "pose_err_vs_targets_best": [res[int(np.argmin(costs))]["report"]["max_pos_err_m"],
                                                         res[int(np.argmin(costs))]["report"]["max_rot_err_rad"]]}
    ctx.close()
    return out


def run_schedule(iters=50):
    """The T=300, K=256 request refined by the alternating schedule with
    anytime validity, both precisions, beside the weighted objective."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    p = _targets(ctx, synth.config2(), torch, dev)
    out = {"mode": "schedule", "T": p.T, "K": p.K, "lm_iters": iters, "arms": {}}
    for arm, prec, sched in (("schedule_mixed", "mixed", 1), ("schedule_fp64", "fp64", 1),
                             ("weighted_mixed", "mixed", 0)):
        o = cpf.make_opts(prec=prec, schedule=sched)
        with ctx.plan(p.robot, p.targets, p.cand, opts=o) as plan:
            plan.dp_search()
            plan.lm_refine(1)                          # warm-up
        with ctx.plan(p.robot, p.targets, p.cand, opts=o) as plan:
            plan.dp_search()
            ctx.profile(True)
            t0 = time.perf_counter()
            _, rep = plan.lm_refine(iters, want_xi=False)
            t1 = time.perf_counter()
            lm_ms = ctx.kernel_stats("lm")[0]
            ctx.profile(False)
        a = {"latency_ms": (t1 - t0) * 1e3, "lm_kernel_ms": lm_ms,
             "waypoint_lm_iters_per_s": p.T * iters / (lm_ms * 1e-3),
             "final_pose_err": [rep["max_pos_err_m"], rep["max_rot_err_rad"]],
             "final_mjac": rep["mjac"]}
        if sched:
            a.update({k: rep[k] for k in ("n_valid", "first_valid", "pose_steps", "diff_steps",
                                          "valid_length")})
        out["arms"][arm] = a
    ctx.close()
    return out


def run_research(K_add=256, reps=5):
    """The T=300, K=256 request searched, then K_add more candidates
    appended and the search repeated (Sec. III-B), against a fresh plan over
    all K + K_add candidates searched from scratch."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    p = _targets(ctx, synth.config2(), torch, dev)
    extra = synth.more_candidates(p, K_add)
    allc = np.concatenate([p.cand, extra])
    out = {"mode": "research", "T": p.T, "K": p.K, "K_add": K_add, "reps": reps}
    app, fresh, app_dev, fresh_dev, mj = [], [], [], [], []
    for r in range(reps + 1):
        with ctx.plan(p.robot, p.targets, p.cand) as plan:
            plan.dp_search()
            ctx.profile(True)
            t0 = time.perf_counter()
            plan.append(extra)
            _, best_a, mj_a = plan.dp_search()
            t1 = time.perf_counter()
            dev_a = ctx.kernel_stats("dp")[0]
            ctx.profile(False)
        ctx.profile(True)
        t2 = time.perf_counter()
        with ctx.plan(p.robot, p.targets, allc) as plan:
            _, best_f, _ = plan.dp_search()
        t3 = time.perf_counter()
        dev_f = ctx.kernel_stats("dp")[0]
        ctx.profile(False)
        assert best_a == best_f
        if r:   # the first round warms up
            app.append(t1 - t0)
            fresh.append(t3 - t2)
            app_dev.append(dev_a)
            fresh_dev.append(dev_f)
            mj.append(mj_a)
    out.update({"append_and_research_ms": 1e3 * float(np.median(app)),
                "fresh_plan_and_search_ms": 1e3 * float(np.median(fresh)),
                "append_device_ms": float(np.median(app_dev)),
                "fresh_search_device_ms": float(np.median(fresh_dev)),
                "seed_mjac_before_after": [None, float(mj[0])]})
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        _, _, mj0 = plan.dp_search()
    out["seed_mjac_before_after"][0] = float(mj0)
    ctx.close()
    return out


def run_collision(iters=50, n_obs=6, obstacle_seed=4):
    """The T=300, K=256 request with a capsule on every link and six cuboid
    obstacles: the collision checker over all K x T candidates, the search
    with the collision penalty, and 50 LM iterations with the collision
    residuals, both precisions, beside the same request without geometry."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    p = _targets(ctx, synth.config2(), torch, dev)
    coll = synth.collision_model(p.robot, synth.make_obstacles(obstacle_seed, n_obs))
    out = {"mode": "collision", "T": p.T, "K": p.K, "n_obstacles": n_obs, "lm_iters": iters, "arms": {}}
    q = p.cand.reshape(-1, 7)
    for name, dt in (("checker_fp32", torch.float32), ("checker_fp64", torch.float64)):
        qd = torch.tensor(q.T.copy(), dtype=dt, device=dev)
        ctx.coll_batch(p.robot, coll, qd)                      # warm-up
        ctx.profile(True)
        dist, _ = ctx.coll_batch(p.robot, coll, qd)
        torch.cuda.synchronize()
        ms = ctx.kernel_stats("fk")[0]
        ctx.profile(False)
        out[name] = {"configs": q.shape[0], "kernel_ms": ms, "configs_per_s": q.shape[0] / (ms * 1e-3),
                     "colliding_frac": float((dist < 0).any(dim=0).float().mean())}
    for arm, prec, c in (("coll_mixed", "mixed", coll), ("coll_fp64", "fp64", coll), ("plain_mixed", "mixed", None)):
        o = cpf.make_opts(prec=prec)
        with ctx.plan(p.robot, p.targets, p.cand, opts=o, coll=c) as plan:
            plan.dp_search()
            plan.lm_refine(1)                                  # warm-up
        with ctx.plan(p.robot, p.targets, p.cand, opts=o, coll=c) as plan:
            ctx.profile(True)
            t0 = time.perf_counter()
            _, best, mj = plan.dp_search()
            _, rep = plan.lm_refine(iters, want_xi=False)
            t1 = time.perf_counter()
            st = {k: ctx.kernel_stats(k)[0] for k in ("dp", "lm")}
            ctx.profile(False)
        out["arms"][arm] = {"latency_ms": (t1 - t0) * 1e3, "kernels_ms": st, "search_best": best,
                            "seed_mjac": mj, "waypoint_lm_iters_per_s": p.T * iters / (st["lm"] * 1e-3),
                            "pose_err_vs_targets": [rep["max_pos_err_m"], rep["max_rot_err_rad"]],
                            "min_self_dist_m": rep["min_self_dist_m"], "min_env_dist_m": rep["min_env_dist_m"]}
    ctx.close()
    return out


def run_prismatic(iters=50, robot_seed=0):
    """The T=300, K=256 request (seed 2, sigma 0.1, a quarter of the
    candidates branch-offset) on the robot of the same seed with a prismatic
    first joint (travel 0-0.4 m): the search with the seed's steps split by
    joint type and the re-search decision (12 deg / 3 cm), then 50 LM
    iterations in both precisions and the alternating schedule with its 2 cm
    step threshold, beside the all-revolute robot on the same request."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    out = {"mode": "prismatic", "T": 300, "K": 256, "lm_iters": iters, "arms": {}}
    robots = (("prismatic", synth.make_robot_prismatic(robot_seed)), ("revolute", synth.make_robot(robot_seed)))
    for rname, rb in robots:
        p = _targets(ctx, synth.make_problem(rb, seed=2, T=300, K=256, sigma=0.1, branch_frac=0.25), torch, dev)
        arms = (("mixed", dict(prec="mixed")), ("fp64", dict(prec="fp64")),
                ("schedule_mixed", dict(prec="mixed", schedule=1)))
        for arm, kw in arms:
            o = cpf.make_opts(**kw)
            with ctx.plan(p.robot, p.targets, p.cand, opts=o) as plan:
                plan.dp_search()
                plan.lm_refine(1)                              # warm-up
            with ctx.plan(p.robot, p.targets, p.cand, opts=o) as plan:
                ctx.profile(True)
                t0 = time.perf_counter()
                _, best, mj = plan.dp_search()
                rev, pri = plan.seed_steps()
                _, rep = plan.lm_refine(iters, want_xi=False)
                t1 = time.perf_counter()
                st = {k: ctx.kernel_stats(k)[0] for k in ("dp", "lm")}
                ctx.profile(False)
                research = plan.needs_research()
            out["arms"][f"{rname}_{arm}"] = {
                "latency_ms": (t1 - t0) * 1e3, "kernels_ms": st, "search_best": best, "seed_mjac": mj,
                "seed_step_revolute_rad": rev, "seed_step_prismatic_m": pri, "needs_research": research,
                "waypoint_lm_iters_per_s": p.T * iters / (st["lm"] * 1e-3),
                "pose_err_vs_targets": [rep["max_pos_err_m"], rep["max_rot_err_rad"]],
                "n_valid": rep["n_valid"], "first_valid": rep["first_valid"]}
    ctx.close()
    return out


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def _serve_stream(ctx, items, opts, iters, t_start):
    """Submit items [(arrival_s, problem)] at their arrival times (a
    submitter thread) and poll them in order; returns latencies (ms), the
    waypoint-iterations done, statuses and the wall time."""
    tickets = [None] * len(items)

    def submitter():
        for n, (at, p) in enumerate(items):
            d = t_start + at - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets[n] = ctx.submit(p.robot, p.targets, p.cand, opts)

    th = threading.Thread(target=submitter)
    th.start()
    lat, work, statuses = [], 0, set()
    for n, (at, p) in enumerate(items):
        while tickets[n] is None:
            time.sleep(0.0005)
        r = ctx.poll(tickets[n], p.T, timeout_ms=-1)
        lat.append((r["t_done_ns"] - r["t_submit_ns"]) * 1e-6)
        work += p.T * iters
        statuses.add(int(r["status"]))
    th.join()
    return lat, work, statuses, time.perf_counter() - t_start


def _one_at_a_time(ctx, items, opts, iters, budget_s):
    """The plain path: each request searched and refined alone, in arrival
    order, by the synchronous calls; stops after budget_s."""
    lat, work, served = [], 0, 0
    t0 = time.perf_counter()
    for at, p in items:
        now = time.perf_counter() - t0
        if now < at:
            time.sleep(at - now)
        if time.perf_counter() - t0 > budget_s:
            break
        plan = ctx.plan(p.robot, p.targets, p.cand, opts=opts)
        plan.dp_search()
        plan.lm_refine(iters, want_xi=True)
        plan.free()
        lat.append((time.perf_counter() - t0 - at) * 1e3)
        work += p.T * iters
        served += 1
    return lat, work, served, time.perf_counter() - t0


def run_serve(duration_s=10.0, rate_hz=200.0, pool=48, iters=30, slots=256, ipt=10,
              burst=240, fp64_budget_s=None):
    """Open loop: Poisson arrivals at rate_hz for duration_s, served by
    continuous batching (mixed precision) and, on the same schedule, one
    request at a time by the all-FP64 path.  Closed loop (saturation): a
    burst of `burst` requests submitted at once, both ways."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    arrivals = synth.config5_arrivals(rate_hz, duration_s)
    gen_ctx = cpf.Context(0)
    reqs = [_targets(gen_ctx, synth.config5_request(i), torch, dev) for i in range(pool)]
    gen_ctx.close()
    items = [(float(a), reqs[i % pool]) for i, a in enumerate(arrivals)]
    burst_items = [(0.0, reqs[i % pool]) for i in range(burst)]
    o_mix = cpf.make_opts(iters=iters, prec="mixed")
    o_64 = cpf.make_opts(iters=iters, prec="fp64")
    out = {"mode": "serve", "rate_hz": rate_hz, "duration_s": duration_s, "pool": pool,
           "lm_iters": iters, "slots": slots, "iters_per_tick": ipt, "burst": burst,
           "unit": "waypoint-LM-iters/s"}

    # --- mixed precision, continuous batching -----------------------------------
    ctx = cpf.Context(0, 64 << 30)
    ctx.config(slots=slots, iters_per_tick=ipt)
    w = ctx.submit(reqs[0].robot, reqs[0].targets, reqs[0].cand, o_mix)   # warm-up
    ctx.poll(w, reqs[0].T)
    lat, work, st, wall = _serve_stream(ctx, items, o_mix, iters, time.perf_counter())
    out["mixed_open"] = {"requests": len(items), "throughput": work / wall, "p50_ms": _pct(lat, 50),
                         "p99_ms": _pct(lat, 99), "max_ms": max(lat), "wall_s": wall,
                         "statuses": sorted(st)}
    lat, work, st, wall = _serve_stream(ctx, burst_items, o_mix, iters, time.perf_counter())
    out["mixed_closed"] = {"requests": burst, "throughput": work / wall, "p50_ms": _pct(lat, 50),
                           "p99_ms": _pct(lat, 99), "wall_s": wall, "statuses": sorted(st)}
    ctx.close()

    # --- all FP64, one request at a time ----------------------------------------
    ctx = cpf.Context(0, 64 << 30)
    budget = fp64_budget_s if fp64_budget_s is not None else duration_s * 3
    lat, work, served, wall = _one_at_a_time(ctx, items, o_64, iters, budget)
    out["fp64_one_at_a_time_open"] = {
        "requests_served": served, "requests_offered": len(items), "throughput": work / wall,
        "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "wall_s": wall,
        "note": "stops after the time budget; unserved requests are not counted"}
    lat, work, served, wall = _one_at_a_time(ctx, burst_items, o_64, iters, budget)
    out["fp64_one_at_a_time_closed"] = {"requests_served": served, "throughput": work / wall,
                                        "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "wall_s": wall}
    ctx.close()
    out["speedup_open"] = out["mixed_open"]["throughput"] / max(out["fp64_one_at_a_time_open"]["throughput"], 1e-9)
    out["speedup_closed"] = (out["mixed_closed"]["throughput"] /
                             max(out["fp64_one_at_a_time_closed"]["throughput"], 1e-9))
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["batch64", "T1000_K512", "batchopt", "schedule", "research", "collision",
                                     "prismatic", "serve"])
    ap.add_argument("--duration", type=float, default=10.0)
    a = ap.parse_args()
    if a.mode == "batch64":
        print(json.dumps(run_batch64()))
    elif a.mode == "T1000_K512":
        print(json.dumps(run_precision()))
    elif a.mode == "batchopt":
        print(json.dumps(run_batchopt()))
    elif a.mode == "schedule":
        print(json.dumps(run_schedule()))
    elif a.mode == "research":
        print(json.dumps(run_research()))
    elif a.mode == "collision":
        print(json.dumps(run_collision()))
    elif a.mode == "prismatic":
        print(json.dumps(run_prismatic()))
    else:
        print(json.dumps(run_serve(duration_s=a.duration)))
