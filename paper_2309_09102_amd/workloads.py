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
  serve      the serving stream (requests of T ~ U{50..2000}, K in {128,
             256, 512}, sigma ~ U[0.02, 0.15], offset fraction ~ U[0, 0.3],
             30 LM iterations, Poisson arrivals at 200/s), every request
             distinct and its inputs resident on the device before the
             stream starts: continuous batching in mixed precision open
             loop on the arrival schedule, then closed loop (all requests
             at once: saturation), the all-FP64 arm continuously batched
             closed loop, and the all-FP64 path one request at a time on
             the arrival schedule.  bench.py reports this as its headline.

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


def run_single(ctx=None, iters=50, reps=10, xi_out=None):
    """The single T=300, K=256 request, mixed and all-FP64: each step is
    batched FK over the K x T candidates plus cpf_plan_solve (the full
    search with its lists, back-tracking, `iters` LM iterations and the
    report in one stream) on inputs already resident in the plan."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    LM_OPS = 1900
    dev = torch.device("cuda:0")
    own = ctx is None
    if own:
        ctx = cpf.Context(0)
    prob = _targets(ctx, synth.config2(), torch, dev)
    T, K = prob.T, prob.K
    cand_soa = torch.tensor(prob.cand.reshape(-1, 7).T.copy(), dtype=torch.float32, device=dev)
    out = {"mode": "T300_K256", "workload": f"single request T={T} K={K}, {iters} LM iterations", "arms": {}}
    for prec in ("mixed", "fp64"):
        plan = ctx.plan(prob.robot, prob.targets, prob.cand, opts=cpf.make_opts(prec=prec, iters=iters))

        def step():
            ctx.fk_batch(prob.robot, cand_soa)
            return plan.solve(want_xi=False)

        for _ in range(3):
            step()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, _, rep = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = {k: ctx.kernel_stats(k) for k in ("fk", "dp_lists", "dp", "lm", "eval")}
        ctx.profile(False)
        if xi_out is not None:
            xi_out[prec] = plan.solve(want_xi=True)[2]
        plan.free()
        lm_ms = st["lm"][0] / max(st["lm"][1], 1)
        out["arms"][prec] = {"ms_per_step": dt * 1e3, "waypoint_lm_iters_per_s": T * iters / dt,
                             "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in st.items()},
                             "lm_frac": T * iters * LM_OPS / (lm_ms * 1e-3) / 1e12 / 78.6,
                             "cost": rep["cost"],
                             "pose_err_vs_targets": [rep["max_pos_err_m"], rep["max_rot_err_rad"]]}
    if own:
        ctx.close()
    return out


def run_lm_phases(iters=10):
    """One plan each at T = 300 (K = 256), 1000 and 2000 (K = 128), mixed
    arm: a warm-up iteration, then `iters` LM iterations timed.  With the
    diagnostic build of the library (built with -D CPF_PHASE_CYCLES and
    loaded through CPF_LIB) the LM kernel also prints its per-phase and
    per-round shader-clock totals for each launch."""
    import sys
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    out = {"mode": "lm_phases", "iters": iters, "plans": []}
    for T, K in ((300, 256), (1000, 128), (2000, 128)):
        p = _targets(ctx, synth.make_problem(synth.make_robot(0), seed=2, T=T, K=K, sigma=0.1, branch_frac=0.25),
                     torch, dev)
        with ctx.plan(p.robot, p.targets, p.cand, opts=cpf.make_opts(prec="mixed")) as plan:
            plan.dp_search()
            plan.lm_refine(1)
            torch.cuda.synchronize()
            print(f"=== T={T} K={K}: {iters} iterations", flush=True)
            ctx.profile(True)
            plan.lm_refine(iters, want_xi=False)
            ms = ctx.kernel_stats("lm")[0]
            ctx.profile(False)
            sys.stdout.flush()
        out["plans"].append({"T": T, "K": K, "lm_ms_per_iteration": ms / iters})
    ctx.close()
    return out


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
    st = {k: ctx.kernel_stats(k) for k in ("dp_lists", "dp", "lm", "eval")}
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
        st = {k: ctx.kernel_stats(k) for k in ("dp_lists", "dp", "lm")}
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
            dev_a = ctx.kernel_stats("dp")[0] + ctx.kernel_stats("dp_lists")[0]
            ctx.profile(False)
        ctx.profile(True)
        t2 = time.perf_counter()
        with ctx.plan(p.robot, p.targets, allc) as plan:
            _, best_f, _ = plan.dp_search()
        t3 = time.perf_counter()
        dev_f = ctx.kernel_stats("dp")[0] + ctx.kernel_stats("dp_lists")[0]
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
            st = {k: ctx.kernel_stats(k)[0] for k in ("dp_lists", "dp", "lm")}
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
    step threshold, beside the all-revolute robot on the same request and
    the 8-joint chain of the same seed (a torso lift ahead of a 7-joint arm,
    the Fetch.Full stand-in)."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    dev = torch.device("cuda:0")
    ctx = cpf.Context(0)
    out = {"mode": "prismatic", "T": 300, "K": 256, "lm_iters": iters, "arms": {}}
    robots = (("prismatic", synth.make_robot_prismatic(robot_seed)), ("revolute", synth.make_robot(robot_seed)),
              ("torso_arm_8", synth.make_robot_torso_arm(robot_seed)))
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
                st = {k: ctx.kernel_stats(k)[0] for k in ("dp_lists", "dp", "lm")}
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
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


class StreamRequest:
    """One request of the serving stream with its inputs on the device:
    float32 candidates [K][T][7] and float64 targets [T][12] (FK of the
    ground-truth path by the library's FP64 kernel, rounded to float32)."""

    def __init__(self, i, T, K, cand, targets):
        self.i, self.T, self.K, self.cand, self.targets = i, T, K, cand, targets


def stream_requests(ctx, indices, threads=8):
    """Requests synth.config5_request(i) for i in indices, generated on
    `threads` host threads and uploaded as they are made."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2309_09102_amd import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)

    def make(i):
        p = synth.config5_request(i)
        with torch.cuda.stream(stream):
            cand = torch.from_numpy(p.cand).to(dev)
            q = torch.from_numpy(np.ascontiguousarray(p.q_star.T)).to(dev)
            pose, _ = ctx.fk_batch(p.robot, q, stream=stream.cuda_stream)
            tg = pose.t().float().double().contiguous()       # float32 values, [T][12]
        stream.synchronize()
        return StreamRequest(i, p.T, p.K, cand, tg)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(make, indices))


def serve_stream(ctx, reqs, arrivals, opts, keep_xi=()):
    """Submit reqs at their arrival times (s from now; None: all at once)
    from a submitter thread and collect every result.  Returns per-request
    latency (submit -> done, ms), status, wall time (first submit to last
    completion) and the trajectories of the requests whose index is in
    keep_xi."""
    from paper_2309_09102_amd import synth
    robot = synth.make_robot(0)
    n = len(reqs)
    tickets = [None] * n
    t_start = time.perf_counter()
    err = []

    def submitter():
        try:
            for k, r in enumerate(reqs):
                if arrivals is not None:
                    d = t_start + arrivals[k] - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                tickets[k] = ctx.submit(robot, r.targets, r.cand, opts)
        except Exception as e:   # surfaced below
            err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    lat, status, xis, t_sub, t_done = [], [], {}, [], []
    keep = set(keep_xi)
    for k, r in enumerate(reqs):
        while tickets[k] is None and not err:
            time.sleep(0.0002)
        if err:
            break
        res = ctx.poll(tickets[k], r.T, timeout_ms=-1)
        lat.append((res["t_done_ns"] - res["t_submit_ns"]) * 1e-6)
        t_sub.append(res["t_submit_ns"])
        t_done.append(res["t_done_ns"])
        status.append(int(res["status"]))
        if r.i in keep:
            xis[r.i] = res["xi"]
    th.join()
    if err:
        raise err[0]
    wall = (max(t_done) - min(t_sub)) * 1e-9 if t_done else 0.0
    return {"latency_ms": lat, "status": status, "wall_s": wall, "xi": xis}


def one_at_a_time(ctx, reqs, arrivals, opts, budget_s, keep_xi=()):
    """The plain path: each request searched and refined alone by the
    synchronous calls (plan from the device-resident inputs, cpf_plan_solve),
    in arrival order, starting no request after budget_s.  Latency is arrival
    -> done; the requests left unserved are reported as censored at the
    budget (their latency is at least budget_s minus their arrival)."""
    from paper_2309_09102_amd import synth
    robot = synth.make_robot(0)
    lat, xis, served_work = [], {}, 0
    keep = set(keep_xi)
    t0 = time.perf_counter()
    served = 0
    for k, r in enumerate(reqs):
        at = 0.0 if arrivals is None else arrivals[k]
        now = time.perf_counter() - t0
        if now < at:
            time.sleep(at - now)
        if time.perf_counter() - t0 > budget_s:
            break
        with ctx.plan(robot, r.targets, r.cand, opts=opts) as plan:
            _, _, xi, _ = plan.solve(want_xi=True)
        lat.append((time.perf_counter() - t0 - at) * 1e3)
        served_work += r.T * opts.iters
        served += 1
        if r.i in keep:
            xis[r.i] = xi
    wall = time.perf_counter() - t0
    censored = [max(0.0, (wall - (0.0 if arrivals is None else arrivals[k])) * 1e3) for k in range(served, len(reqs))]
    return {"latency_ms": lat, "censored_ms": censored, "served": served, "work": served_work,
            "wall_s": wall, "xi": xis}


def _summary(res, reqs, iters):
    lat = res["latency_ms"]
    work = sum(r.T for r in reqs[:len(lat)]) * iters
    return {"requests": len(lat), "throughput": work / res["wall_s"] if res["wall_s"] > 0 else None,
            "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "max_ms": max(lat) if lat else None,
            "wall_s": res["wall_s"], "statuses": sorted(set(res["status"]))}


def run_serve(duration_s=10.0, warmup_s=2.0, rate_hz=200.0, iters=30, slots=256, ipt=30, tick_budget=6000,
              fp64_budget_s=None, keep_xi=(), open_loop_only=False, host_requests=256):
    """The serving comparison on distinct device-resident requests: the
    arrival schedule's first warmup_s seconds are served untimed, the next
    duration_s seconds are the timed stream.  Returns the summary and the raw
    per-arm results (trajectories of the requests in keep_xi)."""
    import torch
    from paper_2309_09102_amd import cpf, synth
    arrivals = synth.config5_arrivals(rate_hz, warmup_s + duration_s)
    n_warm = int(np.searchsorted(arrivals, warmup_s))
    n = len(arrivals)
    gen_ctx = cpf.Context(0)
    t0 = time.perf_counter()
    reqs = stream_requests(gen_ctx, range(n))
    t_gen = time.perf_counter() - t0
    gen_ctx.close()
    warm, timed = reqs[:n_warm], reqs[n_warm:]
    at = arrivals[n_warm:] - arrivals[n_warm]
    raw = {"targets": {}}
    if keep_xi == "sample":   # every 20th timed request and the 20 longest
        keep_xi = {r.i for r in timed[::20]} | {r.i for r in sorted(timed, key=lambda r: -r.T)[:20]}
    keep_xi = set(keep_xi or ())
    for r in timed:
        if r.i in keep_xi:
            raw["targets"][r.i] = r.targets.cpu().numpy()
    work = sum(r.T for r in timed) * iters
    o_mix = cpf.make_opts(iters=iters, prec="mixed")
    o_64 = cpf.make_opts(iters=iters, prec="fp64")
    out = {"mode": "serve", "rate_hz": rate_hz, "duration_s": duration_s, "warmup_s": warmup_s,
           "requests": len(timed), "warmup_requests": len(warm), "lm_iters": iters, "slots": slots,
           "iters_per_tick": ipt, "tick_budget": tick_budget, "unit": "waypoint-LM-iters/s",
           "waypoint_lm_iters": work,
           "offered_load": work / duration_s, "input_prep_s": t_gen,
           "warmup_waypoint_lm_iters": sum(r.T for r in warm) * iters,
           "search_pairs": sum((r.T - 1) * r.K * r.K for r in timed),
           "warmup_search_pairs": sum((r.T - 1) * r.K * r.K for r in warm),
           "input_bytes_resident": int(sum(r.cand.numel() * 4 + r.targets.numel() * 8 for r in reqs))}

    def kstats(ctx):
        return {k: ctx.kernel_stats(k) for k in ("dp_lists", "dp", "lm")}

    # --- mixed precision, continuous batching -------------------------------
    ctx = cpf.Context(0, 64 << 30)
    ctx.config(slots=slots, iters_per_tick=ipt, tick_budget=tick_budget)
    if warm:
        serve_stream(ctx, warm, None, o_mix)                     # warm-up: graphs, arena pool
    ctx.profile(True)
    res = serve_stream(ctx, timed, at, o_mix, keep_xi)
    ks = kstats(ctx)
    ctx.profile(False)
    out["mixed_open"] = _summary(res, timed, iters)
    out["mixed_open"]["kernels"] = {k: {"ms": v[0], "launches": v[1]} for k, v in ks.items()}
    raw["mixed_open"] = res
    raw["timed"] = [(r.i, r.T, r.K) for r in timed]
    if open_loop_only:
        ctx.close()
        return out, raw
    ctx.profile(True)
    res = serve_stream(ctx, timed, None, o_mix)
    ks = kstats(ctx)
    ctx.profile(False)
    out["mixed_closed"] = _summary(res, timed, iters)
    out["mixed_closed"]["kernels"] = {k: {"ms": v[0], "launches": v[1]} for k, v in ks.items()}

    # --- the same server fed host arrays (float32 candidates, copied by
    # cpf_submit and sent over PCIe at admission): the first requests of the
    # timed stream, all at once
    n_host = min(len(timed), host_requests)
    if n_host:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=8) as ex:
            hp = list(ex.map(lambda r: synth.config5_request(r.i), timed[:n_host]))
        host_reqs = [StreamRequest(r.i, r.T, r.K, p.cand, r.targets.cpu().numpy())
                     for r, p in zip(timed[:n_host], hp)]
        res = serve_stream(ctx, host_reqs, None, o_mix)
        out["mixed_closed_host_inputs"] = _summary(res, host_reqs, iters)
        del hp, host_reqs
    ctx.close()

    # --- all FP64, continuous batching (the precision comparison at equal batching)
    ctx = cpf.Context(0, 64 << 30)
    ctx.config(slots=slots, iters_per_tick=ipt, tick_budget=tick_budget)
    if warm:
        serve_stream(ctx, warm[:64], None, o_64)
    ctx.profile(True)
    res = serve_stream(ctx, timed, None, o_64)
    ks = kstats(ctx)
    ctx.profile(False)
    out["fp64_closed"] = _summary(res, timed, iters)
    out["fp64_closed"]["kernels"] = {k: {"ms": v[0], "launches": v[1]} for k, v in ks.items()}
    ctx.close()

    # --- all FP64, one request at a time on the same arrival schedule --------
    ctx = cpf.Context(0, 64 << 30)
    for r in warm[:2]:
        with ctx.plan(synth.make_robot(0), r.targets, r.cand, opts=o_64) as plan:
            plan.solve(want_xi=False)
    budget = fp64_budget_s if fp64_budget_s is not None else duration_s
    res = one_at_a_time(ctx, timed, at, o_64, budget, keep_xi)
    ctx.close()
    lat_all = res["latency_ms"] + res["censored_ms"]
    out["fp64_one_at_a_time_open"] = {
        "requests_served": res["served"], "requests_offered": len(timed),
        "throughput": res["work"] / res["wall_s"], "wall_s": res["wall_s"],
        "p50_ms_served": _pct(res["latency_ms"], 50), "p99_ms_served": _pct(res["latency_ms"], 99),
        "p50_ms_lower_bound": _pct(lat_all, 50), "p99_ms_lower_bound": _pct(lat_all, 99),
        "note": (f"no request starts after {budget:.0f} s; the unserved ones count in the lower "
                 "bounds with their waiting time at that moment")}
    raw["fp64_one_at_a_time_open"] = res
    out["speedup_open"] = out["mixed_open"]["throughput"] / out["fp64_one_at_a_time_open"]["throughput"]
    out["speedup_closed_vs_one_at_a_time"] = (out["mixed_closed"]["throughput"] /
                                              out["fp64_one_at_a_time_open"]["throughput"])
    out["speedup_mixed_vs_fp64_batched"] = out["mixed_closed"]["throughput"] / out["fp64_closed"]["throughput"]
    del reqs, warm, timed
    torch.cuda.empty_cache()
    return out, raw


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["batch64", "T1000_K512", "batchopt", "schedule", "research", "collision",
                                     "prismatic", "serve", "lm_phases"])
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
    elif a.mode == "lm_phases":
        print(json.dumps(run_lm_phases()))
    else:
        print(json.dumps(run_serve(duration_s=a.duration)[0]))
