"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (stated for the refinement path): final trajectories agree with
the oracle's to <= 1e-5 m in position and <= 1e-5 rad in rotation (both
under the oracle's FP64 FK) and to <= 1e-6 relative cost; the search path
is index-identical (the search is exact FP64 on both sides, so ties resolve
identically).  FK: FP64 to 1e-12, FP32 to 2e-6 per component (a 7-link chain
of unit-scale float operations).
"""
import numpy as np
import pytest

import oracle
from paper_2309_09102_amd import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_09102_amd import cpf  # noqa: E402

POS_TOL, ROT_TOL, COST_TOL = 1e-5, 1e-5, 1e-6


@pytest.fixture(scope="module")
def ctx():
    c = cpf.Context(0, 8 << 30)
    yield c
    c.close()


def _fk_ref(robot, qT):
    pose, J = oracle.fk(robot, qT, jacobian=True)
    return pose, J


@pytest.mark.parametrize("M", [1, 255, 256, 1000, 4097])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_fk_batch_matches_oracle(ctx, M, dtype, tol):
    rb = synth.make_robot(3)
    q = synth.random_configs(M, M, rb)
    qd = torch.tensor(q.T.copy(), dtype=dtype, device="cuda")
    pose, jac = ctx.fk_batch(rb, qd, want_jac=True)
    torch.cuda.synchronize()
    pose = pose.double().cpu().numpy().T
    jac = jac.double().cpu().numpy().T.reshape(M, 6, 7)
    pr, Jr = _fk_ref(rb, q)
    np.testing.assert_allclose(pose, pr, atol=tol, rtol=0)
    np.testing.assert_allclose(jac, Jr, atol=tol, rtol=0)


def test_fk_batch_candidates_full_size(ctx):
    """K*T = 76,800 configurations of the T=300, K=256 workload."""
    p = synth.config2()
    q = p.cand.reshape(-1, 7)
    qd = torch.tensor(q.T.copy(), dtype=torch.float32, device="cuda")
    pose, _ = ctx.fk_batch(p.robot, qd)
    torch.cuda.synchronize()
    pose = pose.double().cpu().numpy().T
    idx = np.random.default_rng(0).choice(q.shape[0], 2000, replace=False)
    np.testing.assert_allclose(pose[idx], oracle.fk(p.robot, q[idx]), atol=2e-6, rtol=0)


def test_fk_batch_empty_and_errors(ctx):
    rb = synth.make_robot(0)
    q = torch.zeros((7, 0), dtype=torch.float32, device="cuda")
    pose, _ = ctx.fk_batch(rb, q)
    assert pose.shape == (12, 0)
    bad = synth.Robot(a=np.zeros(6), d=np.zeros(6), alpha=np.zeros(6), theta_off=np.zeros(6),
                      q_lo=-np.ones(6), q_hi=np.ones(6))
    with pytest.raises(cpf.CpfError) as ei:
        cpf.fk_batch(ctx.h, bad, 1, cpf.F32, 1, 1)
    assert ei.value.status == cpf.E_UNSUPPORTED


# ---- search --------------------------------------------------------------------

SEARCH_CASES = [
    dict(seed=1, T=1, K=5),
    dict(seed=2, T=7, K=1),
    dict(seed=3, T=2, K=3),
    dict(seed=4, T=33, K=65),       # ragged K
    dict(seed=5, T=50, K=16),
    dict(seed=6, T=120, K=300),     # K above 256: two lanes per part, ragged
    dict(seed=7, T=64, K=1024),     # maximum K
]


@pytest.mark.parametrize("case", SEARCH_CASES, ids=lambda c: f"T{c['T']}K{c['K']}")
def test_dp_search_index_identical(ctx, case):
    p = H.small_problem(seed=case["seed"], T=case["T"], K=case["K"])
    path_ref, best_ref, _, _ = oracle.dp(p.cand, p.robot)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        path, best, mj = plan.dp_search()
    assert np.array_equal(path, path_ref)
    assert best == best_ref
    assert mj == oracle.mjac(H.seed_of(p, path_ref))


def test_dp_search_with_node_penalty_and_ties(ctx):
    p = H.small_problem(seed=9, T=30, K=40, sigma=0.0)     # identical candidates: all ties
    extra = np.zeros((p.T, p.K))
    extra[:, :3] = 0.25
    extra[10, 5] = 100.0
    path_ref, best_ref, _, _ = oracle.dp(p.cand, p.robot, extra=extra)
    with ctx.plan(p.robot, p.targets, p.cand, node_pen=extra) as plan:
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref


def test_dp_search_list_fallback(ctx):
    """The 20 'hub' candidates equal the ground truth, so they are the nearest
    predecessors of every node, but carry a node cost of 50: each node's
    16-entry nearest list holds only hubs and cannot prove the minimum, which
    forces the exhaustive scan."""
    p = H.small_problem(seed=12, T=24, K=64, sigma=0.3, frac=0.0)
    cand = p.cand.copy()
    cand[:20] = p.q_star[None]
    extra = np.zeros((p.T, p.K))
    extra[:, :20] = 50.0
    path_ref, best_ref, _, _ = oracle.dp(cand, p.robot, extra=extra)
    with ctx.plan(p.robot, p.targets, cand, node_pen=extra) as plan:
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref
    assert best < 50.0 and not np.any(path < 20)


def test_dp_search_best_in_second_half_of_lists(ctx):
    """Eight candidates sit on the ground truth and cost 5 at even waypoints;
    eight more are offset by 0.05 rad on joint 0 and cost nothing.  A node
    of the first group at an odd waypoint then has the costly candidates as
    its 8 nearest predecessors and finds its best among entries 8-15 of its
    list, so the stage pass must evaluate the second half (checked here on
    the oracle's tables: more than a thousand nodes need it)."""
    p = H.small_problem(seed=13, T=200, K=64, sigma=0.3, frac=0.0)
    cand = p.cand.copy()
    cand[:8] = p.q_star[None]
    cand[8:16] = p.q_star[None]
    cand[8:16, :, 0] += 0.05
    cand = cand.astype(np.float32).astype(np.float64)
    extra = np.zeros((p.T, p.K))
    extra[0::2, :8] = 5.0
    path_ref, best_ref, B, _ = oracle.dp(cand, p.robot, extra=extra, want_tables=True)
    lo, hi = p.robot.q_lo, p.robot.q_hi
    m = oracle.oracle.LIMIT_MARGIN
    need = 0
    for t in range(1, p.T):
        e = np.max(np.abs(cand[:, t, None, :] - cand[None, :, t - 1, :]), axis=2)
        q = cand[:, t, :]
        pen = np.where(np.any((q <= lo + m) | (q >= hi - m), axis=1), oracle.oracle.LIMIT_PENALTY, 0.0) + extra[t]
        order = np.argsort(e, axis=1, kind="stable")[:, :16]
        c = np.take_along_axis(e, order, axis=1) + pen[:, None]
        v = np.maximum(B[t - 1][order], c)
        need += int(np.sum(v[:, :8].min(axis=1) > c[:, 8]))
    assert need > 1000
    with ctx.plan(p.robot, p.targets, cand, node_pen=extra) as plan:
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref


def test_dp_search_config2_full_size(ctx):
    p = H.with_targets(synth.config2())
    path_ref, best_ref, _, _ = oracle.dp(p.cand, p.robot)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref


# ---- LM ------------------------------------------------------------------------

def _lm_case(ctx, p, iters, prec, opts=None):
    o = dict(opts or {})
    copts = cpf.make_opts(prec=prec, **o)
    path_ref, _, _, _ = oracle.dp(p.cand, p.robot)
    ref = oracle.lm(p.robot, H.seed_of(p, path_ref), p.targets, iters, opts=o)
    with ctx.plan(p.robot, p.targets, p.cand, opts=copts) as plan:
        path, _, _ = plan.dp_search()
        xi, rep = plan.lm_refine(iters)
    assert np.array_equal(path, path_ref)
    return xi, rep, ref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lm_small_matches_oracle(ctx, prec):
    p = H.small_problem(seed=21, T=150, K=32)
    xi, rep, ref = _lm_case(ctx, p, 50, prec)
    ep, er, ec = H.parity_metrics(p, xi, ref["xi"])
    assert ep <= POS_TOL and er <= ROT_TOL and ec <= COST_TOL, (ep, er, ec)
    assert rep["iters_done"] == 50
    assert rep["cost"] <= rep["cost0"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lm_config2_full_size(ctx, prec):
    p = H.with_targets(synth.config2())
    xi, rep, ref = _lm_case(ctx, p, 50, prec)
    ep, er, ec = H.parity_metrics(p, xi, ref["xi"])
    print(f"config2 {prec}: pos {ep:.3e} m rot {er:.3e} rad cost {ec:.3e}")
    assert ep <= POS_TOL and er <= ROT_TOL and ec <= COST_TOL, (ep, er, ec)


@pytest.mark.parametrize("T", [1, 2, 3])
def test_lm_tiny_paths(ctx, T):
    p = H.small_problem(seed=30 + T, T=T, K=4)
    xi, rep, ref = _lm_case(ctx, p, 10, "fp64")
    ep, er, ec = H.parity_metrics(p, xi, ref["xi"])
    assert ep <= POS_TOL and er <= ROT_TOL and ec <= COST_TOL, (ep, er, ec)


def test_lm_without_smoothness_is_per_waypoint(ctx):
    p = H.small_problem(seed=40, T=20, K=8)
    xi, rep, ref = _lm_case(ctx, p, 15, "fp64", opts=dict(w_smooth=0.0))
    ep, er, _ = H.parity_metrics(p, xi, ref["xi"], opts=dict(w_smooth=0.0))
    assert ep <= POS_TOL and er <= ROT_TOL


def test_lm_resumable_bitwise(ctx):
    p = H.small_problem(seed=50, T=90, K=16)
    with ctx.plan(p.robot, p.targets, p.cand) as a, ctx.plan(p.robot, p.targets, p.cand) as b:
        a.dp_search()
        b.dp_search()
        xa, ra = a.lm_refine(30)
        b.lm_refine(12)
        xb, rb = b.lm_refine(18)
    assert np.array_equal(xa, xb) and ra["cost"] == rb["cost"] and rb["iters_done"] == 30


def test_plan_solve_equals_search_then_refine(ctx):
    p = H.small_problem(seed=53, T=120, K=40)
    opts = cpf.make_opts(iters=25)
    with ctx.plan(p.robot, p.targets, p.cand, opts=opts) as a, ctx.plan(p.robot, p.targets, p.cand, opts=opts) as b:
        pa, ba, xa, ra = a.solve()
        pb, bb, _ = b.dp_search()
        xb, rb = b.lm_refine(25)
        pa2, ba2, xa2, ra2 = a.solve()            # a second solve restarts from the search
    assert np.array_equal(pa, pb) and ba == bb
    assert np.array_equal(xa, xb) and ra["cost"] == rb["cost"] and ra["iters_done"] == 25
    assert np.array_equal(pa2, pa) and np.array_equal(xa2, xa) and ra2["iters_done"] == 25


def test_lm_before_search_is_state_error(ctx):
    p = H.small_problem(seed=51, T=10, K=4)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        with pytest.raises(cpf.CpfError) as ei:
            plan.lm_refine(1)
    assert ei.value.status == cpf.E_STATE


def test_bad_inputs_rejected(ctx):
    p = H.small_problem(seed=52, T=10, K=4)
    cand = p.cand.copy()
    cand[0, 0, 0] = np.nan
    with pytest.raises(cpf.CpfError) as ei:
        ctx.plan(p.robot, p.targets, cand)
    assert ei.value.status == cpf.E_ARG
    small = cpf.Context(0, 1024)
    try:
        with pytest.raises(cpf.CpfError) as ei:
            small.plan(p.robot, p.targets, p.cand)
        assert ei.value.status == cpf.E_NOMEM
    finally:
        small.close()


# ---- BatchOpt: the M smoothest candidates, optimised directly --------------------

@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batchopt_matches_oracle(ctx, prec):
    p = H.small_problem(seed=81, T=60, K=24)
    cand = p.cand.copy()
    cand[7] = cand[3]                    # a tie in mjac: the lower index first
    # 50 iterations: both arms converged, so the comparison is not of two
    # mid-descent iterates from a raw (noisy) candidate
    idx, res = ctx.batchopt(p.robot, p.targets, cand, 6, opts=cpf.make_opts(iters=50, prec=prec))
    idx_ref, ref = oracle.batchopt(p.robot, cand, p.targets, 6, 50)
    assert idx == idx_ref
    for r, rr in zip(res, ref):
        assert r["status"] == 0 and np.all(r["path"] == 0)
        ep, er, ec = H.parity_metrics(p, r["xi"], rr["xi"])
        assert ep <= POS_TOL and er <= ROT_TOL and ec <= COST_TOL, (ep, er, ec)


def test_batchopt_rejects_bad_m(ctx):
    p = H.small_problem(seed=82, T=10, K=4)
    for M in (0, 5):
        with pytest.raises(cpf.CpfError) as ei:
            ctx.batchopt(p.robot, p.targets, p.cand, M)
        assert ei.value.status == cpf.E_ARG


# ---- batching invariance -------------------------------------------------------

def test_solve_batch_equals_single(ctx):
    probs = [H.small_problem(seed=60 + i, T=40 + 17 * i, K=16 + 9 * i, robot_seed=i)
             for i in range(5)]
    opts = cpf.make_opts(iters=20)
    res = ctx.solve_batch([(p.robot, p.targets, p.cand) for p in probs], opts)
    for p, r in zip(probs, res):
        with ctx.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
            path, best, _ = plan.dp_search()
            xi, rep = plan.lm_refine(20)
        assert r["status"] == 0
        assert np.array_equal(r["path"], path) and r["search_best"] == best
        assert np.array_equal(r["xi"], xi) and r["report"]["cost"] == rep["cost"]


def test_solve_batch_more_plans_than_compute_units(ctx):
    """300 ragged plans in one launch (the chip has 256 compute units, so the
    last workgroups start only as the first finish): each result, sampled on
    both sides of the 256th plan, is the one it gets alone."""
    n = 300
    probs = [H.small_problem(seed=400 + i, T=12 + (i % 7) * 5, K=6 + (i % 5) * 3, robot_seed=i % 3)
             for i in range(n)]
    opts = cpf.make_opts(iters=8)
    res = ctx.solve_batch([(p.robot, p.targets, p.cand) for p in probs], opts)
    assert len(res) == n and all(r["status"] == 0 for r in res)
    for i in sorted(set(range(0, n, 37)) | {255, 256, 257, n - 1}):
        p, r = probs[i], res[i]
        with ctx.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
            path, best, _ = plan.dp_search()
            xi, rep = plan.lm_refine(8)
        assert np.array_equal(r["path"], path) and r["search_best"] == best, i
        assert np.array_equal(r["xi"], xi) and r["report"]["cost"] == rep["cost"], i


def test_serving_results_equal_alone(ctx):
    probs = [H.small_problem(seed=70 + i, T=30 + 11 * i, K=12 + 5 * i) for i in range(6)]
    opts = cpf.make_opts(iters=12)
    tickets = [ctx.submit(p.robot, p.targets, p.cand, opts) for p in probs]
    outs = [ctx.poll(t, p.T, timeout_ms=60000) for t, p in zip(tickets, probs)]
    for p, r in zip(probs, outs):
        assert r is not None and r["status"] == 0
        with ctx.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
            plan.dp_search()
            xi, rep = plan.lm_refine(12)
        assert np.array_equal(r["xi"], xi)
        assert r["t_done_ns"] >= r["t_search_done_ns"] >= r["t_admit_ns"] >= r["t_submit_ns"]
    with pytest.raises(cpf.CpfError) as ei:
        ctx.poll(tickets[0], probs[0].T, timeout_ms=0)
    assert ei.value.status == cpf.E_NOTFOUND


def test_serving_few_slots_admits_as_slots_free():
    """Continuous batching under slot pressure: a server with 3 slots and 2 LM
    iterations per tick takes 24 ragged requests; later requests are admitted
    only as earlier ones finish, and every result is the one it gets alone."""
    n, iters = 24, 9
    probs = [H.small_problem(seed=500 + i, T=10 + (i % 6) * 7, K=5 + (i % 4) * 4, robot_seed=i % 2)
             for i in range(n)]
    opts = cpf.make_opts(iters=iters)
    with cpf.Context(0, 1 << 30) as c:
        c.config(slots=3, iters_per_tick=2)
        tickets = [c.submit(p.robot, p.targets, p.cand, opts) for p in probs]
        outs = [c.poll(t, p.T, timeout_ms=60000) for t, p in zip(tickets, probs)]
        assert all(r is not None and r["status"] == 0 for r in outs)
        # admission waited for a slot: some request was admitted after another finished
        first_done = min(r["t_done_ns"] for r in outs)
        assert sum(r["t_admit_ns"] >= first_done for r in outs) >= n - 3
        for p, r in zip(probs, outs):
            with c.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
                plan.dp_search()
                xi, rep = plan.lm_refine(iters)
            assert np.array_equal(r["xi"], xi)
            assert r["report"]["cost"] == rep["cost"]


def test_serving_memory_budget_admits_as_arenas_return():
    """Continuous batching under memory pressure: with a budget of 2.5 plan
    arenas, 10 equal-size requests run at most two at a time (a third waits
    for an arena to come back), and every result is the one it gets alone."""
    n, iters = 10, 6
    probs = [H.small_problem(seed=600 + i, T=30, K=10, robot_seed=i % 2) for i in range(n)]
    opts = cpf.make_opts(iters=iters)
    with cpf.Context(0, 1 << 30) as probe:
        with probe.plan(probs[0].robot, probs[0].targets, probs[0].cand, opts=opts):
            arena = probe.bytes_in_use()
    assert arena > 0
    with cpf.Context(0, 2 * arena + arena // 2) as c:
        tickets = [c.submit(p.robot, p.targets, p.cand, opts) for p in probs]
        outs = [c.poll(t, p.T, timeout_ms=60000) for t, p in zip(tickets, probs)]
        assert all(r is not None and r["status"] == 0 for r in outs)
        first_done = min(r["t_done_ns"] for r in outs)
        assert sum(r["t_admit_ns"] >= first_done for r in outs) >= n - 2
        assert c.bytes_in_use() <= 2 * arena
        for p, r in zip(probs, outs):
            with c.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
                plan.dp_search()
                xi, rep = plan.lm_refine(iters)
            assert np.array_equal(r["xi"], xi)
            assert r["report"]["cost"] == rep["cost"]
