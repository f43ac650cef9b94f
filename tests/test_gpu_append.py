"""GPU parity of the re-search with appended candidates (Sec. III-B: more
candidate plans, then the search again) against the oracle's search over the
concatenated candidates: index-identical path and bit-identical B*, as for
every search.  The appended plan must also behave exactly like a plan created
with all candidates at once (search and the LM after it, bitwise).
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


@pytest.fixture(scope="module")
def ctx():
    c = cpf.Context(0, 8 << 30)
    yield c
    c.close()


def _node_pen(rng, T, K):
    pen = np.zeros((T, K))
    mask = rng.random((T, K)) < 0.1
    pen[mask] = np.round(rng.uniform(0.0, 0.3, mask.sum()), 3)
    return pen


@pytest.mark.parametrize("T,K0,Kadd", [(40, 24, 24), (33, 65, 40), (7, 5, 3), (1, 4, 4), (2, 3, 30),
                                       (120, 300, 200)])
def test_append_then_search_matches_oracle(ctx, T, K0, Kadd):
    p = H.small_problem(seed=100 + T, T=T, K=K0)
    extra = synth.more_candidates(p, Kadd)
    allc = np.concatenate([p.cand, extra])
    path_ref, best_ref, _, _ = oracle.dp(allc, p.robot)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        plan.dp_search()
        plan.append(extra)
        path, best, mj = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref
    assert mj == oracle.mjac(allc[path, np.arange(T)])


@pytest.mark.parametrize("old_pen,new_pen", [(True, True), (False, True), (True, False)])
def test_append_with_node_costs(ctx, old_pen, new_pen):
    T, K0, Kadd = 30, 20, 12
    p = H.small_problem(seed=131, T=T, K=K0)
    rng = np.random.default_rng(7)
    pen0 = _node_pen(rng, T, K0) if old_pen else None
    pen1 = _node_pen(rng, T, Kadd) if new_pen else None
    extra = synth.more_candidates(p, Kadd)
    full = np.concatenate([pen0 if old_pen else np.zeros((T, K0)),
                           pen1 if new_pen else np.zeros((T, Kadd))], axis=1)
    path_ref, best_ref, _, _ = oracle.dp(np.concatenate([p.cand, extra]), p.robot, extra=full)
    with ctx.plan(p.robot, p.targets, p.cand, node_pen=pen0) as plan:
        plan.append(extra, pen1)            # before any search: the search builds every list
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref
    with ctx.plan(p.robot, p.targets, p.cand, node_pen=pen0) as plan:
        plan.dp_search()
        plan.append(extra, pen1)            # after a search: lists merged
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref


def test_append_twice_equals_fresh_plan_with_lm(ctx):
    p = H.small_problem(seed=141, T=90, K=40)
    e1 = synth.more_candidates(p, 30, batch=1)
    e2 = synth.more_candidates(p, 50, batch=2)
    allc = np.concatenate([p.cand, e1, e2])
    with ctx.plan(p.robot, p.targets, p.cand) as a, ctx.plan(p.robot, p.targets, allc) as b:
        a.dp_search()
        a.lm_refine(3)
        a.append(e1)
        with pytest.raises(cpf.CpfError) as ei:
            a.lm_refine(1)                  # must search again first
        assert ei.value.status == cpf.E_STATE
        a.append(e2)
        pa, ba, _ = a.dp_search()
        xa, ra = a.lm_refine(12)
        pb, bb, _ = b.dp_search()
        xb, rb = b.lm_refine(12)
    assert np.array_equal(pa, pb) and ba == bb
    assert np.array_equal(xa, xb) and ra["cost"] == rb["cost"] and ra["iters_done"] == 12


def test_append_config2_full_size(ctx):
    """T=300, K=256 plus 256 more: equal to the oracle's search over 512."""
    p = H.with_targets(synth.config2())
    extra = synth.more_candidates(p, 256)
    path_ref, best_ref, _, _ = oracle.dp(np.concatenate([p.cand, extra]), p.robot)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        plan.dp_search()
        plan.append(extra)
        path, best, _ = plan.dp_search()
    assert np.array_equal(path, path_ref) and best == best_ref


def test_research_loop_lowers_mjac(ctx):
    """The paper's loop: while the seed's mjac exceeds 12 degrees, ask for
    more candidates and search again (here: 32 at a time, at most 6 times)."""
    p = H.with_targets(synth.make_problem(synth.make_robot(0), seed=5, T=150, K=16, sigma=0.25))
    history = []
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        _, _, mj = plan.dp_search()
        history.append(mj)
        allc = p.cand
        b = 0
        while mj > cpf.RESEARCH_MJAC_RAD and b < 6:
            b += 1
            extra = synth.more_candidates(p, 32, batch=b)
            allc = np.concatenate([allc, extra])
            plan.append(extra)
            path, best, mj = plan.dp_search()
            history.append(mj)
    assert history[0] > cpf.RESEARCH_MJAC_RAD and len(history) >= 2
    assert all(b <= a for a, b in zip(history, history[1:]))   # more candidates never hurt
    path_ref, best_ref, _, _ = oracle.dp(allc, p.robot)
    assert np.array_equal(path, path_ref) and best == best_ref


def test_append_errors(ctx):
    p = H.small_problem(seed=151, T=10, K=1000)
    with ctx.plan(p.robot, p.targets, p.cand) as plan:
        with pytest.raises(cpf.CpfError) as ei:
            plan.append(synth.more_candidates(p, 25))
        assert ei.value.status == cpf.E_UNSUPPORTED
        bad = synth.more_candidates(p, 2)
        bad[1, 3, 2] = np.inf
        with pytest.raises(cpf.CpfError) as ei:
            plan.append(bad)
        assert ei.value.status == cpf.E_ARG
        with pytest.raises(ValueError):
            plan.append(np.zeros((2, 9, 7)))
        path, best, _ = plan.dp_search()    # the plan is unchanged
    path_ref, best_ref, _, _ = oracle.dp(p.cand, p.robot)
    assert np.array_equal(path, path_ref) and best == best_ref
