"""GPU tests of the input forms of cpf_problem and of request validation,
through the C ABI.

Float32 candidates (host) and device-resident inputs (float32 candidates
and float64 targets read in place) give results bitwise equal to the
float64 host form when the values are float32-representable, in plans,
batches and served requests; a non-finite device-resident value (which the
host cannot check) ends the call or the request with CPF_E_ARG; a served
request asking for no LM iteration is refused.
"""
import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_09102_amd import cpf, synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = cpf.Context(0, 8 << 30)
    yield c
    c.close()


def _forms(p):
    """The problem's candidates and targets as float64 host arrays, float32
    host candidates, and device tensors."""
    c32 = np.ascontiguousarray(p.cand, dtype=np.float32)
    dev = torch.device("cuda:0")
    return [("f64", p.targets, p.cand),
            ("f32", p.targets, c32),
            ("device", torch.tensor(p.targets, dtype=torch.float64, device=dev),
             torch.tensor(c32, device=dev))]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_input_forms_give_the_same_plan(ctx, prec):
    p = H.small_problem(seed=51, T=90, K=40)
    out = {}
    for name, tg, cd in _forms(p):
        with ctx.plan(p.robot, tg, cd, opts=cpf.make_opts(prec=prec, iters=12)) as plan:
            path, best, xi, rep = plan.solve()
        out[name] = (path, best, xi, rep["cost"])
    ref = out["f64"]
    for name in ("f32", "device"):
        path, best, xi, cost = out[name]
        assert np.array_equal(path, ref[0]) and best == ref[1], name
        assert np.array_equal(xi, ref[2]) and cost == ref[3], name


def test_input_forms_in_batch_and_serving(ctx):
    probs = [H.small_problem(seed=60 + i, T=30 + 17 * i, K=10 + 6 * i) for i in range(3)]
    opts = cpf.make_opts(iters=9)
    base = ctx.solve_batch([(p.robot, p.targets, p.cand) for p in probs], opts)
    for form in (1, 2):
        items = [(p.robot,) + _forms(p)[form][1:] for p in probs]
        res = ctx.solve_batch(items, opts)
        tickets = [ctx.submit(*it, opts) for it in items]
        served = [ctx.poll(t, p.T, timeout_ms=60000) for t, p in zip(tickets, probs)]
        for b, r, s in zip(base, res, served):
            for x in (r, s):
                assert x is not None and x["status"] == 0
                assert np.array_equal(x["xi"], b["xi"]) and np.array_equal(x["path"], b["path"])


def test_nonfinite_device_input_is_an_argument_error(ctx):
    p = H.small_problem(seed=70, T=20, K=6)
    _, tg, cd = _forms(p)[2]
    bad_c = cd.clone()
    bad_c[2, 5, 3] = float("nan")
    with pytest.raises(cpf.CpfError) as ei:
        ctx.plan(p.robot, tg, bad_c)
    assert ei.value.status == cpf.E_ARG
    bad_t = tg.clone()
    bad_t[4, 1] = float("inf")
    with pytest.raises(cpf.CpfError) as ei:
        ctx.plan(p.robot, bad_t, cd)
    assert ei.value.status == cpf.E_ARG
    res = ctx.solve_batch([(p.robot, tg, bad_c), (p.robot, tg, cd)], cpf.make_opts(iters=3))
    assert res[0]["status"] == cpf.E_ARG and res[1]["status"] == 0
    t = ctx.submit(p.robot, tg, bad_c, cpf.make_opts(iters=3))
    r = ctx.poll(t, p.T, timeout_ms=60000)
    assert r is not None and r["status"] == cpf.E_ARG
    # the server goes on serving
    t = ctx.submit(p.robot, tg, cd, cpf.make_opts(iters=3))
    r = ctx.poll(t, p.T, timeout_ms=60000)
    assert r is not None and r["status"] == 0


def test_submit_refuses_zero_iterations(ctx):
    p = H.small_problem(seed=71, T=12, K=4)
    with pytest.raises(cpf.CpfError) as ei:
        ctx.submit(p.robot, p.targets, p.cand, cpf.make_opts(iters=0))
    assert ei.value.status == cpf.E_ARG


def test_needs_research_is_decided_by_the_library(ctx):
    """The re-search test runs in the library (cpf_dp_needs_research) and
    agrees with the seed's steps and the thresholds."""
    for seed, sigma in ((5, 0.25), (11, 0.02)):
        p = H.small_problem(seed=seed, T=60, K=8, sigma=sigma)
        with ctx.plan(p.robot, p.targets, p.cand) as plan:
            with pytest.raises(cpf.CpfError):
                plan.needs_research()
            plan.dp_search()
            rev, pri = plan.seed_steps()
            assert plan.needs_research() == (rev > cpf.RESEARCH_MJAC_RAD or pri > cpf.RESEARCH_MJAC_M)


def test_server_config_validation():
    """cpf_ctx_config rejects a negative tick budget and any change once the
    server runs; a budget of 0 (every request iters_per_tick per tick) serves
    the same results as the default budget (bitwise)."""
    probs = [H.small_problem(seed=72 + i, T=30 + 400 * i, K=8) for i in range(3)]
    opts = cpf.make_opts(iters=12)
    out = []
    for budget in (0, 6000, 700):
        with cpf.Context(0, 4 << 30) as c:
            with pytest.raises(cpf.CpfError) as ei:
                c.config(slots=8, iters_per_tick=5, tick_budget=-1)
            assert ei.value.status == cpf.E_ARG
            c.config(slots=8, iters_per_tick=5, tick_budget=budget)
            tickets = [c.submit(p.robot, p.targets, p.cand, opts) for p in probs]
            with pytest.raises(cpf.CpfError) as ei:
                c.config(slots=8, iters_per_tick=5, tick_budget=budget)
            assert ei.value.status == cpf.E_STATE
            res = [c.poll(t, p.T, timeout_ms=60000) for t, p in zip(tickets, probs)]
        assert all(r is not None and r["status"] == 0 and r["report"]["iters_done"] == 12 for r in res)
        out.append([r["xi"] for r in res])
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b)
