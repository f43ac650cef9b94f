"""cpf_solve_static, the entry point for callers that cannot allocate device
memory, against the plan entry points it stands in for (cpf_plan_init +
cpf_plan_solve) on the same inputs: bitwise equal search path, B*,
trajectory and report on two calls in a row, the second with a smaller
problem (nothing carries over in the shared static scratch), in both
precisions and input forms; a problem beyond the scratch is refused with
CPF_E_NOMEM and leaves the next call unaffected."""
import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_09102_amd import cpf, synth  # noqa: E402

FIELDS = ("cost0", "cost", "lam", "n_accepted", "iters_done", "max_pos_err_m", "max_rot_err_rad", "mjac")


def _plan_solve(ctx, p, opts):
    with ctx.plan(p.robot, p.targets, p.cand, opts=opts) as plan:
        return plan.solve(want_xi=True)


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    assert np.array_equal(a[2], b[2])
    assert {k: a[3][k] for k in FIELDS} == {k: b[3][k] for k in FIELDS}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_static_solve_equals_plan_solve(prec):
    big = H.with_targets(synth.config2())
    small = H.small_problem(seed=81, T=45, K=20)
    opts = cpf.make_opts(prec=prec, iters=20)
    with cpf.Context(0) as ctx:
        got = [ctx.solve_static(p.robot, p.targets, p.cand, opts) for p in (big, small)]
        ref = [_plan_solve(ctx, p, opts) for p in (big, small)]
    for g, r in zip(got, ref):
        assert g[3]["iters_done"] == 20
        _same(g, r)


def test_static_solve_device_inputs_and_limit():
    p = H.small_problem(seed=82, T=120, K=48)
    dev = torch.device("cuda:0")
    tg = torch.tensor(p.targets, dtype=torch.float64, device=dev)
    cd = torch.tensor(p.cand.astype(np.float32), device=dev)
    opts = cpf.make_opts(iters=15)
    huge = synth.make_problem(synth.make_robot(0), seed=83, T=2000, K=512, sigma=0.1)
    with cpf.Context(0) as ctx:
        a = ctx.solve_static(p.robot, tg, cd, opts)
        with pytest.raises(cpf.CpfError) as ei:
            ctx.solve_static(huge.robot, np.zeros((2000, 12)), huge.cand, opts)
        assert ei.value.status == cpf.E_NOMEM and "static scratch" in str(ei.value)
        b = ctx.solve_static(p.robot, p.targets, p.cand, opts)
        ref = _plan_solve(ctx, p, opts)
    _same(a, ref)
    _same(b, ref)
