"""Shared test helpers: seeded problems with oracle-computed targets."""
import numpy as np

import oracle
from paper_2309_09102_amd import synth


def with_targets(prob):
    """Targets FK(q*) from the oracle (float32-rounded by the generator)."""
    return prob.with_targets(oracle.fk(prob.robot, prob.q_star))


def small_problem(seed=11, T=40, K=24, sigma=0.08, frac=0.25, robot_seed=0):
    return with_targets(synth.make_problem(synth.make_robot(robot_seed), seed=seed, T=T, K=K,
                                           sigma=sigma, branch_frac=frac))


def seed_of(prob, path):
    return prob.cand[path, np.arange(prob.T)]


COST_FLOOR = 1e-12   # m^2-scale cost below which the relative gap is taken against the floor


def parity_metrics(prob, xi_gpu, xi_ref, opts=None):
    """(max position diff m, max rotation diff rad, relative cost gap) under
    the oracle's FP64 FK and cost.  The cost gap is |C_gpu - C_ref| /
    max(C_ref, 1e-12): a path that reaches its targets exactly has cost ~1e-30,
    where a relative gap measures only rounding noise."""
    o = dict(oracle.DEFAULT_LM)
    if opts:
        o.update(opts)
    ep, er = oracle.pose_compare(prob.robot, xi_gpu, xi_ref)
    c_gpu = oracle.cost(prob.robot, xi_gpu, prob.targets, o["w_pose"], o["w_smooth"])
    c_ref = oracle.cost(prob.robot, xi_ref, prob.targets, o["w_pose"], o["w_smooth"])
    return ep, er, abs(c_gpu - c_ref) / max(c_ref, COST_FLOOR)
