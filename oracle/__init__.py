"""FP64 CPU oracle for the CppFlow refinement path (arXiv 2309.09102).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP path and imports nothing from it.

The arithmetic lives in ``cpf_oracle.c`` (plain C, IEEE double,
``-ffp-contract=off``); this module builds it with gcc and wraps it with
ctypes.  Robots are duck-typed objects with float64 arrays ``a, d, alpha,
theta_off, q_lo, q_hi`` and optionally ``joint_type`` (0 revolute, 1
prismatic).

Parity status per function (what pins it, in tests/test_oracle_pins.py):
  fk / jacobian   closed forms at q = 0, single-axis and planar chains;
                  orthonormality; central finite differences
  log_so3         Exp(Log R) = R, known angles, branch continuity
  cost / gradient central finite differences of the cost
  dp              brute-force enumeration on tiny K, T; special cases
  btd_solve       dense numpy solve; DCT closed form of the smoothness system
  lm_step         push-through identity for T = 1; block-diagonal w_s = 0 case
  lm              monotone cost, rejected steps keep xi, fixed point, pose
                  convergence with w_s -> 0.  The exact iterate path (the
                  sequence of accept / reject decisions) is parity unpinned:
                  the paper prints no worked example of it.
  batchopt        selection pinned against numpy's own mjac ordering; each
                  result is plan() on one candidate (pinned above)
  lm_schedule     single steps equal lm() with the other weight zero; the
                  latest valid trajectory meets the thresholds under FK; its
                  length vs numpy; the first check on a valid seed passes
  seg_seg,        the two distance QPs vs closed forms (parallel, crossing,
  seg_box         skew, touching) and vs scipy's bounded minimiser
  coll_eval       capsule endpoints vs FK of the truncated chains, distances vs
                  scipy, gradients vs central differences; adjacent links
                  never checked; the search penalty vs brute force
  prismatic       FK translation along the closed-form axis; pure translation
  joints          anywhere; Jacobian, LM gradient and collision gradients vs
                  central differences; 3 cm limit margin and 2 cm validity
                  step by constructed cases; seed steps split by joint type
"""
from .oracle import (build, lib_path, fk, log_so3, cost, dp, mjac, seed_steps, joint_types, btd_solve,
                     lm_step, lm, lm_schedule, plan, batchopt, pose_compare,
                     seg_seg, seg_box, coll_eval, coll_spec,
                     DEFAULT_LM, VALID_TOL, COLL_MARGIN, COLL_WEIGHT, COLL_PENALTY)

__all__ = ["build", "lib_path", "fk", "log_so3", "cost", "dp", "mjac", "seed_steps", "joint_types",
           "btd_solve", "lm_step", "lm", "lm_schedule", "plan", "batchopt", "pose_compare",
           "seg_seg", "seg_box", "coll_eval", "coll_spec",
           "DEFAULT_LM", "VALID_TOL", "COLL_MARGIN", "COLL_WEIGHT", "COLL_PENALTY"]
