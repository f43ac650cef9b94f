"""Each plausible mistake planted in a copy of the oracle must fail a pin.

The copies are compiled on the CPU into a temporary directory; the real
oracle library is restored afterwards.  This checks that the pins in
test_oracle_pins.py constrain every part of the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong tie-break).
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import oracle as _w
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(_w.__file__), "cpf_oracle.c")

MUTANTS = {
    "fk_sign": ("A[1] = -st * ca;", "A[1] = st * ca;"),
    "fk_param": ("A[11] = d;", "A[11] = a;"),
    "fk_translation_dropped": ("if (c == 3) s += A[r * 4 + 3];", "if (c == 3) s += 0.0;"),
    "fk_chain_stops_at_seven": ("    for (int i = 0; i < n; ++i) {\n        z[i][0] = M[2];",
                                "    for (int i = 0; i < n && i < 7; ++i) {\n        z[i][0] = M[2];"),
    "jac_cross_sign": ("J[0 * n + i] = z[i][1] * dz - z[i][2] * dy;",
                       "J[0 * n + i] = z[i][2] * dy - z[i][1] * dz;"),
    "log_vee_sign": ("double v0 = 0.5 * (R[7] - R[5]);", "double v0 = 0.5 * (R[5] - R[7]);"),
    "residual_sign": ("r[0] = pose[0] - target[0];", "r[0] = target[0] - pose[0];"),
    "cost_weight": ("return 0.5 * w_p * pose_sum + 0.5 * w_s * diff_sum + 0.5 * w_c * coll_sum;",
                    "return 0.5 * w_p * pose_sum + w_s * diff_sum + 0.5 * w_c * coll_sum;"),
    "grad_term_dropped": ("if (t > 0) sm += q[j] - xi[(size_t)(t - 1) * n + j];",
                          "if (t > 0) sm += 0.0;"),
    "jtj_index": ("s += J6[k * n + i] * J6[k * n + j];", "s += J6[k * n + i] * J6[k * n + i];"),
    "dp_tiebreak": ("if (v < bv || (v == bv && e < be))", "if (v < bv || (v == bv && e > be))"),
    "dp_penalty_dropped": ("double v = e + pen;", "double v = e;"),
    "dp_end_tie": ("if (Bp[k] < Bp[kend]) kend = k;", "if (Bp[k] <= Bp[kend]) kend = k;"),
    "btd_forward_sign": ("for (int i = 0; i < n; ++i) rhs[i] += w * tmp[i];\n            }\n            lsolve",
                         "for (int i = 0; i < n; ++i) rhs[i] -= w * tmp[i];\n            }\n            lsolve"),
    "btd_schur_power": ("Lt[e] -= w * w * inv[e];", "Lt[e] -= w * inv[e];"),
    "lm_diag_dropped": ("Dbuf[nn * t + (size_t)i * n + i] += w_s * ct + lambda;",
                        "Dbuf[nn * t + (size_t)i * n + i] += lambda;"),
    "lm_always_accept": ("int acc = Cn < C;", "int acc = 1;"),
    "lm_damping_floor": ("if (f < 1.0 / 3.0) f = 1.0 / 3.0;\n            lambda *= f;",
                         "if (f < 0.5) f = 0.5;\n            lambda *= f;"),
    "lm_damping_square": ("double f = 1.0 - u * u * u;\n            if (f < 1.0 / 3.0) f = 1.0 / 3.0;\n            lambda *= f;",
                          "double f = 1.0 - u * u;\n            if (f < 1.0 / 3.0) f = 1.0 / 3.0;\n            lambda *= f;"),
    "lm_nu_not_doubled": ("lambda *= nu;\n            nu *= 2.0;", "lambda *= nu;\n            nu *= 1.0;"),
    "lm_no_clamp": ("if (v > hi[j]) v = hi[j];\n                trial[e] = v;",
                    "trial[e] = v;"),
    "sched_modes_swapped": ("const int m = pose_ok ? 1 : 0;", "const int m = pose_ok ? 0 : 1;"),
    "sched_step_check_dropped": ("steps_ok = 0;", "steps_ok = 1;"),
    "sched_diff_damping_adapts": ("const double l = m ? o.lambda0 : lam;", "const double l = lam;"),
    "sched_reject_keeps_damping": ("lam *= nu;\n                nu *= 2.0;\n            }\n            if (lam < o.lambda_min)",
                                   "nu *= 2.0;\n            }\n            if (lam < o.lambda_min)"),
    "coll_radius_dropped": ("double d = sqrt(d2) - c->caps[7 * i + 6] - c->caps[7 * j + 6];",
                            "double d = sqrt(d2) - c->caps[7 * i + 6];"),
    "coll_grad_sign": ("point_grad(rb->jtype, z, o, bj, pb, u, -1.0, grad);",
                       "point_grad(rb->jtype, z, o, bj, pb, u, 1.0, grad);"),
    "seg_seg_edge_sign": ("double s = side, t = e > 0.0 ? (b * s + f) / e : 0.0;",
                          "double s = side, t = e > 0.0 ? (b * s - f) / e : 0.0;"),
    "seg_box_upper_gap": ("if (x > hi) return (x - hi) * (x - hi);", "if (x > hi) return (x - lo) * (x - lo);"),
    "coll_adjacent_checked": ("for (int j = i + 3; j < n; ++j) {", "for (int j = i + 2; j < n; ++j) {"),
    "coll_penalty_dropped": ("return (dmin[0] < 0.0 || dmin[1] < 0.0) ? rb->coll->penalty : 0.0;", "return 0.0;"),
    "coll_residual_sign": ("J[h * rb->n + k] = r > 0.0 ? -g[h * rb->n + k] : 0.0;",
                           "J[h * rb->n + k] = r > 0.0 ? g[h * rb->n + k] : 0.0;"),
    "box_frame_transposed": ("A[r] = R[0 * 3 + r] * (P0[i][0] - B[0]) + R[1 * 3 + r] * (P0[i][1] - B[1]) +",
                             "A[r] = R[r * 3 + 0] * (P0[i][0] - B[0]) + R[r * 3 + 1] * (P0[i][1] - B[1]) +"),
    "sched_collision_ignored": ("if (dmin[0] < 0.0 || dmin[1] < 0.0) coll_ok = 0;", "if (0) coll_ok = 0;"),
    "sched_length_signed": ("len += fabs(xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j]);",
                            "len += xi[(size_t)(t + 1) * n + j] - xi[(size_t)t * n + j];"),
    "prism_moves_as_revolute": ("if (prismatic(jtype, i)) { *th = off; *di = d[i] + qi; }",
                                "if (0) { *th = off; *di = d[i] + qi; }"),
    "prism_jac_angular_kept": ("J[3 * n + i] = 0.0;", "J[3 * n + i] = z[i][0];"),
    "prism_jac_linear_index": ("J[0 * n + i] = z[i][0];", "J[0 * n + i] = z[i][1];"),
    "prism_margin_revolute": ("double m = prismatic(jtype, j) ? margin_m : margin;", "double m = margin;"),
    "prism_step_threshold_revolute": ("tol[prismatic(jtype, j) ? 3 : 2]", "tol[2]"),
    "prism_point_grad_revolute": ("if (prismatic(jtype, k)) {", "if (0) {"),
}


def battery():
    """Fast calls of the pin tests; each raises if its pin is violated."""
    return [
        lambda: P.test_p1_fk_zero_configuration(0),
        lambda: P.test_p2_fk_single_axis(0, 1.0),
        lambda: P.test_p5_jacobian_finite_differences(0),
        lambda: P.test_p5_jacobian_planar_closed_form(),
        lambda: P.test_p6_gradient_matches_cost_fd(0.1),
        lambda: P.test_p6_cost_definition_small_case(),
        lambda: P.test_p7_log_branches_match_library(0.5),
        lambda: P.test_p8_dp_matches_brute_force(),
        lambda: P.test_p9_single_waypoint_is_argmin_penalty(),
        lambda: P.test_p9_exact_tie_breaks_on_edge_then_index(),
        lambda: P.test_p9_penalised_node_avoided_when_possible(),
        lambda: P.test_p10_block_solve_matches_dense(7, 0.1),
        lambda: P.test_p11_smoothness_only_step_dct_closed_form(9, 1e-3),
        lambda: P.test_p12_dls_push_through_identity(1e-2),
        lambda: P.test_p13_lm_cost_monotone_and_rejects_keep_xi(0),
        lambda: P.test_p13_lm_clamps_to_limits(),
        lambda: P.test_p13_lm_damping_follows_the_gain_ratio_rule(0, 30, 0.1, 25),
        lambda: P.test_p13_lm_damping_follows_the_gain_ratio_rule(8, 20, 1.5, 20),
        lambda: P.test_p15_schedule_pose_step_is_lm_without_smoothness(),
        lambda: P.test_p15_schedule_valid_seed_takes_a_differencing_step(),
        lambda: P.test_p15_schedule_latest_valid_meets_the_thresholds(),
        lambda: P.test_p15_schedule_rejects_a_discontinuous_pose_valid_trajectory(),
        lambda: P.test_p15_schedule_steps_are_single_objective_lm_steps(),
        lambda: P.test_p16_seg_seg_closed_forms(),
        lambda: P.test_p16_seg_seg_matches_bounded_minimiser(0),
        lambda: P.test_p16_seg_box_closed_forms(),
        lambda: P.test_p16_seg_box_matches_dense_sampling(0),
        lambda: P.test_p16_distances_match_independent_evaluation(0),
        lambda: P.test_p16_distance_gradients_match_central_differences(0),
        lambda: P.test_p16_adjacent_links_never_checked(),
        lambda: P.test_p16_search_penalises_colliding_nodes_brute_force(),
        lambda: P.test_p16_lm_gradient_with_collision_matches_cost_differences(),
        lambda: P.test_p16_schedule_rejects_a_colliding_pose_valid_trajectory(),
        lambda: P.test_p17_prismatic_joint_translates_along_its_axis(2, 0.3),
        lambda: P.test_p17_jacobian_with_prismatic_joint_finite_differences(1),
        lambda: P.test_p17_lm_gradient_with_prismatic_joint_matches_cost_differences(),
        lambda: P.test_p17_limit_margin_is_three_cm_for_a_prismatic_joint(),
        lambda: P.test_p17_schedule_step_threshold_is_two_cm_for_a_prismatic_joint(),
        lambda: P.test_p17_collision_gradient_with_prismatic_joint(0),
        lambda: P.test_p18_fk_zero_configuration_eight_joints(0),
        lambda: P.test_p18_torso_lift_is_a_translation_along_the_base_axis(0),
        lambda: P.test_p18_jacobian_torso_arm_finite_differences(0),
        lambda: P.test_p18_lm_gradient_eight_joints_matches_cost_differences(),
    ]


def test_unmutated_battery_passes():
    for check in battery():
        check()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    lib = _w.build_copy(src.replace(old, new, 1), str(tmp_path / f"lib_{name}.so"))
    prev = _w.use_library(lib)
    caught = []
    try:
        for i, check in enumerate(battery()):
            try:
                check()
            except Exception as exc:   # AssertionError, LinAlgError, hypothesis errors
                caught.append((i, type(exc).__name__))
    finally:
        _w.restore_library(prev)
    assert caught, f"mutant {name} passed every pin"
