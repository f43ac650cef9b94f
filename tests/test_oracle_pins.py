"""Pins of the FP64 oracle against what the mathematics fixes.

None of these re-type the oracle's own formulas: each check uses a closed
form, a library routine (scipy rotations, numpy dense solve), finite
differences, brute-force enumeration or an algebraic identity.  The paper
prints no worked numerical example, so there are no paper-printed values to
pin against (only its constants, checked in test_paper_constants).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.spatial.transform import Rotation

import oracle
from paper_2309_09102_amd import synth

HALF_PI = math.pi / 2


def robot_of(a, d, alpha, lo=-2.8, hi=2.8):
    n = len(a)
    return synth.Robot(a=np.asarray(a, float), d=np.asarray(d, float),
                       alpha=np.asarray(alpha, float), theta_off=np.zeros(n),
                       q_lo=np.full(n, lo), q_hi=np.full(n, hi))


def exact_robot(seed=0, n=7):
    """Random chain with alpha exactly +-pi/2 (so sin/cos are exactly 0/+-1)."""
    rng = np.random.default_rng(seed)
    return robot_of(rng.uniform(0, 0.1, n), rng.uniform(0, 0.4, n),
                    np.where(rng.integers(0, 2, n) == 0, -HALF_PI, HALF_PI))


def split(pose):
    return pose[..., :3], pose[..., 3:].reshape(pose.shape[:-1] + (3, 3))


# ---- P1: FK at q = 0 --------------------------------------------------------

def zero_pose_closed_form(rb):
    """All Rz are identity: the chain is a sequence of x-rotations and
    translations (a_i, 0, d_i) expressed in the frame rotated by the running
    sum of twists."""
    A = np.concatenate([[0.0], np.cumsum(rb.alpha)])
    p = np.zeros(3)
    for i in range(rb.dof):
        p += np.array([rb.a[i], -rb.d[i] * math.sin(A[i]), rb.d[i] * math.cos(A[i])])
    R = Rotation.from_rotvec([A[-1], 0, 0]).as_matrix()
    return p, R, A


@pytest.mark.parametrize("seed", range(5))
def test_p1_fk_zero_configuration(seed):
    rb = exact_robot(seed)
    p, R = split(oracle.fk(rb, np.zeros(7)))
    p_ref, R_ref, _ = zero_pose_closed_form(rb)
    np.testing.assert_allclose(p, p_ref, atol=1e-15)
    np.testing.assert_allclose(R, R_ref, atol=1e-15)


# ---- P2: FK at single-axis configurations -----------------------------------

@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("theta", [1.0, -1.0, HALF_PI, -HALF_PI, 2.5])
def test_p2_fk_single_axis(seed, theta):
    rb = exact_robot(seed)
    p0, R0, A = zero_pose_closed_form(rb)
    for i in range(7):
        axis = np.array([0.0, -math.sin(A[i]), math.cos(A[i])])
        origin = np.zeros(3)
        for k in range(i):
            origin += np.array([rb.a[k], -rb.d[k] * math.sin(A[k]), rb.d[k] * math.cos(A[k])])
        Rot = Rotation.from_rotvec(theta * axis).as_matrix()
        q = np.zeros(7)
        q[i] = theta
        p, R = split(oracle.fk(rb, q))
        np.testing.assert_allclose(p, origin + Rot @ (p0 - origin), atol=1e-14)
        np.testing.assert_allclose(R, Rot @ R0, atol=1e-14)


# ---- P3: planar chain (all twists zero) -------------------------------------

@given(st.lists(st.floats(-3, 3), min_size=7, max_size=7), st.integers(0, 2**31 - 1))
@settings(max_examples=50, deadline=None)
def test_p3_fk_planar(q, seed):
    rng = np.random.default_rng(seed)
    rb = robot_of(rng.uniform(0, 0.5, 7), rng.uniform(-0.3, 0.3, 7), np.zeros(7))
    q = np.asarray(q)
    Th = np.cumsum(q)
    p_ref = np.array([np.sum(rb.a * np.cos(Th)), np.sum(rb.a * np.sin(Th)), np.sum(rb.d)])
    R_ref = Rotation.from_rotvec([0, 0, Th[-1]]).as_matrix()
    p, R = split(oracle.fk(rb, q))
    np.testing.assert_allclose(p, p_ref, atol=1e-14)
    np.testing.assert_allclose(R, R_ref, atol=1e-14)


# ---- P4: rotation invariants ------------------------------------------------

@given(st.integers(0, 2**31 - 1))
@settings(max_examples=50, deadline=None)
def test_p4_fk_rotation_is_orthonormal(seed):
    rb = synth.make_robot(seed)
    q = np.random.default_rng(seed).uniform(-math.pi, math.pi, (8, 7))
    _, R = split(oracle.fk(rb, q))
    for Rm in R:
        np.testing.assert_allclose(Rm.T @ Rm, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(Rm) - 1.0) < 1e-14


# ---- P5: Jacobian vs central finite differences -----------------------------

@pytest.mark.parametrize("seed", range(6))
def test_p5_jacobian_finite_differences(seed):
    rb = synth.make_robot(seed)
    q = np.random.default_rng(100 + seed).uniform(-2.5, 2.5, 7)
    _, J = oracle.fk(rb, q, jacobian=True)
    h = 1e-6
    for i in range(7):
        e = np.zeros(7)
        e[i] = h
        pp, Rp = split(oracle.fk(rb, q + e))
        pm, Rm = split(oracle.fk(rb, q - e))
        np.testing.assert_allclose(J[:3, i], (pp - pm) / (2 * h), atol=1e-8)
        w = Rotation.from_matrix(Rp @ Rm.T).as_rotvec() / (2 * h)
        np.testing.assert_allclose(J[3:, i], w, atol=1e-8)


def test_p5_jacobian_planar_closed_form():
    rb = robot_of([0.3, 0.2, 0.1, 0.25, 0.05, 0.15, 0.1], np.zeros(7), np.zeros(7))
    q = np.linspace(-1, 1, 7)
    _, J = oracle.fk(rb, q, jacobian=True)
    Th = np.cumsum(q)
    for i in range(7):
        jx = -np.sum(rb.a[i:] * np.sin(Th[i:]))
        jy = np.sum(rb.a[i:] * np.cos(Th[i:]))
        np.testing.assert_allclose(J[:, i], [jx, jy, 0, 0, 0, 1], atol=1e-15)


# ---- P6: cost gradient vs finite differences --------------------------------

@pytest.mark.parametrize("w_s", [0.0, 0.1, 2.0])
def test_p6_gradient_matches_cost_fd(w_s):
    rb = synth.make_robot(7)
    prob = synth.make_problem(rb, seed=7, T=5, K=1, sigma=0.0)
    targets = oracle.fk(rb, prob.q_star)
    xi = prob.q_star + np.random.default_rng(1).normal(0, 0.2, prob.q_star.shape)
    _, g = oracle.lm_step(rb, xi, targets, 1.0, w_s, 1.0)
    h = 1e-6
    fd = np.zeros_like(xi)
    for t in range(xi.shape[0]):
        for j in range(7):
            e = np.zeros_like(xi)
            e[t, j] = h
            fd[t, j] = (oracle.cost(rb, xi + e, targets, 1.0, w_s)
                        - oracle.cost(rb, xi - e, targets, 1.0, w_s)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_p6_cost_definition_small_case():
    """Cost of a 2-waypoint path whose poses hit the targets exactly is the
    smoothness term alone: w_s/2 |q1 - q0|^2."""
    rb = synth.make_robot(3)
    xi = np.array([np.linspace(-1, 1, 7), np.linspace(-0.9, 1.2, 7)])
    tg = oracle.fk(rb, xi)
    dq = xi[1] - xi[0]
    assert oracle.cost(rb, xi, tg, 1.0, 0.3) == pytest.approx(0.15 * dq @ dq, rel=1e-13)
    # and a pure position offset adds w_p/2 |offset|^2
    tg2 = tg.copy()
    tg2[0, :3] += [0.01, -0.02, 0.005]
    assert oracle.cost(rb, xi, tg2, 2.0, 0.0) == pytest.approx(0.01**2 + 0.02**2 + 0.005**2,
                                                              rel=1e-12)


# ---- P7: log map ------------------------------------------------------------

@given(st.lists(st.floats(-1, 1), min_size=3, max_size=3),
       st.floats(0.0, math.pi - 1e-9))
@settings(max_examples=200, deadline=None)
def test_p7_log_inverts_exp(axis, angle):
    u = np.asarray(axis)
    if np.linalg.norm(u) < 1e-3:
        return
    u = u / np.linalg.norm(u)
    R = Rotation.from_rotvec(angle * u).as_matrix()
    phi = oracle.log_so3(R)
    assert np.linalg.norm(phi) == pytest.approx(angle, abs=1e-9)
    np.testing.assert_allclose(Rotation.from_rotvec(phi).as_matrix(), R, atol=1e-9)


@pytest.mark.parametrize("angle", [0.0, 1e-12, 1e-6, 9.99e-5, 1.0001e-4, 0.5, 3.0,
                                   math.pi - 2e-6, math.pi - 5e-7, math.pi])
def test_p7_log_branches_match_library(angle):
    u = np.array([0.3, -0.5, 0.81])
    u /= np.linalg.norm(u)
    R = Rotation.from_rotvec(angle * u).as_matrix()
    phi = oracle.log_so3(R)
    ref = Rotation.from_matrix(R).as_rotvec()
    if angle >= math.pi - 1e-6:   # +-pi*u are the same rotation
        assert np.linalg.norm(phi) == pytest.approx(angle, abs=1e-8)
        assert min(np.linalg.norm(phi - ref), np.linalg.norm(phi + ref)) < 1e-7
    else:
        np.testing.assert_allclose(phi, ref, atol=1e-12 + 1e-10 * angle)


# ---- P8 / P9: search vs brute force and special cases -----------------------

def brute_force_tables(cand, rb, margin=oracle.oracle.LIMIT_MARGIN, penalty=10.0, extra=None):
    """B_t(k) = min over all prefixes ending at (t, k) of the path's maximum
    of (pen_0, e_s + pen_s), by enumeration."""
    K, T, n = cand.shape
    pen = np.zeros((T, K))
    for t in range(T):
        for k in range(K):
            q = cand[k, t]
            near = np.any((q <= rb.q_lo + margin) | (q >= rb.q_hi - margin))
            pen[t, k] = (penalty if near else 0.0) + (0.0 if extra is None else extra[t, k])

    def value(path):
        v = pen[0, path[0]]
        for s in range(1, len(path)):
            e = np.max(np.abs(cand[path[s], s] - cand[path[s - 1], s - 1]))
            v = max(v, e + pen[s, path[s]])
        return v

    B = np.full((T, K), np.inf)
    for t in range(T):
        for prefix in itertools.product(range(K), repeat=t + 1):
            B[t, prefix[-1]] = min(B[t, prefix[-1]], value(prefix))
    return B, value


@given(st.integers(1, 4), st.integers(1, 6), st.integers(0, 2**31 - 1),
       st.booleans())
@settings(max_examples=80, deadline=None)
def test_p8_dp_matches_brute_force(K, T, seed, coarse):
    rng = np.random.default_rng(seed)
    rb = synth.make_robot(1)
    if coarse:   # values on a coarse grid: many exact ties
        cand = rng.integers(-10, 11, (K, T, 7)) * 0.25
    else:
        cand = rng.uniform(-2.8, 2.8, (K, T, 7))
    cand = np.clip(cand, rb.q_lo, rb.q_hi)
    path, best, B_all, bp_all = oracle.dp(cand, rb, want_tables=True)
    B_ref, value = brute_force_tables(cand, rb)
    assert np.array_equal(B_all, B_ref)           # bitwise
    assert best == B_ref[-1].min()
    assert value(tuple(path)) == best
    # each back-pointer is the smallest predecessor under (value, e, k')
    for t in range(1, T):
        for k in range(K):
            keys = []
            for kp in range(K):
                e = np.max(np.abs(cand[k, t] - cand[kp, t - 1]))
                near = np.any((cand[k, t] <= rb.q_lo + oracle.oracle.LIMIT_MARGIN)
                              | (cand[k, t] >= rb.q_hi - oracle.oracle.LIMIT_MARGIN))
                v = max(B_ref[t - 1, kp], e + (10.0 if near else 0.0))
                keys.append((v, e, kp))
            assert bp_all[t, k] == min(keys)[2]


def test_p9_single_candidate_gives_zero_path():
    rb = synth.make_robot(0)
    cand = np.random.default_rng(0).uniform(-1, 1, (1, 9, 7))
    path, best, _, _ = oracle.dp(cand, rb)
    assert np.all(path == 0)
    assert best == oracle.mjac(cand[0])


def test_p9_single_waypoint_is_argmin_penalty():
    rb = synth.make_robot(0)
    cand = np.zeros((5, 1, 7))
    cand[0, 0, 2] = 2.79          # near the upper limit
    cand[1, 0, 0] = -2.78         # near the lower limit
    extra = np.array([[0.0, 0.0, 3.0, 0.5, 0.5]])
    path, best, _, _ = oracle.dp(cand, rb, extra=extra)
    assert path[0] == 3 and best == 0.5


def test_p9_exact_tie_breaks_on_edge_then_index():
    rb = synth.make_robot(0)
    K, T = 4, 3
    cand = np.zeros((K, T, 7))
    # waypoint 1: every node is reached with change 0.5 on joint 1, so all
    # B_1 tie at 0.5; nodes 0 and 3 are identical
    cand[:, 1, 0] = [0.30, 0.35, 0.0, 0.30]
    cand[:, 1, 1] = [0.5, 0.5, -0.5, 0.5]
    # waypoint 2
    cand[:, 2, 0] = [0.33, 0.30, 0.0, 0.0]
    cand[:, 2, 1] = [0.5, 0.5, -0.5, -0.5]
    path, best, B_all, bp = oracle.dp(cand, rb, want_tables=True)
    assert best == 0.5 and np.all(B_all[1:] == 0.5)
    assert list(bp[1]) == [0, 0, 0, 0]      # full ties -> smallest index
    assert bp[2, 0] == 1    # value tie 0.5; edge 0.02 (from 1) beats 0.03 (from 0, 3)
    assert bp[2, 1] == 0    # value and edge tie between 0 and 3 -> smaller index
    assert bp[2, 2] == 2 and bp[2, 3] == 2
    assert list(path) == [0, 1, 0]


def test_p9_penalised_node_avoided_when_possible():
    rb = synth.make_robot(0)
    K, T = 2, 4
    cand = np.zeros((K, T, 7))
    cand[1] = 0.01                   # the smooth path...
    cand[1, 2, 3] = 2.79             # ...except one node near a limit
    cand[0, :, 0] = [0.0, 0.3, 0.6, 0.9]   # rougher but penalty free
    path, best, _, _ = oracle.dp(cand, rb)
    assert path[2] != 1
    assert best < 10.0


# ---- P10 / P11: block-tridiagonal solve -------------------------------------

def dense_from_blocks(D, w):
    T, n, _ = D.shape
    H = np.zeros((T * n, T * n))
    for t in range(T):
        H[t * n:(t + 1) * n, t * n:(t + 1) * n] = D[t]
        if t + 1 < T:
            H[t * n:(t + 1) * n, (t + 1) * n:(t + 2) * n] = -w * np.eye(n)
            H[(t + 1) * n:(t + 2) * n, t * n:(t + 1) * n] = -w * np.eye(n)
    return H


@pytest.mark.parametrize("T", [1, 2, 3, 7, 20])
@pytest.mark.parametrize("w", [0.0, 0.1, 1.0])
def test_p10_block_solve_matches_dense(T, w):
    rng = np.random.default_rng(T * 10 + int(w * 10))
    n = 7
    D = np.empty((T, n, n))
    for t in range(T):
        Jt = rng.normal(size=(6, n))
        D[t] = Jt.T @ Jt + (2 * w + 0.05) * np.eye(n)
    b = rng.normal(size=(T, n))
    x = oracle.btd_solve(D, w, b)
    x_ref = np.linalg.solve(dense_from_blocks(D, w), b.reshape(-1)).reshape(T, n)
    np.testing.assert_allclose(x, x_ref, rtol=1e-12, atol=1e-12 * np.abs(x_ref).max())


def test_p10_block_solve_rejects_indefinite():
    D = np.stack([np.eye(7), -np.eye(7)])
    with pytest.raises(np.linalg.LinAlgError):
        oracle.btd_solve(D, 0.1, np.ones((2, 7)))


@pytest.mark.parametrize("T", [1, 2, 9, 40])
@pytest.mark.parametrize("lam", [1e-3, 1.0])
def test_p11_smoothness_only_step_dct_closed_form(T, lam):
    """With w_p = 0 the system is (w_s L + lam I) delta = -w_s L xi per joint,
    diagonal in the DCT-II basis with eigenvalues 4 sin^2(pi k / 2T)."""
    w_s = 0.7
    rb = synth.make_robot(0)
    xi = np.random.default_rng(T).uniform(-1, 1, (T, 7))
    targets = np.tile([0.0, 0.0, 0.0, 1, 0, 0, 0, 1, 0, 0, 0, 1], (T, 1))
    delta, _ = oracle.lm_step(rb, xi, targets, 0.0, w_s, lam)
    t = np.arange(T)
    ref = np.zeros_like(xi)
    for k in range(T):
        v = np.cos(math.pi * k * (t + 0.5) / T)
        mu = 4 * math.sin(math.pi * k / (2 * T)) ** 2
        proj = (v @ xi) / (v @ v)
        ref -= (w_s * mu / (w_s * mu + lam)) * np.outer(v, proj)
    np.testing.assert_allclose(delta, ref, atol=1e-12)


# ---- P12: damped least squares, T = 1 and block-diagonal w_s = 0 -------------

def residual_by_library(rb, q, target):
    pose = oracle.fk(rb, q)
    p, R = split(pose)
    pt, Rt = target[:3], target[3:].reshape(3, 3)
    return np.concatenate([p - pt, Rotation.from_matrix(R @ Rt.T).as_rotvec()])


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0])
def test_p12_dls_push_through_identity(lam):
    rb = synth.make_robot(5)
    q = np.random.default_rng(3).uniform(-2, 2, 7)
    target = oracle.fk(rb, q + 0.05)
    _, J = oracle.fk(rb, q, jacobian=True)
    r = residual_by_library(rb, q, target)
    ref = -J.T @ np.linalg.solve(J @ J.T + lam * np.eye(6), r)
    delta, _ = oracle.lm_step(rb, q[None], target[None], 1.0, 0.3, lam)
    np.testing.assert_allclose(delta[0], ref, rtol=1e-9, atol=1e-12)


def test_p12_block_diagonal_when_smoothness_off():
    rb = synth.make_robot(5)
    rng = np.random.default_rng(4)
    xi = rng.uniform(-2, 2, (6, 7))
    targets = oracle.fk(rb, xi + rng.normal(0, 0.05, xi.shape))
    delta, _ = oracle.lm_step(rb, xi, targets, 1.0, 0.0, 1e-2)
    for t in range(6):
        d1, _ = oracle.lm_step(rb, xi[t:t + 1], targets[t:t + 1], 1.0, 0.0, 1e-2)
        np.testing.assert_allclose(delta[t], d1[0], rtol=1e-12, atol=1e-15)


# ---- P13: LM invariants -----------------------------------------------------

@pytest.mark.parametrize("cfg_seed", [0, 1, 2])
def test_p13_lm_cost_monotone_and_rejects_keep_xi(cfg_seed):
    rb = synth.make_robot(cfg_seed)
    prob = synth.make_problem(rb, seed=cfg_seed, T=30, K=1, sigma=0.1)
    targets = oracle.fk(rb, prob.q_star)
    out = oracle.lm(rb, prob.cand[0], targets, 25)
    assert out["rc"] == 0
    c = np.concatenate([[out["cost0"]], out["cost_hist"]])
    assert np.all(np.diff(c) <= 0)
    assert c[-1] < 0.5 * c[0]
    # a rejected iteration leaves xi unchanged
    for k in range(1, 25):
        if not out["accepted"][k]:
            a = oracle.lm(rb, prob.cand[0], targets, k)["xi"]
            b = oracle.lm(rb, prob.cand[0], targets, k + 1)["xi"]
            assert np.array_equal(a, b)
            break


def _nielsen_replay(rb, x0, tg, iters, lam0=1e-3, w_p=1.0, w_s=0.1):
    """LM written out from its definition, one damped step at a time (the
    step itself from the oracle's single-step routine, the rest here): a
    trial clip(x + delta) is accepted iff it lowers the cost; Nielsen's gain
    ratio rule then scales the damping by max(1/3, 1 - (2 rho - 1)^3) and
    resets nu to 2, where rho is the cost drop over the predicted drop
    delta^T (lam delta - g) / 2; a rejected trial multiplies the damping by
    nu and doubles nu; the damping stays in [1e-10, 1e10].  Returns the
    damping each iteration used, the accept flags and the final iterate."""
    x = np.clip(np.asarray(x0, dtype=float), rb.q_lo, rb.q_hi)
    lam, nu = lam0, 2.0
    lams, accs = [], []
    for _ in range(iters):
        d, g = oracle.lm_step(rb, x, tg, w_p, w_s, lam)
        trial = np.clip(x + d, rb.q_lo, rb.q_hi)
        c, cn = oracle.cost(rb, x, tg, w_p, w_s), oracle.cost(rb, trial, tg, w_p, w_s)
        lams.append(lam)
        accs.append(cn < c)
        if cn < c:
            rho = (c - cn) / (0.5 * float(np.sum(d * (lam * d - g))))
            lam *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            x = trial
        else:
            lam *= nu
            nu *= 2.0
        lam = min(max(lam, 1e-10), 1e10)
    return np.array(lams), np.array(accs), x


@pytest.mark.parametrize("seed,T,sigma,iters", [(0, 30, 0.1, 25), (8, 20, 1.5, 20)])
def test_p13_lm_damping_follows_the_gain_ratio_rule(seed, T, sigma, iters):
    """The damping history, accept flags and result of a whole LM run equal a
    step-by-step replay of the Levenberg-Marquardt loop with Nielsen's rule
    (the reading taken where the paper gives no damping schedule).  The
    smooth case reaches the 1/3 floor (a gain ratio near 1) and takes the
    cubic factor between the floor and 1; the rough case (1.5 rad noise)
    raises the damping after a poor accepted step (rho < 1/2) and rejects
    three trials in a row, so nu doubles twice."""
    rb = synth.make_robot(seed)
    prob = synth.make_problem(rb, seed=seed, T=T, K=1, sigma=sigma)
    tg = oracle.fk(rb, prob.q_star)
    out = oracle.lm(rb, prob.cand[0], tg, iters)
    lams, accs, x = _nielsen_replay(rb, prob.cand[0], tg, iters)
    np.testing.assert_array_equal(out["accepted"], accs)
    np.testing.assert_allclose(out["lambda_hist"], lams, rtol=1e-13, atol=0)
    np.testing.assert_allclose(out["xi"], x, rtol=0, atol=1e-12)
    run = longest = 0
    for a in accs:
        run = 0 if a else run + 1
        longest = max(longest, run)
    ratios = lams[1:] / lams[:-1]
    acc_ratios = ratios[accs[:-1]]
    if sigma < 1.0:
        assert np.any(np.isclose(acc_ratios, 1.0 / 3.0))
        assert np.any((acc_ratios > 0.34) & (acc_ratios < 0.99))
    else:
        assert longest >= 3 and np.any(acc_ratios > 1.01)


def test_p13_fixed_point_gives_zero_step():
    rb = synth.make_robot(2)
    q = np.random.default_rng(0).uniform(-1, 1, 7)
    xi = np.tile(q, (5, 1))
    targets = oracle.fk(rb, xi)
    delta, g = oracle.lm_step(rb, xi, targets, 1.0, 0.1, 1e-3)
    assert np.abs(g).max() < 1e-15 and np.abs(delta).max() < 1e-12


def test_p13_pose_converges_without_smoothness():
    rb = synth.make_robot(1)
    prob = synth.make_problem(rb, seed=1, T=12, K=1, sigma=0.02)
    targets = oracle.fk(rb, prob.q_star)
    out = oracle.lm(rb, prob.cand[0], targets, 30,
                    opts=dict(w_smooth=0.0, lambda0=1e-3))
    ep, er = oracle.pose_compare(rb, out["xi"], targets=targets)
    assert ep < 1e-12 and er < 1e-12


def test_p13_lm_clamps_to_limits():
    rb = synth.make_robot(1)
    prob = synth.make_problem(rb, seed=1, T=10, K=1, sigma=0.0)
    targets = oracle.fk(rb, prob.q_star)
    xi0 = prob.q_star.copy()
    xi0[:, 0] = 3.5                      # outside the limits
    out = oracle.lm(rb, xi0, targets, 5)
    assert np.all(out["xi"] <= rb.q_hi) and np.all(out["xi"] >= rb.q_lo)


# ---- constants the paper states ---------------------------------------------

def test_paper_constants():
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
    with open(path) as f:
        c = json.load(f)
    assert oracle.oracle.LIMIT_PENALTY == c["limit_penalty"]["value"]
    assert oracle.oracle.LIMIT_MARGIN == pytest.approx(math.radians(c["limit_margin_deg"]["value"]))
    # the penalty exceeds any possible joint change of a revolute joint (pi)
    assert c["limit_penalty"]["value"] > math.pi


# ---- BatchOpt: the M smoothest candidates, optimised directly -------------------

def test_p14_batchopt_selects_least_mjac_candidates():
    rb = synth.make_robot(3)
    prob = synth.make_problem(rb, seed=9, T=12, K=9, sigma=0.1, n_branch=3)
    cand = prob.cand.copy()
    cand[4] = cand[2]                    # an exact tie: the lower index goes first
    targets = oracle.fk(rb, prob.q_star)
    idx, res = oracle.batchopt(rb, cand, targets, 5, 3)
    # numpy's own mjac: max |q_{t+1} - q_t| over steps and joints
    m = np.abs(np.diff(cand, axis=1)).max(axis=(1, 2))
    expect = sorted(range(len(cand)), key=lambda k: (m[k], k))[:5]
    assert idx == expect
    assert idx.index(2) < idx.index(4) if 4 in idx else True
    for k, r in zip(idx, res):
        assert np.all(r["path"] == 0)   # one candidate: the search keeps it
        ref = oracle.plan(rb, cand[k:k + 1], targets, 3)
        assert np.array_equal(r["xi"], ref["xi"])


# ---- pose-first alternating schedule with the latest-valid store --------------

def _sched_case(seed=1, T=30, sigma=0.02):
    rb = synth.make_robot(seed)
    prob = synth.make_problem(rb, seed=seed, T=T, K=1, sigma=sigma)
    return rb, prob, oracle.fk(rb, prob.q_star)


def test_p15_schedule_pose_step_is_lm_without_smoothness():
    rb, prob, tg = _sched_case()
    r = oracle.lm_schedule(rb, prob.cand[0], tg, 1)
    ref = oracle.lm(rb, prob.cand[0], tg, 1, opts=dict(w_smooth=0.0))
    assert r["pose_steps"] == 1 and r["diff_steps"] == 0 and r["first_valid"] == -1
    assert np.array_equal(r["xi"], ref["xi"])


def test_p15_schedule_valid_seed_takes_a_differencing_step():
    rb, prob, tg = _sched_case()
    xi0 = prob.q_star.copy()             # exact targets: pose error 0, smooth path
    r = oracle.lm_schedule(rb, xi0, tg, 1)
    ref = oracle.lm(rb, xi0, tg, 1, opts=dict(w_pose=0.0))
    assert r["first_valid"] == 0 and r["diff_steps"] == 1 and r["pose_steps"] == 0
    assert np.array_equal(r["xi"], ref["xi"])
    assert np.array_equal(r["xi_valid"], np.clip(xi0, rb.q_lo, rb.q_hi))


def test_p15_schedule_latest_valid_meets_the_thresholds():
    rb, prob, tg = _sched_case(seed=2, T=40, sigma=0.03)
    r = oracle.lm_schedule(rb, prob.cand[0], tg, 40)
    assert r["rc"] == 0 and r["n_valid"] >= 1 and r["pose_steps"] + r["diff_steps"] == 40
    xv = r["xi_valid"]
    ep, er = oracle.pose_compare(rb, xv, targets=tg)
    assert ep <= 1e-4 and er <= np.deg2rad(0.1)
    steps = np.abs(np.diff(xv, axis=0))
    assert steps.max() <= np.deg2rad(7.0)
    assert r["valid_length"] == pytest.approx(steps.sum(), rel=1e-12)


def test_p15_schedule_unreachable_targets_stay_invalid():
    rb, prob, tg = _sched_case(seed=3, T=10)
    far = tg.copy()
    far[:, :3] += 10.0                   # 10 m away: beyond any 7-link reach here
    r = oracle.lm_schedule(rb, prob.cand[0], far, 5)
    assert r["n_valid"] == 0 and r["first_valid"] == -1 and r["xi_valid"] is None
    assert r["pose_steps"] == 5


def test_p15_schedule_rejects_a_discontinuous_pose_valid_trajectory():
    rb, prob, tg = _sched_case(seed=4, T=20)
    q = prob.q_star.copy()
    q[10:, 0] += np.deg2rad(10.0)        # a 10 degree step of joint 1 between waypoints 9 and 10
    q = np.clip(q, rb.q_lo, rb.q_hi)
    tgj = oracle.fk(rb, q)
    r = oracle.lm_schedule(rb, q, tgj, 1)
    # the seed reaches its targets exactly (a differencing step follows) but
    # is not valid: one joint changes by more than 7 degrees
    assert r["diff_steps"] == 1 and r["pose_steps"] == 0
    assert r["first_valid"] == -1 and r["n_valid"] == 0


def _replay_schedule(rb, x0, tg, kmax):
    """Replays a schedule run step by step from the oracle's own LM step:
    returns (differencing steps, rejected steps, longest run of rejects)."""
    lam0 = oracle.DEFAULT_LM["lambda0"]
    prev = oracle.lm_schedule(rb, x0, tg, 0)
    lam_pose, nu_pose = lam0, 2.0
    n_diff = n_rej = run = longest = 0
    for k in range(1, kmax + 1):
        cur = oracle.lm_schedule(rb, x0, tg, k)
        x = prev["xi"]
        diff = cur["diff_steps"] > prev["diff_steps"]
        wp, ws = (0.0, 0.1) if diff else (1.0, 0.0)
        lam = lam0 if diff else lam_pose
        d, g = oracle.lm_step(rb, x, tg, wp, ws, lam)
        trial = np.clip(x + d, rb.q_lo, rb.q_hi)
        c, cn = oracle.cost(rb, x, tg, wp, ws), oracle.cost(rb, trial, tg, wp, ws)
        np.testing.assert_allclose(cur["xi"], trial if cn < c else x, rtol=0, atol=1e-12)
        if not diff:   # the Nielsen rule on the pose objective
            if cn < c:
                u = 2.0 * (c - cn) / (0.5 * np.sum(d * (lam * d - g))) - 1.0
                lam_pose, nu_pose = lam * max(1.0 / 3.0, 1.0 - u * u * u), 2.0
            else:
                lam_pose, nu_pose = lam * nu_pose, 2.0 * nu_pose
            lam_pose = min(max(lam_pose, 1e-10), 1e10)
        n_diff += diff
        run = run + 1 if cn >= c else 0
        n_rej += cn >= c
        longest = max(longest, run)
        prev = cur
    return n_diff, n_rej, longest


def test_p15_schedule_steps_are_single_objective_lm_steps():
    """Each step of a run is one damped step of its own objective from the
    previous iterate (runs of k and k+1 iterations share their first k): a
    differencing step with the fixed damping lambda0 (w_pose = 0), a pose
    step with the damping the pose steps before it left by the Nielsen rule
    (w_smooth = 0), accepted iff it lowers that objective.  One smooth case
    alternates; one rough case (1.5 rad noise) has rejected pose steps, two
    in a row."""
    rb, prob, tg = _sched_case(seed=2, T=40, sigma=0.03)
    n_diff, _, _ = _replay_schedule(rb, prob.cand[0], tg, 15)
    assert n_diff >= 2
    rb, prob, tg = _sched_case(seed=8, T=20, sigma=1.5)
    _, n_rej, longest = _replay_schedule(rb, prob.cand[0], tg, 12)
    assert n_rej >= 3 and longest >= 2


# ---- collision distances, residuals and penalty (Sec. II, III-B, III-C) --------

def test_p16_seg_seg_closed_forms():
    # parallel segments 0.3 apart, overlapping in x: distance 0.3
    d2, s, t = oracle.seg_seg([0, 0, 0], [1, 0, 0], [0.5, 0.3, 0], [2, 0.3, 0])
    assert d2 == pytest.approx(0.09, abs=1e-15)
    # crossing segments: distance 0 at the midpoints
    d2, s, t = oracle.seg_seg([-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0])
    assert d2 == 0.0 and s == pytest.approx(0.5) and t == pytest.approx(0.5)
    # skew perpendicular lines 0.2 apart in z, closest points interior
    d2, s, t = oracle.seg_seg([-1, 0, 0], [1, 0, 0], [0.25, -1, 0.2], [0.25, 1, 0.2])
    assert d2 == pytest.approx(0.04, abs=1e-15) and s == pytest.approx(0.625) and t == pytest.approx(0.5)
    # closest points at the ends: collinear, gap 0.5
    d2, s, t = oracle.seg_seg([0, 0, 0], [1, 0, 0], [1.5, 0, 0], [3, 0, 0])
    assert d2 == pytest.approx(0.25, abs=1e-15) and s == 1.0 and t == 0.0
    # a point (zero-length segment) against a segment
    d2, s, t = oracle.seg_seg([0.5, 0.4, 0], [0.5, 0.4, 0], [0, 0, 0], [1, 0, 0])
    assert d2 == pytest.approx(0.16, abs=1e-15) and t == pytest.approx(0.5)


@pytest.mark.parametrize("seed", range(6))
def test_p16_seg_seg_matches_bounded_minimiser(seed):
    from scipy.optimize import minimize
    rng = np.random.default_rng(seed)
    P0, P1, Q0, Q1 = rng.uniform(-1, 1, (4, 3))
    f = lambda x: np.sum((P0 + x[0] * (P1 - P0) - Q0 - x[1] * (Q1 - Q0)) ** 2)
    best = min(minimize(f, x0, bounds=[(0, 1), (0, 1)], method="L-BFGS-B", tol=1e-14).fun
               for x0 in ([0.5, 0.5], [0, 0], [1, 1], [0, 1], [1, 0]))
    d2, s, t = oracle.seg_seg(P0, P1, Q0, Q1)
    assert d2 == pytest.approx(best, abs=1e-10)
    assert d2 == pytest.approx(f([s, t]), abs=1e-14) and 0 <= s <= 1 and 0 <= t <= 1


def test_p16_seg_box_closed_forms():
    lo, hi = np.array([-0.1, -0.2, -0.3]), np.array([0.1, 0.2, 0.3])
    # parallel to the +x face, 0.25 outside it, spanning the face: distance 0.25
    d2, s = oracle.seg_box([0.35, -1, 0], [0, 2, 0], lo, hi)
    assert d2 == pytest.approx(0.0625, abs=1e-15)
    # through the box: 0
    d2, s = oracle.seg_box([-1, 0, 0], [2, 0, 0], lo, hi)
    assert d2 == 0.0
    # towards a corner, stopping short: the end point's distance to the corner
    d2, s = oracle.seg_box([1, 1, 1], [-0.5, -0.5, -0.5], lo, hi)
    assert s == 1.0 and d2 == pytest.approx(0.4 ** 2 + 0.3 ** 2 + 0.2 ** 2, abs=1e-15)
    # passing an edge diagonally: closest approach at the edge x=0.1, y=0.2
    d2, s = oracle.seg_box([0.3, -0.5, 0], [0, 2, 0], lo, hi)
    assert d2 == pytest.approx(0.04, abs=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_p16_seg_box_matches_dense_sampling(seed):
    rng = np.random.default_rng(100 + seed)
    A, D = rng.uniform(-0.6, 0.6, 3), rng.uniform(-1, 1, 3)
    h = rng.uniform(0.05, 0.3, 3)
    lo, hi = -h + rng.uniform(-0.1, 0.1, 3), h
    s = np.linspace(0, 1, 200001)
    x = A[None, :] + s[:, None] * D[None, :]
    gap = np.maximum(lo - x, 0) + np.maximum(x - hi, 0)
    sampled = (gap ** 2).sum(axis=1)
    d2, sm = oracle.seg_box(A, D, lo, hi)
    assert d2 <= sampled.min() + 1e-15                     # the QP is the true minimum
    assert sampled.min() - d2 <= 2e-10 * (1 + np.abs(D).sum())  # and the samples approach it
    xm = A + sm * D
    assert d2 == pytest.approx(float(((np.maximum(lo - xm, 0) + np.maximum(xm - hi, 0)) ** 2).sum()), abs=1e-15)


def _coll_case(robot_seed=0, n_obs=4):
    rb = synth.make_robot(robot_seed)
    return rb, synth.collision_model(rb, synth.make_obstacles(robot_seed, n_obs))


def _link_frame(rb, q, i):
    """Frame after link i from FK of the chain cut after link i."""
    cut = synth.Robot(a=rb.a[:i + 1], d=rb.d[:i + 1], alpha=rb.alpha[:i + 1],
                      theta_off=rb.theta_off[:i + 1], q_lo=rb.q_lo[:i + 1], q_hi=rb.q_hi[:i + 1])
    pose = oracle.fk(cut, q[:i + 1])
    return pose[3:12].reshape(3, 3), pose[:3]


def test_p16_capsules_span_consecutive_joints():
    """Untrimmed synthetic capsules run from the joint of link i (origin of
    the frame before it) to the next joint (origin of the frame after it)."""
    rb = synth.make_robot(1)
    caps = synth.make_capsules(rb, trim=0.0)
    q = np.random.default_rng(3).uniform(-1, 1, 7)
    prev = np.zeros(3)
    for i in range(7):
        R, p = _link_frame(rb, q, i)
        np.testing.assert_allclose(R @ caps[i, 0:3] + p, prev, atol=1e-12)
        np.testing.assert_allclose(R @ caps[i, 3:6] + p, p, atol=1e-12)
        prev = p


@pytest.mark.parametrize("seed", range(4))
def test_p16_distances_match_independent_evaluation(seed):
    """Self and environment distances against capsules placed by FK of the
    truncated chains and scipy's bounded minimiser over the QP variables."""
    from scipy.optimize import minimize
    rb, cm = _coll_case(seed % 2)
    q = np.random.default_rng(seed).uniform(-2, 2, 7)
    caps = cm["capsules"]
    ends = []
    for i in range(7):
        R, p = _link_frame(rb, q, i)
        ends.append((R @ caps[i, 0:3] + p, R @ caps[i, 3:6] + p, caps[i, 6]))
    self_d = np.inf
    for i in range(7):
        for j in range(i + 3, 7):
            (a0, a1, ra), (b0, b1, rb_) = ends[i], ends[j]
            f = lambda x: np.sum((a0 + x[0] * (a1 - a0) - b0 - x[1] * (b1 - b0)) ** 2)
            m = min(minimize(f, x0, bounds=[(0, 1), (0, 1)], method="L-BFGS-B", tol=1e-14).fun
                    for x0 in ([0.5, 0.5], [0, 0], [1, 1], [0, 1], [1, 0]))
            self_d = min(self_d, np.sqrt(max(m, 0)) - ra - rb_)
    env_d = np.inf
    for i in range(7):
        a0, a1, ra = ends[i]
        for B in cm["obstacles"]:
            R, o = B[3:12].reshape(3, 3), B[0:3]
            lo, hi = B[12:15], B[15:18]
            def f(x):
                pw = a0 + x[0] * (a1 - a0)
                return np.sum((R @ x[1:4] + o - pw) ** 2)
            x0s = [np.r_[s0, np.clip(R.T @ (a0 + s0 * (a1 - a0) - o), lo, hi)] for s0 in (0, 0.5, 1)]
            m = min(minimize(f, x0, bounds=[(0, 1)] + list(zip(lo, hi)), method="L-BFGS-B",
                             tol=1e-15).fun for x0 in x0s)
            env_d = min(env_d, np.sqrt(max(m, 0)) - ra)
    d = oracle.coll_eval(rb, cm, q)
    assert d[0] == pytest.approx(self_d, abs=1e-6)
    assert d[1] == pytest.approx(env_d, abs=1e-6)


@pytest.mark.parametrize("seed", range(5))
def test_p16_distance_gradients_match_central_differences(seed):
    rb, cm = _coll_case(1)
    q = np.random.default_rng(50 + seed).uniform(-2, 2, 7)
    d, g = oracle.coll_eval(rb, cm, q, gradient=True)
    h = 1e-6
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        fd = (oracle.coll_eval(rb, cm, q + e) - oracle.coll_eval(rb, cm, q - e)) / (2 * h)
        np.testing.assert_allclose(g[:, k], fd, atol=2e-6)


def test_p16_adjacent_links_never_checked():
    """Capsules of links fewer than three apart may overlap freely: a robot
    whose capsules are huge spheres around each joint reports only the pairs
    three or more apart."""
    rb, cm = _coll_case(0, n_obs=0)
    caps = cm["capsules"].copy()
    caps[:, 0:6] = 0.0                 # every capsule a sphere at its frame's origin
    caps[:, 6] = 0.01
    caps[2, 6] = caps[3, 6] = caps[4, 6] = 5.0   # links 2, 3, 4 overlap each other hugely
    cm2 = dict(cm, capsules=caps)
    q = np.zeros(7)
    d = oracle.coll_eval(rb, cm2, q)
    frames = [_link_frame(rb, q, i)[1] for i in range(7)]
    expect = min(np.linalg.norm(frames[i] - frames[j]) - caps[i, 6] - caps[j, 6]
                 for i in range(7) for j in range(i + 3, 7))
    assert d[0] == pytest.approx(expect, abs=1e-12)
    assert np.isinf(d[1])


def test_p16_search_penalises_colliding_nodes_brute_force():
    """Tiny search (K=3, T=4) with collision geometry against enumeration of
    all 81 paths, node penalty = joint-limit term + 100 if in collision."""
    rb, cm = _coll_case(3)
    rng = np.random.default_rng(9)
    cand = rng.uniform(-2.0, 2.0, (3, 4, 7))
    dist = oracle.coll_eval(rb, cm, cand)
    coll = (dist < 0).any(axis=-1)
    assert coll.any() and not coll.all()
    lo, hi = rb.q_lo, rb.q_hi
    near = ((cand <= lo + oracle.oracle.LIMIT_MARGIN) | (cand >= hi - oracle.oracle.LIMIT_MARGIN)).any(-1)
    pen = 10.0 * near + 100.0 * coll                       # [K][T]
    best = np.inf
    for path in itertools.product(range(3), repeat=4):
        v = pen[path[0], 0]
        for t in range(1, 4):
            e = np.abs(cand[path[t], t] - cand[path[t - 1], t - 1]).max()
            v = max(v, e + pen[path[t], t])
        best = min(best, v)
    path, B, _, _ = oracle.dp(cand, rb, coll=cm)
    assert B == best
    _, B0, _, _ = oracle.dp(cand, rb)
    assert B0 < B or not coll.any()


def test_p16_lm_gradient_with_collision_matches_cost_differences():
    rb, cm = _coll_case(3)
    prob = synth.make_problem(rb, seed=7, T=12, K=1, sigma=0.3)
    tg = oracle.fk(rb, prob.q_star)
    xi = prob.cand[0]
    cm = dict(cm, margin=0.3)                  # wide margin: residuals active
    assert (oracle.coll_eval(rb, cm, xi) < 0.3).any()
    _, g = oracle.lm_step(rb, xi, tg, 1.0, 0.1, 1e-3, coll=cm, w_coll=1.0)
    h = 1e-6
    for t, j in [(0, 0), (3, 2), (6, 4), (11, 6), (5, 1)]:
        e = np.zeros_like(xi)
        e[t, j] = h
        fd = (oracle.cost(rb, xi + e, tg, coll=cm) - oracle.cost(rb, xi - e, tg, coll=cm)) / (2 * h)
        assert g[t, j] == pytest.approx(fd, abs=1e-5, rel=1e-5)
    # no geometry: the collision terms vanish
    assert oracle.cost(rb, xi, tg, coll=dict(cm, w_coll=0.0)) == oracle.cost(rb, xi, tg)


def test_p16_schedule_rejects_a_colliding_pose_valid_trajectory():
    rb, cm = _coll_case(1)
    prob = synth.make_problem(rb, seed=7, T=80, K=1, sigma=0.02)
    q = prob.q_star.copy()
    tg = oracle.fk(rb, q)
    d = oracle.coll_eval(rb, cm, q)
    assert (d >= 0).all() and oracle.mjac(q) <= oracle.VALID_TOL[2]
    # a cuboid around the end effector's second waypoint makes q collide
    box = np.zeros(18)
    box[0:3] = tg[1, :3]
    box[3:12] = np.eye(3).ravel()
    box[12:15], box[15:18] = -0.02, 0.02
    cm_hit = dict(cm, obstacles=np.vstack([cm["obstacles"], box]))
    assert oracle.coll_eval(rb, cm_hit, q)[1, 1] < 0
    r = oracle.lm_schedule(rb, q, tg, 0, coll=cm_hit)
    assert r["n_valid"] == 0
    r = oracle.lm_schedule(rb, q, tg, 0, coll=cm)
    assert r["n_valid"] == 1


# ---- P17: prismatic joints (Sec. IV's Fetch.Full torso lift) ----------------

def _prismatic_exact(seed=0, joint=2):
    rb = exact_robot(seed)
    jt = np.zeros(7, dtype=np.int32)
    jt[joint] = 1
    rb.joint_type = jt
    rb.q_lo[joint], rb.q_hi[joint] = 0.0, 0.4
    return rb


@pytest.mark.parametrize("joint", [0, 2, 6])
@pytest.mark.parametrize("s", [0.05, 0.3])
def test_p17_prismatic_joint_translates_along_its_axis(joint, s):
    """At q = 0 the axis of joint i is (0, -sin A_i, cos A_i) with A_i the sum
    of the twists before it (the closed form of P1): extending a prismatic
    joint by s moves the end effector by s times that axis and leaves the
    rotation alone."""
    rb = _prismatic_exact(1, joint)
    p0, R0, A = zero_pose_closed_form(rb)
    axis = np.array([0.0, -math.sin(A[joint]), math.cos(A[joint])])
    q = np.zeros(7)
    q[joint] = s
    p, R = split(oracle.fk(rb, q))
    np.testing.assert_allclose(p, p0 + s * axis, atol=1e-15)
    np.testing.assert_allclose(R, R0, atol=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_p17_prismatic_motion_is_a_pure_translation_anywhere(seed):
    """At any configuration the end effector moves linearly in the joint's
    value along a unit direction, without rotating."""
    rb = synth.make_robot_prismatic(seed, joint=seed % 3)
    j = seed % 3
    q = synth.random_configs(seed, 1, rb)[0]
    q[j] = 0.1
    base_p, base_R = split(oracle.fk(rb, q))
    dirs = []
    for s in (0.05, 0.2):
        q2 = q.copy()
        q2[j] += s
        p, R = split(oracle.fk(rb, q2))
        np.testing.assert_allclose(R, base_R, atol=1e-15)
        dirs.append((p - base_p) / s)
    np.testing.assert_allclose(dirs[0], dirs[1], atol=1e-13)
    assert np.linalg.norm(dirs[0]) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_p17_jacobian_with_prismatic_joint_finite_differences(seed):
    rb = synth.make_robot_prismatic(seed, joint=seed % 7)
    q = synth.random_configs(100 + seed, 1, rb)[0]
    _, J = oracle.fk(rb, q, jacobian=True)
    h = 1e-6
    for i in range(7):
        e = np.zeros(7)
        e[i] = h
        pp, Rp = split(oracle.fk(rb, q + e))
        pm, Rm = split(oracle.fk(rb, q - e))
        np.testing.assert_allclose(J[:3, i], (pp - pm) / (2 * h), atol=1e-8)
        w = Rotation.from_matrix(Rp @ Rm.T).as_rotvec() / (2 * h)
        np.testing.assert_allclose(J[3:, i], w, atol=1e-8)


def test_p17_lm_gradient_with_prismatic_joint_matches_cost_differences():
    rb = synth.make_robot_prismatic(3)
    prob = synth.make_problem(rb, seed=3, T=6, K=1, sigma=0.3)
    tg = oracle.fk(rb, prob.q_star)
    xi = prob.cand[0]
    _, g = oracle.lm_step(rb, xi, tg, 1.0, 0.1, 1.0)
    h = 1e-6
    for t in range(6):
        for j in range(7):
            e = np.zeros_like(xi)
            e[t, j] = h
            fd = (oracle.cost(rb, xi + e, tg) - oracle.cost(rb, xi - e, tg)) / (2 * h)
            assert g[t, j] == pytest.approx(fd, abs=1e-7, rel=1e-6)


def test_p17_limit_margin_is_three_cm_for_a_prismatic_joint():
    """Sec. III-B: the penalty applies within 1.5 degrees of a revolute
    joint's limit and within 3 cm of a prismatic joint's.  0.028 m is inside
    3 cm but outside 1.5 degrees (0.0262) read as a number."""
    rb = synth.make_robot_prismatic(0)
    cand = np.zeros((4, 1, 7))
    cand[:, 0, 0] = [0.028, 0.2, 0.032, 0.372]   # joint 0 travels [0, 0.4]
    extra = np.array([[0.0, 0.5, 0.7, 0.0]])
    path, best, _, _ = oracle.dp(cand, rb, extra=extra)
    assert path[0] == 1 and best == 0.5          # 0 and 3 lie within 3 cm of a limit
    cand[1, 0, 0] = 0.2 + 1e-3
    extra[0, 1] = 0.8
    path, best, _, _ = oracle.dp(cand, rb, extra=extra)
    assert path[0] == 2 and best == 0.7


def test_p17_seed_steps_split_by_joint_type():
    rb = synth.make_robot_prismatic(1)
    prob = synth.make_problem(rb, seed=2, T=40, K=1, sigma=0.1)
    xi = prob.cand[0]
    rev, pri = oracle.seed_steps(xi, rb)
    st = np.abs(np.diff(xi, axis=0))
    assert pri == st[:, 0].max() and rev == st[:, 1:].max()
    assert max(rev, pri) == oracle.mjac(xi)
    rb0 = synth.make_robot(1)
    assert oracle.seed_steps(xi, rb0) == (oracle.mjac(xi), 0.0)


def test_p17_schedule_step_threshold_is_two_cm_for_a_prismatic_joint():
    """Sec. II: at most 7 degrees per revolute joint and 2 cm per prismatic
    joint between waypoints.  A pose-exact trajectory whose prismatic joint
    steps by 2.5 cm (well under 7 degrees read as a number) is not valid; the
    same with a 1.5 cm step is."""
    rb = synth.make_robot_prismatic(2)
    prob = synth.make_problem(rb, seed=5, T=20, K=1, sigma=0.0)
    for step, valid in [(0.025, 0), (0.015, 1)]:
        q = prob.q_star.copy()
        q[:, 0] = 0.1
        q[10:, 0] += step
        assert np.abs(np.diff(q[:, 1:], axis=0)).max() <= oracle.VALID_TOL[2]
        tg = oracle.fk(rb, q)
        r = oracle.lm_schedule(rb, q, tg, 0)
        assert r["n_valid"] == valid, step


@pytest.mark.parametrize("seed", range(3))
def test_p17_collision_gradient_with_prismatic_joint(seed):
    rb = synth.make_robot_prismatic(seed + 1)
    cm = synth.collision_model(rb, synth.make_obstacles(seed + 1, 6))
    q = synth.random_configs(70 + seed, 1, rb, spread=2.0)[0]
    d, g = oracle.coll_eval(rb, cm, q, gradient=True)
    h = 1e-6
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        fd = (oracle.coll_eval(rb, cm, q + e) - oracle.coll_eval(rb, cm, q - e)) / (2 * h)
        np.testing.assert_allclose(g[:, k], fd, atol=2e-6)
    # the prismatic joint moves every capsule after it rigidly along its
    # axis: the self-distance gradient of joint 0 vanishes (links 1.. move
    # together; link 0's capsule rides on the joint too)
    assert g[0, 0] == pytest.approx(0.0, abs=1e-12)


# ---- P18: chains of 8 joints (Sec. IV's Fetch.Full: torso lift + 7-joint arm) --

@pytest.mark.parametrize("seed", range(3))
def test_p18_fk_zero_configuration_eight_joints(seed):
    rb = exact_robot(seed, n=8)
    p, R = split(oracle.fk(rb, np.zeros(8)))
    p_ref, R_ref, _ = zero_pose_closed_form(rb)
    np.testing.assert_allclose(p, p_ref, atol=1e-15)
    np.testing.assert_allclose(R, R_ref, atol=1e-15)


@pytest.mark.parametrize("theta", [1.0, -HALF_PI, 2.5])
def test_p18_fk_single_axis_eight_joints(theta):
    """Turning joint i alone rotates everything after it about joint i's axis
    through its origin (both from the zero configuration's closed form)."""
    rb = exact_robot(4, n=8)
    p0, R0, A = zero_pose_closed_form(rb)
    for i in range(8):
        axis = np.array([0.0, -math.sin(A[i]), math.cos(A[i])])
        origin = np.zeros(3)
        for k in range(i):
            origin += np.array([rb.a[k], -rb.d[k] * math.sin(A[k]), rb.d[k] * math.cos(A[k])])
        Rot = Rotation.from_rotvec(theta * axis).as_matrix()
        q = np.zeros(8)
        q[i] = theta
        p, R = split(oracle.fk(rb, q))
        np.testing.assert_allclose(p, origin + Rot @ (p0 - origin), atol=1e-14)
        np.testing.assert_allclose(R, Rot @ R0, atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_p18_torso_lift_is_a_translation_along_the_base_axis(seed):
    """The first joint of the torso-arm chain is prismatic along the base z
    axis: extending it by s moves the end effector by s along z and leaves
    its orientation, at any arm configuration."""
    rb = synth.make_robot_torso_arm(seed)
    q = synth.random_configs(200 + seed, 1, rb)[0]
    q2 = q.copy()
    q2[0] = q[0] + 0.05 if q[0] < 0.3 else q[0] - 0.05
    p, R = split(oracle.fk(rb, q))
    p2, R2 = split(oracle.fk(rb, q2))
    np.testing.assert_allclose(p2 - p, [0.0, 0.0, q2[0] - q[0]], atol=1e-14)
    np.testing.assert_allclose(R2, R, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_p18_jacobian_torso_arm_finite_differences(seed):
    rb = synth.make_robot_torso_arm(seed)
    q = synth.random_configs(300 + seed, 1, rb)[0]
    _, J = oracle.fk(rb, q, jacobian=True)
    assert J.shape == (6, 8)
    h = 1e-6
    for i in range(8):
        e = np.zeros(8)
        e[i] = h
        pp, Rp = split(oracle.fk(rb, q + e))
        pm, Rm = split(oracle.fk(rb, q - e))
        np.testing.assert_allclose(J[:3, i], (pp - pm) / (2 * h), atol=1e-8)
        w = Rotation.from_matrix(Rp @ Rm.T).as_rotvec() / (2 * h)
        np.testing.assert_allclose(J[3:, i], w, atol=1e-8)
    np.testing.assert_allclose(J[:, 0], [0, 0, 1, 0, 0, 0], atol=1e-15)


@given(st.integers(1, 3), st.integers(1, 5), st.integers(0, 2**31 - 1))
@settings(max_examples=40, deadline=None)
def test_p18_dp_matches_brute_force_eight_joints(K, T, seed):
    rng = np.random.default_rng(seed)
    rb = synth.make_robot(2, 8)
    cand = np.clip(rng.uniform(-2.8, 2.8, (K, T, 8)), rb.q_lo, rb.q_hi)
    path, best, B_all, _ = oracle.dp(cand, rb, want_tables=True)
    B_ref, value = brute_force_tables(cand, rb)
    assert np.array_equal(B_all, B_ref)
    assert best == B_ref[-1].min() and value(tuple(path)) == best


def test_p18_lm_gradient_eight_joints_matches_cost_differences():
    rb = synth.make_robot_torso_arm(3)
    prob = synth.make_problem(rb, seed=3, T=5, K=1, sigma=0.3)
    tg = oracle.fk(rb, prob.q_star)
    xi = prob.cand[0]
    _, g = oracle.lm_step(rb, xi, tg, 1.0, 0.1, 1.0)
    h = 1e-6
    for t in range(5):
        for j in range(8):
            e = np.zeros_like(xi)
            e[t, j] = h
            fd = (oracle.cost(rb, xi + e, tg) - oracle.cost(rb, xi - e, tg)) / (2 * h)
            assert g[t, j] == pytest.approx(fd, abs=1e-7, rel=1e-6)
