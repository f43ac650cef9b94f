"""Seeded synthetic workloads for the CppFlow refinement path (arXiv 2309.09102).

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no kinematics, no search, no optimisation). Target poses
are FK(q*), so they are produced by the caller with whichever forward
kinematics it owns and passed back in through ``Problem.with_targets``.

Workload shapes follow the paper: candidate plans come from a generative IK
model as K joint-space trajectories over T waypoints (Sec. III-A), the robot is
a redundant 7-DOF serial chain (Sec. II), and the default K sits in the range
of the paper's K=175 (Sec. III-A).  The paper's robots and target paths are
not available, so a random standard-DH chain and a sum-of-sinusoids joint path
stand in for them.

Draw order (fixed; changing it changes every workload):
  robot   rng = default_rng([seed, 0]):  a ~ U[0, 0.1] (n), d ~ U[0, 0.4] (n),
          alpha sign bit ~ U{0, 1} (n)  -> alpha = -pi/2 or +pi/2
  prismatic robot: the robot of the same seed with joint 0 prismatic,
          travel [0, 0.4] m (no draws)
  problem rng = default_rng([seed, 1]):  centre c ~ U[-1, 1] (n),
          amplitude A ~ U[0, 0.5/3] (n, 3), frequency f ~ U[0.25, 1.5] (n, 3)
          cycles per path, phase ~ U[0, 2 pi) (n, 3); then the candidate noise
          N(0, sigma) (K, T, n); then a permutation of K (the first nb get a
          branch offset); then one sign per (offset candidate, joint 2/4/6).
A prismatic joint's path, noise and branch offset are drawn in the same
units as a revolute joint's and then mapped affinely onto its travel: the
revolute limit range [-2.8, 2.8] onto [q_lo, q_hi] (scale (q_hi - q_lo) / 5.6
about the middle of the travel).
Every value handed to either implementation is rounded to the nearest float32
and stored as float64, so both sides see bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

N_JOINTS = 7
Q_LIMIT = float(np.float32(2.8))
# 1-based joints 2, 4 and 6 of the chain get the branch offset.
BRANCH_JOINTS = (1, 3, 5)


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass
class Robot:
    """Standard (distal) DH chain: one joint per row, revolute unless
    joint_type marks it prismatic (1)."""
    a: np.ndarray
    d: np.ndarray
    alpha: np.ndarray
    theta_off: np.ndarray
    q_lo: np.ndarray
    q_hi: np.ndarray
    joint_type: np.ndarray | None = None

    @property
    def dof(self) -> int:
        return int(self.a.shape[0])

    def prismatic(self) -> np.ndarray:
        """bool [n]: which joints are prismatic."""
        if self.joint_type is None:
            return np.zeros(self.dof, dtype=bool)
        return np.asarray(self.joint_type) == 1


def _joint_map(robot: Robot):
    """(centre, scale) per joint: identity for revolute joints; for a
    prismatic joint the map of [-Q_LIMIT, Q_LIMIT] onto its travel."""
    pr = robot.prismatic()
    ctr = np.where(pr, 0.5 * (robot.q_lo + robot.q_hi), 0.0)
    sc = np.where(pr, (robot.q_hi - robot.q_lo) / (2.0 * Q_LIMIT), 1.0)
    return ctr, sc


@dataclasses.dataclass
class Problem:
    """One planning request: T target poses and K candidate plans."""
    robot: Robot
    q_star: np.ndarray          # [T][n] ground-truth joint path
    cand: np.ndarray            # [K][T][n] candidate plans
    targets: np.ndarray | None  # [T][12] (x, y, z, R row-major); None until set
    seed: int
    sigma: float
    branch_frac: float

    @property
    def T(self) -> int:
        return int(self.q_star.shape[0])

    @property
    def K(self) -> int:
        return int(self.cand.shape[0])

    def with_targets(self, fk_poses: np.ndarray) -> "Problem":
        """Attach target poses FK(q*) computed by the caller ([T][12])."""
        fk_poses = np.asarray(fk_poses, dtype=np.float64).reshape(self.T, 12)
        return dataclasses.replace(self, targets=_f32(fk_poses))


def make_robot(seed: int, n: int = N_JOINTS) -> Robot:
    rng = np.random.default_rng([seed, 0])
    a = rng.uniform(0.0, 0.1, n)
    d = rng.uniform(0.0, 0.4, n)
    bit = rng.integers(0, 2, n)
    alpha = np.where(bit == 0, -math.pi / 2, math.pi / 2)
    return Robot(a=_f32(a), d=_f32(d), alpha=_f32(alpha),
                 theta_off=np.zeros(n), q_lo=np.full(n, -Q_LIMIT),
                 q_hi=np.full(n, Q_LIMIT))


def make_robot_prismatic(seed: int, joint: int = 0, travel: float = 0.4) -> Robot:
    """The robot of make_robot(seed) with one prismatic joint (a torso lift
    like the Fetch.Full chain's, Sec. IV) of travel [0, travel] m; its DH
    offset d is the link's length at zero extension."""
    rb = make_robot(seed)
    jt = np.zeros(rb.dof, dtype=np.int32)
    jt[joint] = 1
    lo, hi = rb.q_lo.copy(), rb.q_hi.copy()
    lo[joint], hi[joint] = 0.0, float(np.float32(travel))
    return dataclasses.replace(rb, q_lo=lo, q_hi=hi, joint_type=jt)


def make_robot_torso_arm(seed: int, travel: float = 0.4) -> Robot:
    """An 8-joint chain standing in for the Fetch.Full robot of the
    experiments (Sec. IV): a prismatic torso lift of travel [0, travel] m
    (joint 0; its DH offset d is the link's length at zero extension) ahead
    of a 7-joint revolute arm, all rows drawn as make_robot's are."""
    rb = make_robot(seed, N_JOINTS + 1)
    jt = np.zeros(rb.dof, dtype=np.int32)
    jt[0] = 1
    lo, hi = rb.q_lo.copy(), rb.q_hi.copy()
    lo[0], hi[0] = 0.0, float(np.float32(travel))
    return dataclasses.replace(rb, q_lo=lo, q_hi=hi, joint_type=jt)


def _path(robot: Robot, seed: int, T: int, rng=None) -> np.ndarray:
    """Ground-truth joint path q* [T][n] (float32 values): the first draws of
    default_rng([seed, 1]) (rng continues from there when given)."""
    n = robot.dof
    if rng is None:
        rng = np.random.default_rng([seed, 1])
    c = rng.uniform(-1.0, 1.0, n)
    A = rng.uniform(0.0, 0.5 / 3.0, (n, 3))
    f = rng.uniform(0.25, 1.5, (n, 3))
    ph = rng.uniform(0.0, 2 * math.pi, (n, 3))
    s = np.arange(T, dtype=np.float64) / max(T - 1, 1)
    arg = 2 * math.pi * f[None, :, :] * s[:, None, None] + ph[None, :, :]
    q_star = c[None, :] + np.sum(A[None, :, :] * np.sin(arg), axis=2)
    ctr, sc = _joint_map(robot)
    return np.clip(_f32(ctr + sc * q_star), robot.q_lo, robot.q_hi)


def make_problem(robot: Robot, seed: int, T: int, K: int, sigma: float,
                 branch_frac: float = 0.0, n_branch: int | None = None,
                 mode: str = "iid") -> Problem:
    """Ground-truth path q* and K noisy candidate plans around it.

    mode="iid": noise independent per (candidate, waypoint, joint).
    mode="smooth": noise drawn per (candidate, joint) and held along the path,
    closer to the slowly varying plans a generative IK model returns.
    """
    if T < 1 or K < 1:
        raise ValueError("T and K must be >= 1")
    n = robot.dof
    rng = np.random.default_rng([seed, 1])
    q_star = _path(robot, seed, T, rng)
    _, sc = _joint_map(robot)

    if mode == "iid":
        noise = rng.normal(0.0, sigma, (K, T, n))
    elif mode == "smooth":
        noise = np.broadcast_to(rng.normal(0.0, sigma, (K, 1, n)), (K, T, n))
    else:
        raise ValueError(f"unknown candidate mode {mode!r}")
    cand = q_star[None, :, :] + sc * noise
    nb = int(round(branch_frac * K)) if n_branch is None else int(n_branch)
    nb = max(0, min(nb, K))
    perm = rng.permutation(K)
    sel = perm[:nb]
    signs = rng.choice(np.array([-1.0, 1.0]), (nb, len(BRANCH_JOINTS)))
    joints = [j for j in BRANCH_JOINTS if j < n]
    for r, k in enumerate(sel):
        for c_i, j in enumerate(joints):
            cand[k, :, j] += signs[r, c_i] * (math.pi / 2) * sc[j]
    cand = np.clip(_f32(cand), robot.q_lo[None, None, :], robot.q_hi[None, None, :])
    return Problem(robot=robot, q_star=q_star, cand=np.ascontiguousarray(cand),
                   targets=None, seed=seed, sigma=float(sigma),
                   branch_frac=float(nb) / K)


def more_candidates(prob: Problem, K_add: int, batch: int = 1) -> np.ndarray:
    """K_add further candidate plans [K_add][T][n] around the same path q*,
    drawn like the problem's own (same sigma and branch-offset fraction) from
    an independent stream per batch (the stand-in for asking the candidate
    generator for more plans)."""
    if K_add < 1:
        raise ValueError("K_add must be >= 1")
    rb = prob.robot
    n = rb.dof
    rng = np.random.default_rng([prob.seed, 2, batch])
    _, sc = _joint_map(rb)
    cand = prob.q_star[None, :, :] + sc * rng.normal(0.0, prob.sigma, (K_add, prob.T, n))
    nb = int(round(prob.branch_frac * K_add))
    sel = rng.permutation(K_add)[:nb]
    signs = rng.choice(np.array([-1.0, 1.0]), (nb, len(BRANCH_JOINTS)))
    joints = [j for j in BRANCH_JOINTS if j < n]
    for r, k in enumerate(sel):
        for c_i, j in enumerate(joints):
            cand[k, :, j] += signs[r, c_i] * (math.pi / 2) * sc[j]
    return np.ascontiguousarray(np.clip(_f32(cand), rb.q_lo[None, None, :], rb.q_hi[None, None, :]))


def make_capsules(robot: Robot, trim: float = 0.15, radius_frac: float = 0.2,
                  r_max: float = 0.03) -> np.ndarray:
    """One capsule per link [n][7] (p0 xyz, p1 xyz in the frame after the
    link, radius): the part of the segment from the link's joint to the next
    joint that remains after cutting `trim` of its length off both ends, with
    radius min(r_max, radius_frac x length).  In the frame after link i of a
    standard DH chain the joint of link i sits at (-a_i, -d_i sin alpha_i,
    -d_i cos alpha_i) and the next joint at the origin (a prismatic link: at
    zero extension)."""
    a, d, al = robot.a, robot.d, robot.alpha
    out = np.zeros((robot.dof, 7))
    for i in range(robot.dof):
        j0 = np.array([-a[i], -d[i] * math.sin(al[i]), -d[i] * math.cos(al[i])])
        j1 = np.zeros(3)
        L = float(np.linalg.norm(j1 - j0))
        out[i, 0:3] = j0 + trim * (j1 - j0)
        out[i, 3:6] = j1 - trim * (j1 - j0)
        out[i, 6] = min(r_max, radius_frac * L)
    return out


def make_obstacles(seed: int, n_obs: int, r_lo: float = 0.3, r_hi: float = 0.9,
                   ext_lo: float = 0.03, ext_hi: float = 0.12) -> np.ndarray:
    """n_obs cuboids [n_obs][18] (frame origin xyz, rotation row-major, p_min
    xyz, p_max xyz): origins uniform in direction at a distance U[r_lo, r_hi]
    from the base, rotations from uniform unit quaternions, half extents
    U[ext_lo, ext_hi] per axis, centred in their frame."""
    rng = np.random.default_rng([seed, 3])
    out = np.zeros((n_obs, 18))
    for m in range(n_obs):
        v = rng.normal(size=3)
        out[m, 0:3] = v / np.linalg.norm(v) * rng.uniform(r_lo, r_hi)
        w, x, y, z = (lambda u: u / np.linalg.norm(u))(rng.normal(size=4))
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        out[m, 3:12] = R.ravel()
        h = rng.uniform(ext_lo, ext_hi, 3)
        out[m, 12:15] = -h
        out[m, 15:18] = h
    return out


def collision_model(robot: Robot, obstacles: np.ndarray | None = None, margin: float = 0.02,
                    w_coll: float = 1.0, penalty: float = 100.0) -> dict:
    """Collision description shared by the oracle and the library binding."""
    return dict(capsules=make_capsules(robot),
                obstacles=np.zeros((0, 18)) if obstacles is None else np.asarray(obstacles, float),
                margin=float(margin), w_coll=float(w_coll), penalty=float(penalty))


# ---- the five measured configurations ---------------------------------------

def config1() -> Problem:
    """T=50, K=16, sigma=0.05, 4 branch-offset candidates; seed-0 robot."""
    return make_problem(make_robot(0), seed=0, T=50, K=16, sigma=0.05, n_branch=4)


def config2() -> Problem:
    """T=300, K=256, sigma=0.1, 25% branch-offset candidates."""
    return make_problem(make_robot(0), seed=2, T=300, K=256, sigma=0.1,
                        branch_frac=0.25)


def config3() -> Problem:
    """T=1000, K=512, sigma=0.1, 25% branch-offset candidates."""
    return make_problem(make_robot(0), seed=3, T=1000, K=512, sigma=0.1,
                        branch_frac=0.25)


def config4_problem(i: int, T_range=(100, 1000), K_range=(64, 512)) -> Problem:
    """Problem i of the 64-problem ragged batch: fresh robot per problem."""
    seed = 4000 + i
    rng = np.random.default_rng([seed, 2])
    T = int(rng.integers(T_range[0], T_range[1] + 1))
    K = int(rng.integers(K_range[0], K_range[1] + 1))
    return make_problem(make_robot(seed), seed=seed, T=T, K=K, sigma=0.1,
                        branch_frac=0.25)


# The serving stream draws its candidate noise from one pool of float32
# standard normals (2^26 of them, 256 MB, drawn once per process): request i
# takes a contiguous run of K*T*n values at a seeded offset, so each request
# still sees i.i.d. N(0, sigma) noise, and a stream of thousands of distinct
# requests costs a few passes over float32 arrays each instead of fresh
# normal draws.
NOISE_POOL = 1 << 26


@functools.lru_cache(maxsize=1)
def _noise_pool() -> np.ndarray:
    return np.random.default_rng([5, 9]).standard_normal(NOISE_POOL, dtype=np.float32)


def config5_request(i: int, T_range=(50, 2000), K_choices=(128, 256, 512)) -> Problem:
    """Request i of the serving stream: seed-0 robot, per-request shape,
    noise level and branch fraction.  Draw order: rng = default_rng([5000 + i,
    2]): T ~ U{T_range}, K from K_choices, sigma ~ U[0.02, 0.15], frac ~ U[0,
    0.3], the pool offset ~ U{0 .. pool - K*T*n}, a permutation of K (the
    first round(frac*K) get the branch offset), one sign per (offset
    candidate, joint 2/4/6); the path q* as make_problem draws it (seed 5000 +
    i).  Candidates are computed in float32 (q* + sigma * noise, offsets,
    clamp) and returned as a float32 array [K][T][n]."""
    seed = 5000 + i
    rng = np.random.default_rng([seed, 2])
    T = int(rng.integers(T_range[0], T_range[1] + 1))
    K = int(rng.choice(np.array(K_choices)))
    sigma = float(rng.uniform(0.02, 0.15))
    frac = float(rng.uniform(0.0, 0.3))
    robot = make_robot(0)
    n = robot.dof
    q_star = _path(robot, seed, T)
    pool = _noise_pool()
    m = K * T * n
    if m > pool.shape[0]:
        raise ValueError("request larger than the noise pool")
    off = int(rng.integers(0, pool.shape[0] - m + 1))
    cand = pool[off:off + m].reshape(K, T, n) * np.float32(sigma)
    cand += q_star.astype(np.float32)[None, :, :]
    nb = int(round(frac * K))
    sel = rng.permutation(K)[:nb]
    signs = rng.choice(np.array([-1.0, 1.0]), (nb, len(BRANCH_JOINTS)))
    for c_i, j in enumerate(BRANCH_JOINTS):
        cand[sel, :, j] += (signs[:, c_i] * (math.pi / 2)).astype(np.float32)[:, None]
    np.clip(cand, robot.q_lo.astype(np.float32), robot.q_hi.astype(np.float32), out=cand)
    return Problem(robot=robot, q_star=q_star, cand=cand, targets=None, seed=seed, sigma=sigma,
                   branch_frac=float(nb) / K)


def config5_arrivals(rate_hz: float = 200.0, duration_s: float = 60.0,
                     seed: int = 5) -> np.ndarray:
    """Poisson arrival times (s) of the serving stream."""
    rng = np.random.default_rng([seed, 3])
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out)


def random_configs(seed: int, M: int, robot: Robot, spread: float = math.pi) -> np.ndarray:
    """M joint configurations ([M][n]) uniform in [-spread, spread] (a
    prismatic joint: uniform over its travel), float32-exact."""
    rng = np.random.default_rng([seed, 4])
    q = rng.uniform(-spread, spread, (M, robot.dof))
    pr = robot.prismatic()
    if pr.any():
        u = (q + spread) / (2.0 * spread)
        q = np.where(pr, robot.q_lo + (robot.q_hi - robot.q_lo) * u, q)
    return _f32(q)
