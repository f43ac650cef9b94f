"""ctypes wrapper of the FP64 C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# LM options in the order the C side reads them.
DEFAULT_LM = dict(w_pose=1.0, w_smooth=0.1, lambda0=1e-3, lambda_min=1e-10,
                  lambda_max=1e10)
LIMIT_MARGIN = 1.5 * np.pi / 180.0
LIMIT_MARGIN_M = 0.03          # prismatic joints (Sec. III-B: 3 cm)
LIMIT_PENALTY = 10.0
# Collision residual margin (m), weight and search penalty (Sec. III-B: 100)
COLL_MARGIN = 0.02
COLL_WEIGHT = 1.0
COLL_PENALTY = 100.0

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if _LIB == os.path.join(_HERE, "liboracle.so") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.or_fk_many.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, C.c_long, _dp, _dp, _dp]
        lib.or_fk_many.restype = None
        lib.or_log_so3.argtypes = [_dp, _dp]
        lib.or_log_so3.restype = None
        lib.or_cost.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, C.c_int, _dp, _dp,
                                C.c_double, C.c_double, _dp]
        lib.or_cost.restype = C.c_double
        lib.or_dp.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_double, C.c_double,
                              C.c_double, _dp, _ip, _dp, _dp, _ip, _dp, _dp, _dp, _dp, _ip, _dp]
        lib.or_dp.restype = C.c_int
        lib.or_mjac.argtypes = [C.c_int, C.c_int, _dp]
        lib.or_mjac.restype = C.c_double
        lib.or_btd_solve.argtypes = [C.c_int, C.c_int, _dp, C.c_double, _dp, _dp]
        lib.or_btd_solve.restype = C.c_int
        lib.or_lm_step.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, C.c_int, _dp, _dp,
                                   C.c_double, C.c_double, C.c_double, _dp, _dp, _dp, C.c_double]
        lib.or_lm_step.restype = C.c_int
        lib.or_lm.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, _dp, _dp, C.c_int, _dp, _dp,
                              _dp, C.c_int, _dp, _dp, _ip, _dp, _dp]
        lib.or_lm.restype = C.c_int
        lib.or_plan.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, _dp, _dp, C.c_int, C.c_int,
                                _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp, C.c_int, _ip,
                                _dp, _dp, _dp, _dp]
        lib.or_plan.restype = C.c_int
        lib.or_pose_compare.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, C.c_int, _dp, _dp,
                                        _dp, _dp]
        lib.or_pose_compare.restype = None
        lib.or_lm_schedule.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, _dp, _dp, C.c_int, _dp, _dp, _dp,
                                       _dp, C.c_int, _dp, _dp, _dp]
        lib.or_coll_eval.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _ip, _dp, C.c_long, _dp, _dp, _dp]
        lib.or_coll_eval.restype = None
        lib.or_seg_seg.argtypes = [_dp, _dp, _dp, _dp, _dp]
        lib.or_seg_seg.restype = None
        lib.or_seg_box.argtypes = [_dp, _dp, _dp, _dp, _dp]
        lib.or_seg_box.restype = None
        lib.or_lm_schedule.restype = C.c_int
        _lib = lib
        return lib


def use_library(path):
    """Point this wrapper at another build of the oracle source (returns the
    previous handle).  Used by the mutation tests, which compile deliberately
    broken copies of the oracle to check that the pins catch them."""
    global _lib, _LIB
    prev = (_lib, _LIB)
    _lib, _LIB = None, path
    _load()
    return prev


def restore_library(prev):
    global _lib, _LIB
    _lib, _LIB = prev


def build_copy(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source to out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", out_path, src, "-lm"], check=True)
    return out_path


def _d(x):
    """Contiguous float64 array (kept alive by the caller) and its pointer."""
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(arr):
    return None if arr is None else arr.ctypes.data_as(_dp)


def _ipp(arr):
    return None if arr is None else arr.ctypes.data_as(_ip)


def joint_types(rb):
    """int32 [n]: 0 revolute, 1 prismatic (all revolute when the robot has no
    joint_type)."""
    jt = getattr(rb, "joint_type", None)
    n = np.asarray(rb.a).shape[0]
    return np.zeros(n, dtype=np.int32) if jt is None else np.ascontiguousarray(jt, dtype=np.int32)


def _robot(rb):
    return [_d(rb.a), _d(rb.d), _d(rb.alpha), _d(rb.theta_off), joint_types(rb), _d(rb.q_lo), _d(rb.q_hi)]


def fk(robot, q, jacobian: bool = False):
    """q [..., n] -> pose [..., 12] (x, y, z, R row-major) and J [..., 6, n]."""
    lib = _load()
    n = robot.a.shape[0]
    q = _d(q)
    shape = q.shape[:-1]
    M = int(np.prod(shape)) if shape else 1
    a, d, al, th, jt, _, _ = _robot(robot)
    pose = np.empty((M, 12))
    J = np.empty((M, 6, n)) if jacobian else None
    lib.or_fk_many(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), M, _p(q), _p(pose), _p(J))
    pose = pose.reshape(shape + (12,))
    if jacobian:
        return pose, J.reshape(shape + (6, n))
    return pose


def log_so3(R):
    lib = _load()
    R = _d(R).reshape(9)
    out = np.empty(3)
    lib.or_log_so3(_p(R), _p(out))
    return out


def coll_spec(n, coll):
    """Flat collision description for the C oracle, or None.  coll: dict with
    capsules [n][7] (p0 xyz, p1 xyz in the frame after the link, radius),
    obstacles [m][18] (frame origin xyz, rotation row-major, p_min xyz, p_max
    xyz), margin, w_coll, penalty."""
    if coll is None:
        return None
    caps = _d(coll["capsules"]).reshape(n, 7)
    obs = _d(coll.get("obstacles", np.zeros((0, 18)))).reshape(-1, 18)
    head = [coll.get("margin", COLL_MARGIN), coll.get("w_coll", COLL_WEIGHT),
            coll.get("penalty", COLL_PENALTY), float(obs.shape[0])]
    return _d(np.concatenate([head, caps.ravel(), obs.ravel()]))


def seg_seg(P0, P1, Q0, Q1):
    """Robot-robot QP: (squared distance, s, t) of two segments."""
    lib = _load()
    out = np.empty(3)
    lib.or_seg_seg(_p(_d(P0)), _p(_d(P1)), _p(_d(Q0)), _p(_d(Q1)), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def seg_box(A, D, pmin, pmax):
    """Robot-environment QP in the cuboid frame: (squared distance, s) of
    the segment A + s D to the box [pmin, pmax]."""
    lib = _load()
    out = np.empty(3)
    lib.or_seg_box(_p(_d(A)), _p(_d(D)), _p(_d(pmin)), _p(_d(pmax)), _p(out))
    return float(out[0]), float(out[1])


def coll_eval(robot, coll, q, gradient: bool = False):
    """q [..., n] -> distances [..., 2] (self, environment) and optionally
    their gradients [..., 2, n]."""
    lib = _load()
    n = robot.a.shape[0]
    q = _d(q)
    shape = q.shape[:-1]
    M = int(np.prod(shape)) if shape else 1
    a, d, al, th, jt, _, _ = _robot(robot)
    spec = coll_spec(n, coll)
    out = np.empty((M, 2))
    g = np.empty((M, 2, n)) if gradient else None
    lib.or_coll_eval(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), _p(spec), M, _p(q), _p(out), _p(g))
    out = out.reshape(shape + (2,))
    return (out, g.reshape(shape + (2, n))) if gradient else out


def cost(robot, xi, targets, w_pose=1.0, w_smooth=0.1, coll=None) -> float:
    lib = _load()
    xi = _d(xi)
    tg = _d(targets)
    T, n = xi.shape
    a, d, al, th, jt, _, _ = _robot(robot)
    spec = coll_spec(n, coll)
    return float(lib.or_cost(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), T, _p(xi), _p(tg),
                             w_pose, w_smooth, _p(spec)))


def dp(cand, robot, margin=LIMIT_MARGIN, penalty=LIMIT_PENALTY, extra=None,
       want_tables: bool = False, coll=None, margin_m=LIMIT_MARGIN_M):
    """cand [K][T][n] -> (path[T] int32, B*, B_all[T][K] | None, bp_all | None)."""
    lib = _load()
    cand = _d(cand)
    K, T, n = cand.shape
    lo, hi = _d(robot.q_lo), _d(robot.q_hi)
    ex = None if extra is None else _d(extra).reshape(T, K)
    path = np.empty(T, dtype=np.int32)
    best = np.empty(1)
    B_all = np.empty((T, K)) if want_tables else None
    bp_all = np.empty((T, K), dtype=np.int32) if want_tables else None
    a, d, al, th, jt, _, _ = _robot(robot)
    spec = coll_spec(n, coll)
    rc = lib.or_dp(T, K, n, _p(cand), _p(lo), _p(hi), margin, margin_m, penalty, _p(ex),
                   _ipp(path), _p(best), _p(B_all), _ipp(bp_all), _p(a), _p(d), _p(al), _p(th),
                   _ipp(jt), _p(spec))
    if rc != 0:
        raise RuntimeError(f"or_dp failed ({rc})")
    return path, float(best[0]), B_all, bp_all


def seed_steps(xi, robot):
    """(largest revolute step, largest prismatic step) between consecutive
    waypoints of xi [T][n] (0 for a joint type the robot lacks): the two
    quantities of Sec. III-B's re-search test (12 degrees / 3 cm)."""
    xi = _d(xi)
    jt = joint_types(robot)
    st = np.abs(np.diff(xi, axis=0)) if xi.shape[0] > 1 else np.zeros((0, xi.shape[1]))
    rev = st[:, jt == 0]
    pri = st[:, jt == 1]
    return (float(rev.max()) if rev.size else 0.0, float(pri.max()) if pri.size else 0.0)


def mjac(xi) -> float:
    lib = _load()
    xi = _d(xi)
    T, n = xi.shape
    return float(lib.or_mjac(T, n, _p(xi)))


def btd_solve(D, w, b):
    """Solve blocktridiag(-w I, D_t, -w I) x = b; D [T][n][n], b [T][n]."""
    lib = _load()
    D = _d(D)
    b = _d(b)
    T, n = b.shape
    x = np.empty((T, n))
    rc = lib.or_btd_solve(T, n, _p(D), float(w), _p(b), _p(x))
    if rc != 0:
        raise np.linalg.LinAlgError(f"or_btd_solve failed ({rc})")
    return x


def lm_step(robot, xi, targets, w_pose, w_smooth, lam, coll=None, w_coll=0.0):
    """One damped Gauss-Newton step at xi -> (delta [T][n], g [T][n]); with
    collision geometry the collision residuals enter with weight w_coll."""
    lib = _load()
    xi = _d(xi)
    tg = _d(targets)
    T, n = xi.shape
    a, d, al, th, jt, _, _ = _robot(robot)
    delta = np.empty((T, n))
    g = np.empty((T, n))
    spec = coll_spec(n, coll)
    rc = lib.or_lm_step(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), T, _p(xi), _p(tg),
                        w_pose, w_smooth, lam, _p(delta), _p(g), _p(spec), float(w_coll))
    if rc != 0:
        raise np.linalg.LinAlgError(f"or_lm_step failed ({rc})")
    return delta, g


def _opts5(opts):
    o = dict(DEFAULT_LM)
    if opts:
        o.update({k: v for k, v in opts.items() if k in o})
    return _d([o["w_pose"], o["w_smooth"], o["lambda0"], o["lambda_min"], o["lambda_max"]])


def lm(robot, xi0, targets, iters, opts=None, coll=None):
    """LM from xi0 -> dict(xi, cost_hist, lambda_hist, accepted, cost0, rc)."""
    lib = _load()
    xi = _d(xi0).copy()
    tg = _d(targets)
    T, n = xi.shape
    a, d, al, th, jt, lo, hi = _robot(robot)
    o5 = _opts5(opts)
    ch = np.empty(max(iters, 1))
    lh = np.empty(max(iters, 1))
    ah = np.empty(max(iters, 1), dtype=np.int32)
    c0 = np.empty(1)
    spec = coll_spec(n, coll)
    rc = lib.or_lm(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), _p(lo), _p(hi), T, _p(xi), _p(tg),
                   _p(o5), int(iters), _p(ch), _p(lh), _ipp(ah), _p(c0), _p(spec))
    return dict(xi=xi, cost_hist=ch[:iters], lambda_hist=lh[:iters],
                accepted=ah[:iters].astype(bool), cost0=float(c0[0]), rc=int(rc))


def plan(robot, cand, targets, iters, opts=None, extra=None, margin=LIMIT_MARGIN,
         penalty=LIMIT_PENALTY, coll=None, margin_m=LIMIT_MARGIN_M):
    """Search then LM -> dict(path, best, xi, cost, rc).  Releases the GIL."""
    lib = _load()
    cand = _d(cand)
    tg = _d(targets)
    K, T, n = cand.shape
    a, d, al, th, jt, lo, hi = _robot(robot)
    ex = None if extra is None else _d(extra).reshape(T, K)
    o5 = _opts5(opts)
    path = np.empty(T, dtype=np.int32)
    best = np.empty(1)
    xi = np.empty((T, n))
    cst = np.empty(1)
    spec = coll_spec(n, coll)
    rc = lib.or_plan(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), _p(lo), _p(hi), T, K, _p(cand),
                     _p(tg), _p(ex), margin, margin_m, penalty, _p(o5), int(iters), _ipp(path),
                     _p(best), _p(xi), _p(cst), _p(spec))
    return dict(path=path, best=float(best[0]), xi=xi, cost=float(cst[0]), rc=int(rc))


# Validity thresholds of Sec. II: 0.1 mm position, 0.1 degree rotation, and
# at most 7 degrees of change of a revolute joint (2 cm of a prismatic one)
# between waypoints.
VALID_TOL = (1e-4, np.deg2rad(0.1), np.deg2rad(7.0), 0.02)


def lm_schedule(robot, xi0, targets, iters, opts=None, tol=VALID_TOL, coll=None):
    """Pose-first alternating LM with the latest-valid store (see
    or_lm_schedule).  Returns dict(xi, xi_valid | None, n_valid, first_valid,
    valid_length, pose_steps, diff_steps, rc)."""
    lib = _load()
    xi = _d(xi0).copy()
    T, n = xi.shape
    tg = _d(targets)
    a, d, al, th, jt, lo, hi = _robot(robot)
    xv = np.zeros((T, n))
    info = np.zeros(5)
    spec = coll_spec(n, coll)
    tol = tuple(tol) + VALID_TOL[len(tol):]
    rc = lib.or_lm_schedule(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), _p(lo), _p(hi), T, _p(xi), _p(tg),
                            _p(_opts5(opts)), _p(_d(tol)), int(iters), _p(xv), _p(info), _p(spec))
    return dict(xi=xi, xi_valid=xv if info[0] > 0 else None, n_valid=int(info[0]),
                first_valid=int(info[1]), valid_length=float(info[2]), pose_steps=int(info[3]),
                diff_steps=int(info[4]), rc=int(rc))


def batchopt(robot, cand, targets, M, iters, opts=None):
    """Optimise the M smoothest candidate plans directly, without the search
    (the paper's "BatchOpt" planner, described in a comment next to its list
    of planners): the candidates with the least mjac (Sec. III-B's maximum
    joint change between consecutive waypoints), ties to the lower index,
    each clamped and refined by `iters` LM iterations on its own.  Returns
    (indices [M], list of plan() results)."""
    cand = _d(cand)
    K = cand.shape[0]
    m = [mjac(cand[k]) for k in range(K)]
    order = sorted(range(K), key=lambda k: (m[k], k))[:M]
    return order, [plan(robot, cand[k:k + 1], targets, iters, opts) for k in order]


def pose_compare(robot, xi_a, xi_b=None, targets=None):
    """(max position difference m, max rotation angle rad) under oracle FK."""
    lib = _load()
    xa = _d(xi_a)
    T, n = xa.shape
    xb = None if xi_b is None else _d(xi_b)
    tg = None if targets is None else _d(targets)
    if xb is None and tg is None:
        raise ValueError("need xi_b or targets")
    a, d, al, th, jt, _, _ = _robot(robot)
    out = np.empty(2)
    lib.or_pose_compare(n, _p(a), _p(d), _p(al), _p(th), _ipp(jt), T, _p(xa), _p(xb), _p(tg), _p(out))
    return float(out[0]), float(out[1])
