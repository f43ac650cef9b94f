"""Python binding of libcpf.so (the C ABI declared in include/cpf.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch is imported first so that the process has a single HIP
runtime (torch's), which the library then shares; torch tensors serve as
caller-owned device buffers for ``fk_batch``.  If the library has not been
built this module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
# CPF_LIB selects another build of the library (e.g. a diagnostic variant
# built with paper_2309_09102_amd/build.py -D ...); the default is the in-tree one.
LIB_PATH = os.environ.get("CPF_LIB") or os.path.join(_HERE, "libcpf.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                      "(or python paper_2309_09102_amd/build.py) first")
_lib = C.CDLL(LIB_PATH)

OK, PENDING = 0, 1
E_ARG, E_NOMEM, E_DEVICE, E_STATE, E_NOTFOUND, E_NUMERIC, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
MIXED, FP64 = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
RESEARCH_MJAC_RAD = 0.20943951023931953   # CPF_RESEARCH_MJAC_RAD: 12 degrees
RESEARCH_MJAC_M = 0.03                    # CPF_RESEARCH_MJAC_M: 3 cm (prismatic joints)
_NAMES = {0: "OK", 1: "PENDING", -1: "E_ARG", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_STATE",
          -5: "E_NOTFOUND", -6: "E_NUMERIC", -7: "E_UNSUPPORTED"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class CpfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class cpf_robot(C.Structure):
    _fields_ = [("dof", C.c_int32), ("a", _dp), ("d", _dp), ("alpha", _dp),
                ("theta_off", _dp), ("q_lo", _dp), ("q_hi", _dp), ("capsules", _dp),
                ("joint_type", _ip)]


class cpf_problem(C.Structure):
    _fields_ = [("T", C.c_int32), ("K", C.c_int32), ("targets", _dp), ("cand", _dp),
                ("node_pen", _dp), ("n_obstacles", C.c_int32), ("obstacles", _dp),
                ("cand_f32", C.POINTER(C.c_float)), ("mem", C.c_int32)]


class cpf_opts(C.Structure):
    _fields_ = [("w_pose", C.c_double), ("w_smooth", C.c_double), ("lambda0", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("limit_margin", C.c_double), ("limit_penalty", C.c_double),
                ("iters", C.c_int32), ("prec", C.c_int32), ("refine_steps", C.c_int32),
                ("schedule", C.c_int32), ("valid_pos_m", C.c_double),
                ("valid_rot_rad", C.c_double), ("valid_step_rad", C.c_double),
                ("coll_margin", C.c_double), ("w_coll", C.c_double), ("coll_penalty", C.c_double),
                ("limit_margin_m", C.c_double), ("valid_step_m", C.c_double)]


class cpf_lm_report(C.Structure):
    _fields_ = [("cost0", C.c_double), ("cost", C.c_double), ("lambda_", C.c_double),
                ("grad_inf", C.c_double), ("n_accepted", C.c_int32), ("iters_done", C.c_int32),
                ("max_pos_err_m", C.c_double), ("max_rot_err_rad", C.c_double),
                ("mjac", C.c_double), ("n_valid", C.c_int32), ("first_valid", C.c_int32),
                ("pose_steps", C.c_int32), ("diff_steps", C.c_int32),
                ("valid_length", C.c_double), ("min_self_dist_m", C.c_double),
                ("min_env_dist_m", C.c_double)]


class cpf_result(C.Structure):
    _fields_ = [("xi", _dp), ("path", _ip), ("report", cpf_lm_report),
                ("search_best", C.c_double), ("search_mjac", C.c_double),
                ("status", C.c_int32), ("t_submit_ns", C.c_int64), ("t_admit_ns", C.c_int64),
                ("t_search_done_ns", C.c_int64), ("t_done_ns", C.c_int64), ("xi_valid", _dp)]


_vp = C.c_void_p
_lib.cpf_opts_default.argtypes = [C.POINTER(cpf_opts)]
_lib.cpf_last_error.restype = C.c_char_p
_lib.cpf_ctx_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(_vp)]
_lib.cpf_ctx_destroy.argtypes = [_vp]
_lib.cpf_ctx_bytes_in_use.argtypes = [_vp]
_lib.cpf_ctx_bytes_in_use.restype = C.c_uint64
_lib.cpf_plan_init.argtypes = [_vp, C.POINTER(cpf_robot), C.POINTER(cpf_problem),
                               C.POINTER(cpf_opts), C.POINTER(_vp)]
_lib.cpf_plan_free.argtypes = [_vp]
_lib.cpf_fk_batch.argtypes = [_vp, C.POINTER(cpf_robot), C.c_int64, C.c_int32, _vp, _vp, _vp, _vp]
_lib.cpf_dp_search.argtypes = [_vp, _ip, _dp, _dp]
_lib.cpf_dp_seed_steps.argtypes = [_vp, _dp, _dp]
_lib.cpf_dp_needs_research.argtypes = [_vp, _ip]
_lib.cpf_dp_lists.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _dp]
_lib.cpf_lm_refine.argtypes = [_vp, C.c_int32, _dp, C.POINTER(cpf_lm_report)]
_lib.cpf_lm_latest_valid.argtypes = [_vp, _dp]
_lib.cpf_solve_static.argtypes = [_vp, C.POINTER(cpf_robot), C.POINTER(cpf_problem), C.POINTER(cpf_opts), _ip, _dp,
                                  _dp, C.POINTER(cpf_lm_report)]
_lib.cpf_plan_solve.argtypes = [_vp, _ip, _dp, _dp, C.POINTER(cpf_lm_report)]
_lib.cpf_plan_append.argtypes = [_vp, C.c_int32, _dp, _dp]
_lib.cpf_coll_batch.argtypes = [_vp, C.POINTER(cpf_robot), C.c_int32, _vp, C.c_int64, C.c_int32, _vp, _vp,
                                _vp, _vp]
_lib.cpf_solve_batch.argtypes = [_vp, C.c_int32, C.POINTER(cpf_robot), C.POINTER(cpf_problem),
                                 C.POINTER(cpf_opts), C.POINTER(cpf_result)]
_lib.cpf_batchopt.argtypes = [_vp, C.POINTER(cpf_robot), C.POINTER(cpf_problem), C.POINTER(cpf_opts),
                              C.c_int32, _ip, C.POINTER(cpf_result)]
_lib.cpf_submit.argtypes = [_vp, C.POINTER(cpf_robot), C.POINTER(cpf_problem),
                            C.POINTER(cpf_opts), C.POINTER(C.c_uint64)]
_lib.cpf_poll.argtypes = [_vp, C.c_uint64, C.c_int32, C.POINTER(cpf_result)]
_lib.cpf_ctx_config.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32]
_lib.cpf_ctx_profile.argtypes = [_vp, C.c_int32]
_lib.cpf_ctx_kernel_stats.argtypes = [_vp, C.c_char_p, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]
for _f in ("cpf_ctx_create", "cpf_plan_init", "cpf_fk_batch", "cpf_dp_search", "cpf_dp_seed_steps",
           "cpf_dp_needs_research", "cpf_dp_lists", "cpf_lm_refine",
           "cpf_lm_latest_valid", "cpf_plan_append", "cpf_coll_batch", "cpf_plan_solve",
           "cpf_solve_batch", "cpf_batchopt", "cpf_submit", "cpf_poll", "cpf_ctx_profile",
           "cpf_ctx_kernel_stats", "cpf_ctx_config", "cpf_solve_static"):
    getattr(_lib, _f).restype = C.c_int

EXPORTS = ("cpf_opts_default", "cpf_last_error", "cpf_ctx_create", "cpf_ctx_destroy",
           "cpf_ctx_bytes_in_use", "cpf_plan_init", "cpf_plan_free", "cpf_fk_batch", "cpf_coll_batch",
           "cpf_dp_search", "cpf_dp_seed_steps", "cpf_dp_needs_research", "cpf_dp_lists", "cpf_plan_append", "cpf_lm_refine", "cpf_plan_solve", "cpf_lm_latest_valid",
           "cpf_solve_batch", "cpf_batchopt", "cpf_submit", "cpf_poll", "cpf_ctx_profile",
           "cpf_ctx_kernel_stats", "cpf_ctx_config", "cpf_solve_static")


def last_error() -> str:
    return (_lib.cpf_last_error() or b"").decode()


def _check(st):
    if st not in (OK, PENDING):
        raise CpfError(st, last_error())
    return st


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class _Keep:
    """ctypes struct plus the numpy arrays its pointers refer to."""

    def __init__(self, struct, arrays):
        self.struct = struct
        self.arrays = arrays


def make_robot(robot, coll=None) -> _Keep:
    """coll: collision description (dict with capsules [dof][7], obstacles
    [n][18], margin, w_coll, penalty) or None.  The robot's joint_type
    attribute (0 revolute, 1 prismatic per joint), when present, is passed on."""
    arrs = [_f64(robot.a), _f64(robot.d), _f64(robot.alpha), _f64(robot.theta_off),
            _f64(robot.q_lo), _f64(robot.q_hi)]
    caps = None if coll is None else _f64(coll["capsules"])
    jt = getattr(robot, "joint_type", None)
    jt = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
    s = cpf_robot(int(arrs[0].shape[0]), *[_ptr(a) for a in arrs], _ptr(caps),
                  None if jt is None else jt.ctypes.data_as(_ip))
    return _Keep(s, arrs + [caps, jt])


def _obstacles(coll):
    if coll is None or coll.get("obstacles") is None:
        return None
    ob = _f64(coll["obstacles"]).reshape(-1, 18)
    return ob if ob.shape[0] else None


def _is_device_tensor(x) -> bool:
    return isinstance(x, torch.Tensor) and x.is_cuda


def _dof(robot) -> int:
    return int(np.asarray(robot.a).shape[0])


def make_problem(targets, cand, node_pen=None, coll=None, dof=None) -> _Keep:
    """cand: float64 [K][T][dof] (host), float32 [K][T][dof] (host, passed as
    cand_f32), or a contiguous float32 device tensor [K][T][dof] with targets a
    contiguous float64 device tensor [T][12] (device-resident inputs, read in
    place: keep both alive and unchanged until the call or request is done).
    dof: the robot's joint count, checked against the candidates' last axis."""
    if dof is not None and (len(cand.shape) != 3 or int(cand.shape[2]) != dof):
        raise ValueError(f"candidates must be [K][T][{dof}], got {tuple(cand.shape)}")
    npen = None if node_pen is None else _f64(node_pen)
    ob = _obstacles(coll)
    n_ob = 0 if ob is None else int(ob.shape[0])
    if _is_device_tensor(cand):
        if not (cand.dtype == torch.float32 and cand.dim() == 3 and cand.is_contiguous()):
            raise ValueError("device candidates must be a contiguous float32 tensor [K][T][dof]")
        if not (_is_device_tensor(targets) and targets.dtype == torch.float64 and targets.is_contiguous()
                and tuple(targets.shape) == (cand.shape[1], 12)):
            raise ValueError("device targets must be a contiguous float64 tensor [T][12]")
        K, T = int(cand.shape[0]), int(cand.shape[1])
        s = cpf_problem(T, K, C.cast(C.c_void_p(targets.data_ptr()), _dp), None, _ptr(npen), n_ob, _ptr(ob),
                        C.cast(C.c_void_p(cand.data_ptr()), C.POINTER(C.c_float)), MEM_DEVICE)
        return _Keep(s, [targets, cand, npen, ob])
    tg = _f64(targets)
    if isinstance(cand, np.ndarray) and cand.dtype == np.float32:
        cf = np.ascontiguousarray(cand)
        K, T = int(cf.shape[0]), int(cf.shape[1])
        s = cpf_problem(T, K, _ptr(tg), None, _ptr(npen), n_ob, _ptr(ob),
                        cf.ctypes.data_as(C.POINTER(C.c_float)), MEM_HOST)
        return _Keep(s, [tg, cf, npen, ob])
    cd = _f64(cand)
    K, T = int(cd.shape[0]), int(cd.shape[1])
    s = cpf_problem(T, K, _ptr(tg), _ptr(cd), _ptr(npen), n_ob, _ptr(ob), None, MEM_HOST)
    return _Keep(s, [tg, cd, npen, ob])


def _with_coll(opts, coll):
    """opts with the collision margin, weight and penalty of coll."""
    o = cpf_opts.from_buffer_copy(opts if opts is not None else opts_default())
    if coll is not None:
        o.coll_margin = float(coll.get("margin", o.coll_margin))
        o.w_coll = float(coll.get("w_coll", o.w_coll))
        o.coll_penalty = float(coll.get("penalty", o.coll_penalty))
    return o


def opts_default() -> cpf_opts:
    o = cpf_opts()
    _lib.cpf_opts_default(C.byref(o))
    return o


def make_opts(**kw) -> cpf_opts:
    o = opts_default()
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = {"mixed": MIXED, "fp64": FP64}[v]
        setattr(o, k, v)
    return o


def _finite_or_none(v):
    return v if math.isfinite(v) else None


def _report(r: cpf_lm_report) -> dict:
    return dict(cost0=r.cost0, cost=r.cost, lam=r.lambda_, grad_inf=r.grad_inf,
                n_accepted=r.n_accepted, iters_done=r.iters_done,
                max_pos_err_m=r.max_pos_err_m, max_rot_err_rad=r.max_rot_err_rad, mjac=r.mjac,
                n_valid=r.n_valid, first_valid=r.first_valid, pose_steps=r.pose_steps,
                diff_steps=r.diff_steps, valid_length=r.valid_length,
                min_self_dist_m=_finite_or_none(r.min_self_dist_m),
                min_env_dist_m=_finite_or_none(r.min_env_dist_m))


# ---- functions with the C ABI's names ---------------------------------------

def ctx_create(device: int = 0, budget_bytes: int = 0):
    h = _vp()
    _check(_lib.cpf_ctx_create(device, budget_bytes, C.byref(h)))
    return h


def ctx_destroy(ctx):
    _lib.cpf_ctx_destroy(ctx)


def ctx_bytes_in_use(ctx) -> int:
    return int(_lib.cpf_ctx_bytes_in_use(ctx))


def ctx_config(ctx, slots: int, iters_per_tick: int, tick_budget: int = 6000):
    _check(_lib.cpf_ctx_config(ctx, int(slots), int(iters_per_tick), int(tick_budget)))


def ctx_profile(ctx, enable: bool):
    _check(_lib.cpf_ctx_profile(ctx, 1 if enable else 0))


def ctx_kernel_stats(ctx, kernel: str):
    """(total ms, launches) of kernel 'fk' | 'dp_lists' | 'dp' | 'lm' | 'eval' since profiling began."""
    ms = C.c_double()
    n = C.c_int64()
    _check(_lib.cpf_ctx_kernel_stats(ctx, kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, int(n.value)


def plan_init(ctx, robot, targets, cand, node_pen=None, opts=None, coll=None):
    rb = make_robot(robot, coll)
    pb = make_problem(targets, cand, node_pen, coll, _dof(robot))
    o = _with_coll(opts, coll)
    h = _vp()
    _check(_lib.cpf_plan_init(ctx, C.byref(rb.struct), C.byref(pb.struct), C.byref(o), C.byref(h)))
    return h


def plan_free(plan):
    _lib.cpf_plan_free(plan)


def fk_batch(ctx, robot, M, prec, q_ptr, pose_ptr, jac_ptr=None, stream=None):
    """Device pointers (ints) in the SoA layout of include/cpf.h."""
    rb = make_robot(robot)
    _check(_lib.cpf_fk_batch(ctx, C.byref(rb.struct), int(M), int(prec), _vp(q_ptr),
                             _vp(pose_ptr), _vp(jac_ptr) if jac_ptr else None,
                             _vp(stream) if stream else None))


def coll_batch(ctx, robot, coll, M, prec, q_ptr, dist_ptr, grad_ptr=None, obstacles_ptr=None, n_obstacles=0,
               stream=None):
    """Device pointers (ints) in the SoA layout of include/cpf.h."""
    rb = make_robot(robot, coll)
    _check(_lib.cpf_coll_batch(ctx, C.byref(rb.struct), int(n_obstacles), _vp(obstacles_ptr) if obstacles_ptr else None,
                               int(M), int(prec), _vp(q_ptr), _vp(dist_ptr), _vp(grad_ptr) if grad_ptr else None,
                               _vp(stream) if stream else None))


def dp_search(plan, T: int):
    path = np.empty(T, dtype=np.int32)
    best = C.c_double()
    mj = C.c_double()
    _check(_lib.cpf_dp_search(plan, path.ctypes.data_as(_ip), C.byref(best), C.byref(mj)))
    return path, best.value, mj.value


def dp_needs_research(plan) -> bool:
    """The paper's test for more candidate plans after a search (Sec. III-B),
    decided by the library (cpf_dp_needs_research)."""
    v = C.c_int32()
    _check(_lib.cpf_dp_needs_research(plan, C.byref(v)))
    return bool(v.value)


def dp_seed_steps(plan):
    """(largest revolute step rad, largest prismatic step m) of the last search's seed."""
    r, p = C.c_double(), C.c_double()
    _check(_lib.cpf_dp_seed_steps(plan, C.byref(r), C.byref(p)))
    return r.value, p.value


TOPM = 16


def dp_lists(plan, K: int, t0: int, nt: int):
    """The search's predecessor lists of waypoints t0 .. t0 + nt - 1
    (cpf_dp_lists): indices [nt][K][TOPM] (uint16) and c = edge + node
    penalty [nt][K][TOPM]."""
    idx = np.empty((nt, K, TOPM), dtype=np.uint16)
    c = np.empty((nt, K, TOPM))
    _check(_lib.cpf_dp_lists(plan, int(t0), int(nt), idx.ctypes.data_as(_vp), _ptr(c)))
    return idx, c


def lm_refine(plan, iters: int, T: int, want_xi: bool = True, dof: int = 7):
    xi = np.empty((T, dof)) if want_xi else None
    rep = cpf_lm_report()
    st = _lib.cpf_lm_refine(plan, int(iters), _ptr(xi), C.byref(rep))
    if st != OK:
        raise CpfError(st, last_error())
    return xi, _report(rep)


def plan_append(plan, T: int, cand_add, node_pen_add=None, dof: int = 7):
    """Append candidates [K_add][T][dof] (and their node costs [T][K_add])."""
    cd = _f64(cand_add)
    if cd.ndim != 3 or cd.shape[1] != T or cd.shape[2] != dof:
        raise ValueError(f"cand_add must be [K_add][{T}][{dof}], got {cd.shape}")
    npen = None if node_pen_add is None else _f64(node_pen_add)
    if npen is not None and npen.shape != (T, cd.shape[0]):
        raise ValueError(f"node_pen_add must be [{T}][{cd.shape[0]}], got {npen.shape}")
    _check(_lib.cpf_plan_append(plan, int(cd.shape[0]), _ptr(cd), _ptr(npen)))


def plan_solve(plan, T: int, want_xi: bool = True, dof: int = 7):
    """Search + opts.iters LM iterations + report -> (path, B*, xi | None, report)."""
    path = np.empty(T, dtype=np.int32)
    best = C.c_double()
    xi = np.empty((T, dof)) if want_xi else None
    rep = cpf_lm_report()
    st = _lib.cpf_plan_solve(plan, path.ctypes.data_as(_ip), C.byref(best), _ptr(xi), C.byref(rep))
    if st != OK:
        raise CpfError(st, last_error())
    return path, best.value, xi, _report(rep)


def solve_static(ctx, robot, targets, cand, opts=None, node_pen=None, coll=None):
    """cpf_solve_static: search + opts.iters LM iterations + report in the
    library's static device scratch (no device allocation) -> (path, B*, xi,
    report)."""
    rb = make_robot(robot, coll)
    pb = make_problem(targets, cand, node_pen, coll, _dof(robot))
    o = _with_coll(opts, coll)
    T = pb.struct.T
    path = np.empty(T, dtype=np.int32)
    best = C.c_double()
    xi = np.empty((T, _dof(robot)))
    rep = cpf_lm_report()
    st = _lib.cpf_solve_static(ctx, C.byref(rb.struct), C.byref(pb.struct), C.byref(o), path.ctypes.data_as(_ip),
                               C.byref(best), _ptr(xi), C.byref(rep))
    if st != OK:
        raise CpfError(st, last_error())
    return path, best.value, xi, _report(rep)


def lm_latest_valid(plan, T: int, dof: int = 7):
    """Latest valid trajectory [T][dof] of a plan refined under the schedule
    (raises CpfError E_STATE when there is none yet or no schedule)."""
    xi = np.empty((T, dof))
    _check(_lib.cpf_lm_latest_valid(plan, _ptr(xi)))
    return xi


def solve_batch(ctx, problems, opts=None):
    """problems: list of (robot, targets, cand[, node_pen[, coll]]); the
    collision margin, weight and penalty of the first coll apply to the whole
    batch.  Returns list of dicts."""
    n = len(problems)
    keeps, robots, probs = [], (cpf_robot * n)(), (cpf_problem * n)()
    results = (cpf_result * n)()
    outs = []
    first_coll = next((pr[4] for pr in problems if len(pr) > 4 and pr[4] is not None), None)
    for i, pr in enumerate(problems):
        coll = pr[4] if len(pr) > 4 else None
        nj = _dof(pr[0])
        rb = make_robot(pr[0], coll)
        pb = make_problem(pr[1], pr[2], pr[3] if len(pr) > 3 else None, coll, nj)
        keeps += [rb, pb]
        robots[i] = rb.struct
        probs[i] = pb.struct
        T = pb.struct.T
        xi = np.empty((T, nj))
        path = np.empty(T, dtype=np.int32)
        xv = np.empty((T, nj))
        outs.append((xi, path, xv))
        results[i].xi = _ptr(xi)
        results[i].path = path.ctypes.data_as(_ip)
        results[i].xi_valid = _ptr(xv)
    o = _with_coll(opts, first_coll)
    _check(_lib.cpf_solve_batch(ctx, n, robots, probs, C.byref(o), results))
    return [_result(results[i], *outs[i]) for i in range(n)]


def batchopt(ctx, robot, targets, cand, M: int, opts=None, node_pen=None, coll=None):
    """The M smoothest candidates optimised directly.  Returns (indices,
    list of result dicts), in ascending candidate mjac."""
    nj = _dof(robot)
    rb = make_robot(robot, coll)
    pb = make_problem(targets, cand, node_pen, coll, nj)
    T = pb.struct.T
    idx = np.empty(max(M, 0), dtype=np.int32)
    results = (cpf_result * max(M, 1))()
    outs = []
    for i in range(M):
        xi = np.empty((T, nj))
        path = np.empty(T, dtype=np.int32)
        xv = np.empty((T, nj))
        outs.append((xi, path, xv))
        results[i].xi = _ptr(xi)
        results[i].path = path.ctypes.data_as(_ip)
        results[i].xi_valid = _ptr(xv)
    o = _with_coll(opts, coll)
    _check(_lib.cpf_batchopt(ctx, C.byref(rb.struct), C.byref(pb.struct), C.byref(o), M,
                             idx.ctypes.data_as(_ip), results))
    return [int(k) for k in idx], [_result(results[i], *outs[i]) for i in range(M)]


def _result(r: cpf_result, xi, path, xv=None) -> dict:
    rep = _report(r.report)
    return dict(xi=xi, path=path, report=rep, xi_valid=xv if rep["n_valid"] > 0 else None,
                search_best=r.search_best,
                search_mjac=r.search_mjac, status=r.status,
                t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns,
                t_search_done_ns=r.t_search_done_ns, t_done_ns=r.t_done_ns)


def submit(ctx, robot, targets, cand, opts=None, node_pen=None, coll=None) -> int:
    rb = make_robot(robot, coll)
    pb = make_problem(targets, cand, node_pen, coll, _dof(robot))
    o = _with_coll(opts, coll)
    t = C.c_uint64()
    _check(_lib.cpf_submit(ctx, C.byref(rb.struct), C.byref(pb.struct), C.byref(o), C.byref(t)))
    return int(t.value)


def poll(ctx, ticket: int, T: int, timeout_ms: int = -1, dof: int = 7):
    """Result dict, or None while the request is pending."""
    xi = np.empty((T, dof))
    path = np.empty(T, dtype=np.int32)
    xv = np.empty((T, dof))
    r = cpf_result()
    r.xi = _ptr(xi)
    r.path = path.ctypes.data_as(_ip)
    r.xi_valid = _ptr(xv)
    st = _check(_lib.cpf_poll(ctx, int(ticket), int(timeout_ms), C.byref(r)))
    if st == PENDING:
        return None
    return _result(r, xi, path, xv)


# ---- small object layer -------------------------------------------------------

class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self.h = ctx_create(device, budget_bytes)

    def close(self):
        if self.h:
            ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def bytes_in_use(self) -> int:
        return ctx_bytes_in_use(self.h)

    def config(self, slots: int = 256, iters_per_tick: int = 30, tick_budget: int = 6000):
        ctx_config(self.h, slots, iters_per_tick, tick_budget)

    def profile(self, enable: bool = True):
        ctx_profile(self.h, enable)

    def kernel_stats(self, kernel: str):
        return ctx_kernel_stats(self.h, kernel)

    def plan(self, robot, targets, cand, node_pen=None, opts=None, coll=None) -> "Plan":
        return Plan(self, plan_init(self.h, robot, targets, cand, node_pen, opts, coll),
                    int(cand.shape[1]), _dof(robot), int(cand.shape[0]))

    def coll_batch(self, robot, coll, q: "torch.Tensor", want_grad: bool = False, stream=None):
        """q: device tensor [dof][M] -> (dist [2][M], grad [2 dof][M] | None): the
        smallest self and environment capsule distances of each configuration."""
        nj = _dof(robot)
        assert q.is_cuda and q.dim() == 2 and q.shape[0] == nj and q.is_contiguous()
        prec = F64 if q.dtype == torch.float64 else F32
        M = q.shape[1]
        ob = _obstacles(coll)
        obt = None if ob is None else torch.tensor(ob, dtype=torch.float64, device=q.device)
        dist = torch.empty((2, M), dtype=q.dtype, device=q.device)
        grad = torch.empty((2 * nj, M), dtype=q.dtype, device=q.device) if want_grad else None
        s = stream if stream is not None else torch.cuda.current_stream(q.device).cuda_stream
        if obt is not None and stream is not None:
            torch.cuda.current_stream(q.device).synchronize()   # the obstacle upload is on torch's stream
        coll_batch(self.h, robot, coll, M, prec, q.data_ptr(), dist.data_ptr(),
                   grad.data_ptr() if grad is not None else None,
                   obt.data_ptr() if obt is not None else None, 0 if ob is None else ob.shape[0], s)
        if obt is not None and stream is not None:
            # the obstacle copy is freed by torch's allocator in the order of
            # its own stream; tell it about the kernel's stream
            obt.record_stream(torch.cuda.ExternalStream(stream))
        return dist, grad

    def fk_batch(self, robot, q: "torch.Tensor", want_jac: bool = False, stream=None):
        """q: device tensor [dof][M] (float32 or float64) -> (pose [12][M], J [6 dof][M] | None)."""
        nj = _dof(robot)
        assert q.is_cuda and q.dim() == 2 and q.shape[0] == nj and q.is_contiguous()
        prec = F64 if q.dtype == torch.float64 else F32
        M = q.shape[1]
        pose = torch.empty((12, M), dtype=q.dtype, device=q.device)
        jac = torch.empty((6 * nj, M), dtype=q.dtype, device=q.device) if want_jac else None
        s = stream if stream is not None else torch.cuda.current_stream(q.device).cuda_stream
        fk_batch(self.h, robot, M, prec, q.data_ptr(), pose.data_ptr(),
                 jac.data_ptr() if jac is not None else None, s)
        return pose, jac

    def solve_batch(self, problems, opts=None):
        return solve_batch(self.h, problems, opts)

    def batchopt(self, robot, targets, cand, M: int, opts=None, node_pen=None, coll=None):
        return batchopt(self.h, robot, targets, cand, M, opts, node_pen, coll)

    def solve_static(self, robot, targets, cand, opts=None, node_pen=None, coll=None):
        return solve_static(self.h, robot, targets, cand, opts, node_pen, coll)

    def submit(self, robot, targets, cand, opts=None, node_pen=None, coll=None) -> int:
        return submit(self.h, robot, targets, cand, opts, node_pen, coll)

    def poll(self, ticket: int, T: int, timeout_ms: int = -1, dof: int = 7):
        return poll(self.h, ticket, T, timeout_ms, dof)


class Plan:
    def __init__(self, ctx: Context, h, T: int, dof: int = 7, K: int = 0):
        self.ctx, self.h, self.T, self.dof, self.K = ctx, h, T, dof, K

    def dp_search(self):
        return dp_search(self.h, self.T)

    def seed_steps(self):
        return dp_seed_steps(self.h)

    def lists(self, t0: int = 1, nt: int | None = None):
        """Predecessor lists of waypoints t0 .. t0 + nt - 1 (default: to the end)."""
        nt = self.T - t0 if nt is None else nt
        return dp_lists(self.h, self.K, t0, nt)

    def needs_research(self) -> bool:
        """The paper's test for more candidate plans (Sec. III-B): a seed step
        above 12 degrees (revolute) or 3 cm (prismatic)."""
        return dp_needs_research(self.h)

    def lm_refine(self, iters: int, want_xi: bool = True):
        return lm_refine(self.h, iters, self.T, want_xi, self.dof)

    def latest_valid(self):
        return lm_latest_valid(self.h, self.T, self.dof)

    def solve(self, want_xi: bool = True):
        return plan_solve(self.h, self.T, want_xi, self.dof)

    def append(self, cand_add, node_pen_add=None):
        plan_append(self.h, self.T, cand_add, node_pen_add, self.dof)
        self.K += int(np.shape(cand_add)[0])

    def free(self):
        if self.h:
            plan_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
