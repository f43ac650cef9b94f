/*
 * cpf.h -- C ABI of the MI355X (gfx950) refinement path of CppFlow
 * (arXiv 2309.09102): batched forward kinematics, the layered-graph search
 * over candidate plans, and Levenberg-Marquardt trajectory optimisation,
 * plus a continuously batched request server.
 *
 * Problem (Sec. II): given a redundant serial robot with forward kinematics
 * FK : R^n -> SE(3) and a target path Y = [y_0 .. y_{T-1}] of T poses, find
 * a joint trajectory xi = [q_0 .. q_{T-1}] whose end effector follows Y.
 * The caller supplies K approximate candidate plans (the role of the
 * generative IK model in Sec. III-A); the library picks one candidate per
 * waypoint minimising the maximum joint-angle change (Sec. III-B) and then
 * refines the result with damped least squares on pose and differencing
 * residuals, clamped to the joint limits (Sec. III-C).
 *
 * Conventions
 *   - n = dof = 7 or 8 joints (an 8-joint chain such as the Fetch.Full
 *     robot's prismatic torso lift ahead of a 7-joint arm, Sec. IV),
 *     standard (distal) Denavit-Hartenberg:
 *     A_i = Rz(q_i + theta_off_i) Tz(d_i) Tx(a_i) Rx(alpha_i) for a revolute
 *     joint, Rz(theta_off_i) Tz(d_i + q_i) Tx(a_i) Rx(alpha_i) for a
 *     prismatic one (cpf_robot.joint_type), no base or tool transform.
 *     Other dof values return CPF_E_UNSUPPORTED.
 *   - Threads: calls on one context may come from several threads (its
 *     arena pool and profiling records are locked; plan calls queue on the
 *     context's stream and so run one after another); a plan is used by one
 *     thread at a time; cpf_submit / cpf_poll may be called from any thread.
 *   - A pose is 12 doubles: x, y, z, then the 3x3 rotation row-major.
 *   - Host arrays are C-contiguous float64 unless stated otherwise.
 *   - Every function is exception-free; a non-OK status leaves outputs
 *     untouched and sets a per-thread message readable by cpf_last_error().
 *   - Candidate and target values are used as given; the library does not
 *     round them.  (Float32-representable inputs make the search decisions
 *     independent of the precision the candidates are stored in on device.)
 *
 * Status codes
 *   CPF_OK           success
 *   CPF_PENDING      (cpf_poll) the request is not finished yet
 *   CPF_E_ARG        null pointer, bad size, non-finite input
 *   CPF_E_NOMEM      device allocation failed or the request exceeds the
 *                    context's whole memory budget
 *   CPF_E_DEVICE     a HIP runtime error
 *   CPF_E_STATE      call out of order (e.g. lm_refine before dp_search)
 *   CPF_E_NOTFOUND   unknown ticket
 *   CPF_E_NUMERIC    non-finite cost or a non-positive pivot in the solve
 *   CPF_E_UNSUPPORTED a shape the kernels are not built for (dof other than
 *                    7 or 8, K > 1024)
 */
#ifndef CPF_H
#define CPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cpf_status {
    CPF_OK = 0,
    CPF_PENDING = 1,
    CPF_E_ARG = -1,
    CPF_E_NOMEM = -2,
    CPF_E_DEVICE = -3,
    CPF_E_STATE = -4,
    CPF_E_NOTFOUND = -5,
    CPF_E_NUMERIC = -6,
    CPF_E_UNSUPPORTED = -7
} cpf_status;

/* Arithmetic of the LM iteration (Sec. III-C).  Residuals, the cost and its
 * accept test, the gradient J^T r, the Gram J^T J, the block solve and its
 * FP64 refinement, and the validity checks are FP64 in both; CPF_MIXED
 * computes the kinematic Jacobian J from an FP32 chain, CPF_FP64 from an
 * FP64 one.  (The Jacobian only shapes the step; the FP64 residual fixes the
 * point the iteration converges to.)  CPF_F32 / CPF_F64 select
 * cpf_fk_batch's precision. */
enum { CPF_F32 = 0, CPF_F64 = 1 };
enum { CPF_MIXED = 0, CPF_FP64 = 1 };

typedef struct cpf_ctx cpf_ctx;
typedef struct cpf_plan cpf_plan;

/* Robot: dof rows of standard DH parameters and joint limits (host, copied).
 * capsules [dof][7] or NULL: the collision capsule of each link (Sec. II
 * collision avoidance): segment end points p0, p1 (xyz, metres) in the frame
 * after the link, then the radius.  With capsules the search adds
 * opts.coll_penalty to a configuration in collision (Sec. III-B) and the LM
 * adds the collision residuals (Sec. III-C); pairs of links fewer than three
 * apart in the chain are not checked.
 * joint_type [dof] or NULL (all revolute): 0 revolute, 1 prismatic (the
 * torso lift of the paper's Fetch.Full chain, Sec. IV).  A revolute joint's
 * value (rad) adds to theta_off, a prismatic joint's (m) to d, which is then
 * the link's offset at zero extension; its Jacobian column is [z; 0].  Limit
 * margins, validity steps and the re-search threshold take the prismatic
 * values (opts.limit_margin_m, opts.valid_step_m, CPF_RESEARCH_MJAC_M) for
 * prismatic joints; the search's edge cost and mjac take every joint's change
 * in its own unit (Sec. III-B).  A robot with capsules and a prismatic joint
 * is accepted by cpf_fk_batch and cpf_coll_batch only: plans (cpf_plan_init,
 * cpf_solve_batch, cpf_batchopt, cpf_submit) return CPF_E_UNSUPPORTED for it. */
typedef struct cpf_robot {
    int32_t dof;
    const double *a, *d, *alpha, *theta_off; /* theta_off may be NULL (zeros) */
    const double *q_lo, *q_hi;
    const double *capsules;
    const int32_t *joint_type;
} cpf_robot;

/* One problem.
 *   targets  [T][12]   target poses Y (Sec. II)
 *   cand     [K][T][dof] candidate plans (Sec. III-A), float64
 *   node_pen [T][K] or NULL: extra per-node search cost added to the
 *            joint-limit penalty (the paper's collision cost, Sec. III-B)
 *   cand_f32 [K][T][dof] float32 candidates, or NULL: used in place of cand
 *            (which may then be NULL); half the bytes to copy, the same
 *            search and refinement whenever the candidates are float32
 *            values (the device keeps candidates as float32 either way)
 *   mem      where targets and the candidates live:
 *            CPF_MEM_HOST   host arrays, copied before the call returns;
 *            CPF_MEM_DEVICE device pointers on the context's device, read
 *                           in place with no host copy; the candidates must
 *                           be cand_f32 (cand is ignored).  cpf_plan_init,
 *                           cpf_solve_batch and cpf_batchopt read them
 *                           before they return; cpf_submit reads them when
 *                           the server admits the request, so the caller
 *                           keeps them allocated and unchanged until
 *                           cpf_poll has returned the result.  The host
 *                           cannot check device values: a non-finite one is
 *                           read as 0 and the call (cpf_plan_init), the
 *                           plan's result (cpf_solve_batch, cpf_batchopt) or
 *                           the request (cpf_submit) ends with CPF_E_ARG.
 *            node_pen and obstacles are host arrays in both cases. */
enum { CPF_MEM_HOST = 0, CPF_MEM_DEVICE = 1 };
typedef struct cpf_problem {
    int32_t T, K;
    const double *targets;
    const double *cand;
    const double *node_pen;
    /* cuboid obstacles [n_obstacles][18] (used with robot capsules): frame
     * origin xyz, rotation row-major (columns = the cuboid's axes), p_min xyz,
     * p_max xyz in that frame (Sec. III-C); n_obstacles <= 64 */
    int32_t n_obstacles;
    const double *obstacles;
    const float *cand_f32;
    int32_t mem;
} cpf_problem;

/* Options (cpf_opts_default fills the defaults shown).
 *   w_pose 1, w_smooth 0.1: cost C = w_pose/2 sum_t |r_pose,t|^2
 *                           + w_smooth/2 sum_t |q_{t+1} - q_t|^2 (Sec. III-C)
 *   lambda0 1e-3, lambda_min 1e-10, lambda_max 1e10: Levenberg damping and
 *     its bounds; updated by Nielsen's gain-ratio rule
 *   limit_margin 1.5 deg, limit_penalty 10: joint-limit search penalty
 *     (Sec. III-B)
 *   iters: LM iterations run by cpf_submit / cpf_plan_solve
 *   prec: CPF_MIXED or CPF_FP64
 *   refine_steps 1: FP64 iterative-refinement steps after each solve
 *   schedule 0: 1 runs the alternating objective with anytime validity
 *     (Sec. III-C): before every iteration, and once after the last one of a
 *     call, the trajectory is checked in FP64 against the validity thresholds
 *     valid_pos_m 1e-4 (m), valid_rot_rad 0.1 deg and valid_step_rad 7 deg
 *     (largest joint change between consecutive waypoints; Sec. II); one that
 *     passes is kept as the latest valid trajectory.  A trajectory within the
 *     pose thresholds then takes an LM step on the differencing term alone
 *     (weight w_smooth), any other a step on the pose term alone (weight
 *     w_pose).  The pose steps' damping follows the gain-ratio rule; the
 *     differencing steps keep lambda0.
 *   coll_margin 0.02 m, w_coll 1, coll_penalty 100 (robots with capsules):
 *     collision residuals max(0, coll_margin - d) of the smallest self and
 *     environment distances d of every waypoint, weight w_coll in the cost
 *     (w_coll/2 sum r^2; in the schedule they belong to the differencing
 *     step), and the search penalty of a configuration with d < 0.
 *   limit_margin_m 0.03, valid_step_m 0.02: the joint-limit margin (Sec.
 *     III-B) and the validity step threshold (Sec. II) of prismatic joints,
 *     in metres. */
typedef struct cpf_opts {
    double w_pose, w_smooth;
    double lambda0, lambda_min, lambda_max;
    double limit_margin, limit_penalty;
    int32_t iters, prec, refine_steps;
    int32_t schedule;
    double valid_pos_m, valid_rot_rad, valid_step_rad;
    double coll_margin, w_coll, coll_penalty;
    double limit_margin_m, valid_step_m;
} cpf_opts;

typedef struct cpf_lm_report {
    double cost0;            /* cost of the clamped seed */
    double cost;             /* cost after the last iteration */
    double lambda;           /* current damping */
    double grad_inf;         /* max |g| at the last linearisation */
    int32_t n_accepted;      /* accepted iterations so far */
    int32_t iters_done;      /* iterations so far (resumable) */
    double max_pos_err_m;    /* max_t |p(q_t) - p*_t| (FP64 FK) */
    double max_rot_err_rad;  /* max_t angle(R(q_t) R*_t^T) (FP64 FK) */
    double mjac;             /* max joint change along the result */
    /* schedule mode only (zero / -1 otherwise): */
    int32_t n_valid;         /* validity checks passed */
    int32_t first_valid;     /* iteration before which the first check passed
                                (iters_done: after the last), -1 if none */
    int32_t pose_steps;      /* steps taken on the pose objective */
    int32_t diff_steps;      /* steps taken on the differencing objective */
    double valid_length;     /* sum over steps and joints of |change| along the
                                latest valid trajectory */
    double min_self_dist_m;  /* smallest capsule self distance along the result
                                (+inf without capsules) */
    double min_env_dist_m;   /* smallest capsule-obstacle distance (+inf
                                without capsules or obstacles) */
} cpf_lm_report;

typedef struct cpf_result {
    double *xi;              /* [T][dof] caller buffer, or NULL */
    int32_t *path;           /* [T] caller buffer, or NULL */
    cpf_lm_report report;
    double search_best;      /* optimal search value B* */
    double search_mjac;      /* mjac of the searched seed */
    int32_t status;          /* per-request cpf_status */
    int64_t t_submit_ns, t_admit_ns, t_search_done_ns, t_done_ns; /* steady clock */
    double *xi_valid;        /* [T][dof] caller buffer, or NULL: schedule mode's
                                latest valid trajectory, written when
                                report.n_valid > 0 (left untouched otherwise) */
} cpf_result;

void cpf_opts_default(cpf_opts *o);

/* Per-thread message of the last failed call on this thread. */
const char *cpf_last_error(void);

/* Context on HIP device `device` with a device-memory budget in bytes for
 * plans and requests (0 = 64 GiB).  Owns its streams and server thread. */
cpf_status cpf_ctx_create(int device, uint64_t mem_budget_bytes, cpf_ctx **out);
/* Finishes in-flight requests (their tickets resolve), then frees all. */
void cpf_ctx_destroy(cpf_ctx *ctx);
/* Budget bytes currently reserved by live plans and admitted requests. */
uint64_t cpf_ctx_bytes_in_use(const cpf_ctx *ctx);

/* Copy one problem to the device (candidates as float32, SoA).  Inputs are
 * copied before return.  Sec. II (problem), Sec. III-A (candidates). */
cpf_status cpf_plan_init(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                         const cpf_opts *opts, cpf_plan **out);
void cpf_plan_free(cpf_plan *plan);

/* Batched forward kinematics and geometric Jacobian (Sec. II; the kinematic
 * Jacobian of Sec. III-C).  Device pointers owned by the caller, SoA:
 *   q_dev    [dof][M]      joint values
 *   pose_dev [12][M]       x, y, z, R row-major
 *   jac_dev  [6*dof][M] or NULL; element (row, j) of the 6 x dof Jacobian
 *            (rows vx, vy, vz, wx, wy, wz) at index (row*dof + j)*M + m
 * prec selects float (CPF_F32) or double (CPF_F64) for all three arrays.
 * Asynchronous on hip_stream (a hipStream_t, NULL = default stream); only
 * argument errors are reported synchronously. */
cpf_status cpf_fk_batch(cpf_ctx *ctx, const cpf_robot *robot, int64_t M, int32_t prec,
                        const void *q_dev, void *pose_dev, void *jac_dev, void *hip_stream);

/* Batched collision distances (the collision checker of Sec. III-B; the
 * distance QPs of Sec. III-C) of M configurations of a robot with capsules.
 * Device pointers owned by the caller, SoA:
 *   obstacles_dev [n_obstacles][18] double (layout of cpf_problem), or NULL
 *                 when n_obstacles is 0
 *   q_dev         [dof][M]   joint values
 *   dist_dev      [2][M]     smallest self distance, smallest capsule-obstacle
 *                            distance (metres; < 0 in collision; +inf when
 *                            nothing is checked)
 *   grad_dev      [2*dof][M] or NULL: their gradients, row h*dof + j
 * prec selects float or double for q, dist and grad.  Asynchronous on
 * hip_stream; only argument errors are reported synchronously
 * (CPF_E_ARG without capsules). */
cpf_status cpf_coll_batch(cpf_ctx *ctx, const cpf_robot *robot, int32_t n_obstacles,
                          const double *obstacles_dev, int64_t M, int32_t prec, const void *q_dev,
                          void *dist_dev, void *grad_dev, void *hip_stream);

/* Layered-graph search (Sec. III-B): node (t, k) is candidate k at waypoint
 * t; B_0(k) = pen_0(k), B_t(k) = min_k' max(B_{t-1}(k'), e_t(k',k) +
 * pen_t(k)) with e_t = max_j |q_t^k[j] - q_{t-1}^k'[j]| and pen the
 * joint-limit penalty plus node_pen.  Ties go to the smallest (value, e,
 * k'); the end node is the smallest (B_{T-1}(k), k).  Writes path[T], B*
 * and the mjac of the chosen seed; stores the seed in the plan.
 * Synchronous. */
cpf_status cpf_dp_search(cpf_plan *plan, int32_t *path_out, double *best_out,
                         double *mjac_out);

/* Seed mjac above which the paper generates more candidate plans and
 * searches again (12 degrees, Sec. III-B); compare with cpf_dp_search's
 * mjac_out (a robot with prismatic joints: with cpf_dp_seed_steps'
 * rev_rad_out). */
#define CPF_RESEARCH_MJAC_RAD 0.20943951023931953
/* The same threshold for prismatic joints (3 cm, Sec. III-B); compare with
 * cpf_dp_seed_steps' pri_m_out. */
#define CPF_RESEARCH_MJAC_M 0.03

/* The paper's test for more candidate plans after a search (Sec. III-B):
 * *out = 1 when the seed of the plan's last search changes a revolute joint
 * by more than CPF_RESEARCH_MJAC_RAD or a prismatic joint by more than
 * CPF_RESEARCH_MJAC_M between consecutive waypoints, else 0.  The caller
 * then appends candidates (cpf_plan_append) and searches again.  Reads
 * values kept on the host by the search: no device work.  CPF_E_STATE before
 * the first search. */
cpf_status cpf_dp_needs_research(const cpf_plan *plan, int32_t *out);

/* Largest change of a revolute joint (rad) and of a prismatic joint (m)
 * between consecutive waypoints of the seed found by the plan's last search
 * (cpf_dp_search or cpf_plan_solve); 0 for a joint type the robot lacks.
 * mjac_out of the search is the larger of the two.  The paper searches again
 * with more candidate plans when either exceeds its threshold (Sec. III-B).
 * Reads values kept on the host by the search: no device work.  CPF_E_STATE
 * before the first search. */
cpf_status cpf_dp_seed_steps(const cpf_plan *plan, double *rev_rad_out, double *pri_m_out);

/* The pruned predecessor lists the search decides its stages with
 * (Sec. III-B's recursion, exact by construction): for node (t, k), the
 * CPF_TOPM predecessors k' with the smallest (e_t(k', k), k') in that order,
 * e_t as in cpf_dp_search (exact FP64), each with c = e_t(k', k) + pen_t(k).
 * Copies the lists of waypoints t0 .. t0 + nt - 1 (1 <= t0, t0 + nt <= T)
 * to caller host buffers, node-major:
 *   idx_out [nt][K][CPF_TOPM] predecessor indices (or NULL)
 *   c_out   [nt][K][CPF_TOPM] their c values (or NULL)
 * With K < CPF_TOPM the entries past K hold index 0 and c = +inf.
 * Synchronous.  CPF_E_STATE when the plan has no current lists (before its
 * first search, or after cpf_plan_append to a plan never searched: an
 * append to a searched plan merges its lists with the new predecessors);
 * CPF_E_ARG for a range outside [1, T) or two NULL outputs. */
#define CPF_TOPM 16
cpf_status cpf_dp_lists(const cpf_plan *plan, int32_t t0, int32_t nt, uint16_t *idx_out, double *c_out);

/* Append K_add candidate plans to a plan, for a repeated search over K +
 * K_add candidates (Sec. III-B: more plans when the seed's mjac exceeds 12
 * degrees; Sec. III-C: when refinement finds no valid trajectory).
 * cand_add [K_add][T][dof] FP64 as in cpf_plan_init; node_pen_add [T][K_add]
 * or NULL (zero cost for the new nodes; nodes of a plan created without
 * node_pen cost zero).  Kept on the device, not uploaded again: the earlier
 * candidates and node costs and, once the plan has been searched, their
 * penalties and search lists, which are merged with the new predecessors
 * only; the following cpf_dp_search then runs the stage recursion alone.  The plan must be searched again before
 * cpf_lm_refine (CPF_E_STATE otherwise); its LM state restarts from the new
 * search.  CPF_E_UNSUPPORTED if K + K_add exceeds 1024, CPF_E_NOMEM if the
 * larger arena does not fit the budget (the plan is then unchanged).
 * Synchronous. */
cpf_status cpf_plan_append(cpf_plan *plan, int32_t K_add, const double *cand_add,
                           const double *node_pen_add);

/* Run `iters` LM iterations from the plan's current trajectory (the clamped
 * search seed the first time; resumable).  xi_out [T][dof] or NULL.
 * Sec. III-C.  Synchronous. */
cpf_status cpf_lm_refine(cpf_plan *plan, int32_t iters, double *xi_out, cpf_lm_report *rep);

/* The whole refinement of one plan (Sec. III-B then III-C): the complete
 * search (node penalties and predecessor lists rebuilt from the candidates,
 * then the stage recursion and back-tracking), then opts.iters LM iterations
 * from its seed (restarting the LM state) and the report, queued in one
 * stream with a single synchronisation at the end.
 * path_out [T], best_out, xi_out [T][dof], rep: each may be NULL.
 * Synchronous; CPF_E_NUMERIC as cpf_lm_refine. */
cpf_status cpf_plan_solve(cpf_plan *plan, int32_t *path_out, double *best_out, double *xi_out,
                          cpf_lm_report *rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work
 * of cpf_plan_init + cpf_plan_solve + cpf_plan_free in one call (the search,
 * then opts->iters LM iterations and the report; inputs as cpf_problem
 * describes, host or device) with every device buffer in a static array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends.  No hipMalloc, hipFree or other allocating call is made.  A problem
 * whose working memory (the arena of a plan of that T and K: about
 * 198 K + 3.6 KB bytes per waypoint, e.g. 15.5 MB for T = 300, K = 256, so
 * up to T of about 1230 at K = 256) exceeds 64 MiB returns CPF_E_NOMEM with
 * the sizes in the message.  path_out [T], best_out,
 * xi_out [T][dof] (host) and rep may each be NULL.  Calls on one GPU share
 * its array: the library runs them one after another (a per-device lock),
 * and each call starts by clearing the state it needs, so nothing carries
 * over from the previous one.  Synchronous, on the context's stream;
 * statuses as cpf_plan_init and cpf_plan_solve. */
cpf_status cpf_solve_static(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob, const cpf_opts *opts,
                            int32_t *path_out, double *best_out, double *xi_out, cpf_lm_report *rep);

/* Latest valid trajectory of a plan refined with opts.schedule = 1 (the
 * anytime result of Sec. III-C's alternating objective), written to xi_out
 * [T][dof] (caller-owned, not NULL).  CPF_E_STATE if the plan does not use
 * the schedule or no check has passed yet.  Synchronous. */
cpf_status cpf_lm_latest_valid(cpf_plan *plan, double *xi_out);

/* Search + opts->iters LM iterations for nplans independent problems in one
 * launch of each kernel (one workgroup per plan).  results[i].xi / .path may
 * be NULL.  Per-plan errors land in results[i].status; the call returns the
 * first argument / device error. */
cpf_status cpf_solve_batch(cpf_ctx *ctx, int32_t nplans, const cpf_robot *robots,
                           const cpf_problem *probs, const cpf_opts *opts,
                           cpf_result *results);

/* Optimise the M smoothest of the problem's K candidate plans directly,
 * without the search (the "BatchOpt" planner of the paper, Sec. III and its
 * planner list): the M candidates with the least mjac (largest joint change
 * between consecutive waypoints, Sec. III-B), ties to the lower index, each
 * clamped to the limits and refined by opts->iters LM iterations as an
 * independent plan (one workgroup each).  Writes the chosen candidate
 * indices to idx_out[M] (ascending mjac) and one result per candidate to
 * results[M] (xi / path may be NULL; path is all zeros: the seed is the
 * candidate itself).  1 <= M <= K, else CPF_E_ARG.  Synchronous. */
cpf_status cpf_batchopt(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                        const cpf_opts *opts, int32_t M, int32_t *idx_out, cpf_result *results);

/* Server shape, before the first cpf_submit: `slots` requests resident on the
 * device at once (default 256); per tick (one replay of the LM graph) every
 * resident request advances at most iters_per_tick LM iterations (default
 * 30) and, when tick_budget > 0 (default 6000), at most about
 * tick_budget / (T + 330) of them (at least one) for a request of T
 * waypoints, so that a tick lasts about as long for short and long requests
 * and short ones are not held back by long ones; tick_budget = 0 gives every
 * request iters_per_tick.  CPF_E_ARG for values out of range, CPF_E_STATE
 * once the server runs. */
cpf_status cpf_ctx_config(cpf_ctx *ctx, int32_t slots, int32_t iters_per_tick, int32_t tick_budget);

/* Serving: copy the request (host inputs; device inputs stay where they
 * are, see cpf_problem.mem), queue it, return a ticket at once.  The server
 * thread admits queued requests while their device bytes fit the budget,
 * runs their searches, and advances every admitted request by LM iterations
 * in shared launches until it reaches opts->iters, which must be >= 1
 * (CPF_E_ARG otherwise).  A request larger than the whole budget gives
 * CPF_E_NOMEM.  The server keeps three streams busy at once (LM ticks and
 * two search lanes); HIP maps a process's streams onto a pool of hardware
 * queues (GPU_MAX_HW_QUEUES, 4 unless set before HIP starts), where streams
 * sharing a queue serialise, so a process that holds other streams should
 * start with a pool of 8 or more. */
cpf_status cpf_submit(cpf_ctx *ctx, const cpf_robot *robot, const cpf_problem *prob,
                      const cpf_opts *opts, uint64_t *ticket);

/* Wait up to timeout_ms (0 = do not wait, <0 = forever) for a ticket.
 * CPF_PENDING while running; on completion copies xi / path into the
 * caller's buffers in *out (if non-NULL), fills the report and timestamps,
 * releases the ticket and returns CPF_OK (the request's own failure is in
 * out->status).  Unknown or already released ticket: CPF_E_NOTFOUND. */
cpf_status cpf_poll(cpf_ctx *ctx, uint64_t ticket, int32_t timeout_ms, cpf_result *out);

/* Kernel timing (tracing aid for the benchmark): with profiling enabled the
 * context brackets each of its kernel launches with HIP events on the
 * stream the kernel runs on.  cpf_ctx_kernel_stats returns the summed
 * duration (ms) and launch count since profiling was enabled (it
 * synchronises the context's streams) for "fk" (cpf_fk_batch and
 * cpf_coll_batch), "dp_lists" (the search's node penalties and predecessor
 * lists), "dp" (its stage recursion, back-tracking and seed), "lm" (LM
 * launches; in serving, each tick graph) or "eval" (the report). */
cpf_status cpf_ctx_profile(cpf_ctx *ctx, int32_t enable);
cpf_status cpf_ctx_kernel_stats(cpf_ctx *ctx, const char *kernel, double *total_ms,
                                int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* CPF_H */
