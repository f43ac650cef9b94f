// cpf_plan.h -- the plan descriptor of the CppFlow refinement path (arXiv
// 2309.09102) on gfx950, shared by the host code and by the kernels of every
// chain length, and the storage sizes both compute.
//
// Layout of one plan of n = dof joints in HBM (all SoA so that consecutive
// lanes touch consecutive addresses):
//   cand     float  [T][n][K]   candidate joint values (Sec. III-A), lane = k
//   extra    double [T][K]      optional caller search cost (Sec. III-B)
//   bp       uint16 [T][K]      search back-pointers
//   pen      double [T][K]      search node penalties
//   topk     uint32 [T][8][K]   nearest predecessors of each search node (16, in pairs)
//   topc     double [T][16][K]  their edges plus the node's penalty
//   path     int32  [T]
//   targets  double [12][T]     target poses (Sec. II): x y z, R row-major
//   xi, xt   double [n][T]      trajectory master copy and LM trial point
//   A        double [T][n(n+1)/2] w_p J_t^T J_t, packed lower triangles (row by row)
//   g        double [n][T]      gradient of the cost
//   cr       double             cyclic-reduction levels of the LM system (cr_doubles(T, n))
//   dx, rb   double [n][T]      step, refinement residual
//   rr, rt   double [8][T]      FP64 residual rows of xi and of the trial point
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Device code reaches the per-plan arrays through pointers stored in the plan
// descriptor.  Marking them as global-address-space pointers lets the
// compiler emit global (not flat) memory instructions, whose completion is
// counted separately from LDS traffic, so loads issued ahead stay in flight
// across LDS waits.  Host code sees plain pointers (same size and layout).
#ifdef __HIP_DEVICE_COMPILE__
#define CPF_GLOBAL __attribute__((address_space(1)))
#else
#define CPF_GLOBAL
#endif

// Host-side store of a device address into a descriptor field (an integer
// round trip, valid whichever address space the field carries).
template <class Field, class Ptr>
inline void set_dev_ptr(Field &field, Ptr *p) {
    field = (Field)(uintptr_t)p;
}

namespace cpf {

constexpr int NJMAX = 8;      // joints of the longest chain the kernels are built for
constexpr int MAX_K = 1024;   // search kernel limit (one lane per destination)
constexpr int MAX_OBS = 64;   // cuboid obstacles per problem
constexpr int CPF_STATUS_NUMERIC = -6;
constexpr int TOPM = 16;      // nearest predecessors kept per search node
constexpr int RROWS = 8;      // residual rows per waypoint: 6 pose, then self and environment collision

struct LMState {
    double lambda, nu, cost, cost0, grad_inf;
    // schedule mode: the length of the latest valid trajectory (lambda, nu
    // above belong to the pose objective)
    double valid_length, pad2, pad3;
    int32_t n_acc, iters_done, status, need_lin;
    int32_t iters_target, seeded, reported, checked;
    // schedule mode: objective of the next step (0 pose, 1 differencing) as
    // the last validity check decided, objective of the previous step (-1:
    // none), checks passed, iteration of the first pass (-1: none), steps
    // taken on each objective
    int32_t mode, last_mode, n_valid, first_valid;
    int32_t pose_steps, diff_steps, pad0, pad1;
};

struct DevPlan {
    int32_t T, K, has_extra, prec;
    int32_t refine_steps, schedule, prism, dof;    // prism: bit i set = joint i prismatic
    double w_p, w_s, lam0, lam_min, lam_max, margin, penalty;
    // robot in double and float (cos/sin of the twist precomputed on host),
    // dof rows used
    double a[NJMAX], d[NJMAX], ca[NJMAX], sa[NJMAX], off[NJMAX], lo[NJMAX], hi[NJMAX];
    float af[NJMAX], df[NJMAX], caf[NJMAX], saf[NJMAX], offf[NJMAX];
    CPF_GLOBAL const float *cand;
    CPF_GLOBAL const double *extra;
    CPF_GLOBAL uint16_t *bp;
    CPF_GLOBAL double *pen;       // [T][K] node penalties
    CPF_GLOBAL uint16_t *topk;    // [T][TOPM / 2][K] nearest predecessors of each node, in pairs per 32-bit word
    CPF_GLOBAL double *topc;      // [T][TOPM][K] their edges plus the node penalty
    CPF_GLOBAL int32_t *path;
    CPF_GLOBAL double *dp_out;    // [0] = B*, [1] = mjac of the seed, [2] = end node, [3] / [4] = the
                                  // seed's largest revolute / prismatic joint step
    CPF_GLOBAL double *targets;
    CPF_GLOBAL double *xi, *xt, *A, *g, *cr, *dx, *rb;
    CPF_GLOBAL LMState *st;
    CPF_GLOBAL double *report;    // [0] max pos err, [1] max rot err, [2] mjac, [3] min self
                                  // distance, [4] min environment distance
    // schedule mode: validity thresholds (position m, rotation rad, step of
    // a revolute joint rad, step of a prismatic joint m) and the latest
    // valid trajectory [dof][T]
    double vtol[4];
    CPF_GLOBAL double *xv;
    // collision geometry (has_coll): capsule of each link (endpoints in the
    // frame after the link, radius) in double and float, obstacles [n_obs][18]
    // (frame origin, rotation row-major, p_min, p_max), residual margin,
    // weight and search penalty; margin_p: the joint-limit margin of
    // prismatic joints (m)
    int32_t has_coll, n_obs;
    double coll_margin, w_coll, coll_penalty, margin_p;
    double cap[NJMAX][7];
    float capf[NJMAX][7];
    CPF_GLOBAL const double *obs;
    CPF_GLOBAL double *cpen;      // [T][K] collision penalty of each search node
    // FP64 residual rows [RROWS][T] of xi and of the trial point xt (kept by
    // the mixed arm, whose linearisation takes them instead of recomputing
    // the residual in FP32)
    CPF_GLOBAL double *rr, *rt;
};

// The host fills descriptors and LM states that kernels read, so both
// compilation passes (host and gfx950) must lay them out alike: each pass
// checks every field offset against these figures.
static_assert(offsetof(DevPlan, T) == 0, "DevPlan layout");
static_assert(offsetof(DevPlan, refine_steps) == 16, "DevPlan layout");
static_assert(offsetof(DevPlan, dof) == 28, "DevPlan layout");
static_assert(offsetof(DevPlan, w_p) == 32, "DevPlan layout");
static_assert(offsetof(DevPlan, a) == 88, "DevPlan layout");
static_assert(offsetof(DevPlan, d) == 152, "DevPlan layout");
static_assert(offsetof(DevPlan, ca) == 216, "DevPlan layout");
static_assert(offsetof(DevPlan, sa) == 280, "DevPlan layout");
static_assert(offsetof(DevPlan, off) == 344, "DevPlan layout");
static_assert(offsetof(DevPlan, lo) == 408, "DevPlan layout");
static_assert(offsetof(DevPlan, hi) == 472, "DevPlan layout");
static_assert(offsetof(DevPlan, af) == 536, "DevPlan layout");
static_assert(offsetof(DevPlan, df) == 568, "DevPlan layout");
static_assert(offsetof(DevPlan, caf) == 600, "DevPlan layout");
static_assert(offsetof(DevPlan, saf) == 632, "DevPlan layout");
static_assert(offsetof(DevPlan, offf) == 664, "DevPlan layout");
static_assert(offsetof(DevPlan, cand) == 696, "DevPlan layout");
static_assert(offsetof(DevPlan, extra) == 704, "DevPlan layout");
static_assert(offsetof(DevPlan, bp) == 712, "DevPlan layout");
static_assert(offsetof(DevPlan, pen) == 720, "DevPlan layout");
static_assert(offsetof(DevPlan, topk) == 728, "DevPlan layout");
static_assert(offsetof(DevPlan, topc) == 736, "DevPlan layout");
static_assert(offsetof(DevPlan, path) == 744, "DevPlan layout");
static_assert(offsetof(DevPlan, dp_out) == 752, "DevPlan layout");
static_assert(offsetof(DevPlan, targets) == 760, "DevPlan layout");
static_assert(offsetof(DevPlan, xi) == 768, "DevPlan layout");
static_assert(offsetof(DevPlan, xt) == 776, "DevPlan layout");
static_assert(offsetof(DevPlan, A) == 784, "DevPlan layout");
static_assert(offsetof(DevPlan, g) == 792, "DevPlan layout");
static_assert(offsetof(DevPlan, cr) == 800, "DevPlan layout");
static_assert(offsetof(DevPlan, dx) == 808, "DevPlan layout");
static_assert(offsetof(DevPlan, rb) == 816, "DevPlan layout");
static_assert(offsetof(DevPlan, st) == 824, "DevPlan layout");
static_assert(offsetof(DevPlan, report) == 832, "DevPlan layout");
static_assert(offsetof(DevPlan, vtol) == 840, "DevPlan layout");
static_assert(offsetof(DevPlan, xv) == 872, "DevPlan layout");
static_assert(offsetof(DevPlan, has_coll) == 880, "DevPlan layout");
static_assert(offsetof(DevPlan, n_obs) == 884, "DevPlan layout");
static_assert(offsetof(DevPlan, coll_margin) == 888, "DevPlan layout");
static_assert(offsetof(DevPlan, margin_p) == 912, "DevPlan layout");
static_assert(offsetof(DevPlan, cap) == 920, "DevPlan layout");
static_assert(offsetof(DevPlan, capf) == 1368, "DevPlan layout");
static_assert(offsetof(DevPlan, obs) == 1592, "DevPlan layout");
static_assert(offsetof(DevPlan, cpen) == 1600, "DevPlan layout");
static_assert(offsetof(DevPlan, rr) == 1608, "DevPlan layout");
static_assert(offsetof(DevPlan, rt) == 1616, "DevPlan layout");
static_assert(sizeof(DevPlan) == 1624, "DevPlan layout");
static_assert(sizeof(LMState) == 128, "LMState layout");

__host__ __device__ __forceinline__ bool is_prismatic(uint32_t prism, int i) { return (prism >> i) & 1u; }

__host__ __device__ constexpr int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

// Storage of one cyclic-reduction level with n blocks (no = n / 2 odd
// blocks, ne = n - no even ones) of a chain of nj joints, in doubles: a
// general nj x nj block whole (nb = nj^2, row-major), a symmetric or
// triangular one as its packed lower triangle (nt = nj (nj + 1) / 2), a
// vector whole (nj).  The sub-diagonal blocks E (nb n), the even blocks'
// diagonal block and right-hand side (nt ne + nj ne), the solution (nj n),
// and per odd block the inverse Cholesky factor (nt), the two coupling
// products (2 nb), the two Schur contributions (2 nt), the transformed
// right-hand side and its two contributions (3 nj); the last level (n = 1)
// keeps its factor in the first odd slot.
__host__ __device__ inline size_t cr_level_doubles(int n, int nj) {
    const size_t no = (size_t)(n / 2), ne = (size_t)n - no, nod = no > 0 ? no : 1;
    const size_t nb = (size_t)nj * nj, nt = (size_t)nj * (nj + 1) / 2;
    return (nb + nj) * (size_t)n + (nt + nj) * ne + (3 * nt + 2 * nb + 3 * (size_t)nj) * nod;
}

// All levels of a path of T waypoints (n halves, rounding up, down to 1).
__host__ __device__ inline size_t cr_doubles(int T, int nj) {
    size_t total = 0;
    int n = T;
    while (true) {
        total += cr_level_doubles(n, nj);
        if (n <= 1) break;
        n = (n + 1) / 2;
    }
    return total;
}

}  // namespace cpf
