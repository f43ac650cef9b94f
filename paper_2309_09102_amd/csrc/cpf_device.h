// cpf_device.h -- device-side data layout and per-lane math of the CppFlow
// refinement path (arXiv 2309.09102) on gfx950.
//
// Layout of one plan in HBM (all SoA so that consecutive lanes touch
// consecutive addresses):
//   cand     float  [T][7][K]   candidate joint values (Sec. III-A), lane = k
//   extra    double [T][K]      optional caller search cost (Sec. III-B)
//   bp       uint16 [T][K]      search back-pointers
//   pen      double [T][K]      search node penalties
//   topk     uint16 [T][K][16]  nearest predecessors of each search node
//   topc     double [T][K][16]  their edges plus the node's penalty
//   path     int32  [T]
//   targets  double [12][T]     target poses (Sec. II): x y z, R row-major
//   xi, xt   double [7][T]      trajectory master copy and LM trial point
//   A        double [T][28]     w_p J_t^T J_t, packed lower triangles (row by row)
//   g        double [7][T]      gradient of the cost
//   cr       double             cyclic-reduction levels of the LM system (cr_doubles(T))
//   dx, rb   double [7][T]      step, refinement residual
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

constexpr int NJ = 7;         // joints
constexpr int NTRI = 28;      // packed lower triangle of a 7x7 block
constexpr int NBLK = 49;      // full 7x7 block
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
    int32_t refine_steps, schedule, prism, pad2;   // prism: bit i set = joint i prismatic
    double w_p, w_s, lam0, lam_min, lam_max, margin, penalty;
    // robot in double and float (cos/sin of the twist precomputed on host);
    // margin_p, the joint-limit margin of prismatic joints (m), takes the
    // eighth slot after the seven link lengths a
    double a[NJ], margin_p, d[8], ca[8], sa[8], off[8], lo[8], hi[8];
    float af[8], df[8], caf[8], saf[8], offf[8];
    CPF_GLOBAL const float *cand;
    CPF_GLOBAL const double *extra;
    CPF_GLOBAL uint16_t *bp;
    CPF_GLOBAL double *pen;       // [T][K] node penalties
    CPF_GLOBAL uint16_t *topk;    // [T][K][TOPM] nearest predecessors of each node
    CPF_GLOBAL double *topc;      // [T][K][TOPM] their edges plus the node penalty
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
    // weight and search penalty
    int32_t has_coll, n_obs;
    double coll_margin, w_coll, coll_penalty;
    double cap[NJ][7];
    float capf[NJ][7];
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
static_assert(offsetof(DevPlan, w_p) == 32, "DevPlan layout");
static_assert(offsetof(DevPlan, a) == 88, "DevPlan layout");
static_assert(offsetof(DevPlan, margin_p) == 144, "DevPlan layout");
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
static_assert(offsetof(DevPlan, coll_margin) == 888, "DevPlan layout");
static_assert(offsetof(DevPlan, cap) == 912, "DevPlan layout");
static_assert(offsetof(DevPlan, capf) == 1304, "DevPlan layout");
static_assert(offsetof(DevPlan, obs) == 1504, "DevPlan layout");
static_assert(offsetof(DevPlan, cpen) == 1512, "DevPlan layout");
static_assert(offsetof(DevPlan, rr) == 1520, "DevPlan layout");
static_assert(offsetof(DevPlan, rt) == 1528, "DevPlan layout");
static_assert(sizeof(DevPlan) == 1536, "DevPlan layout");
static_assert(sizeof(LMState) == 128, "LMState layout");

template <typename S>
struct RobotT {
    S a[NJ], d[NJ], ca[NJ], sa[NJ], off[NJ];
    uint32_t prism;   // bit i set: joint i is prismatic
};

__host__ __device__ __forceinline__ bool is_prismatic(uint32_t prism, int i) { return (prism >> i) & 1u; }

// The plan's robot in precision S.  PRISM false: a chain known to be all
// revolute (the plans with collision capsules, which cannot hold a
// prismatic joint); the joint-type mask is then neither loaded nor used, and
// the chain functions below compile their revolute-only form.
template <typename S> struct RobotRows;
template <> struct RobotRows<double> {
    static __device__ __forceinline__ void get(const DevPlan &P, RobotT<double> &r) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            r.a[i] = P.a[i]; r.d[i] = P.d[i]; r.ca[i] = P.ca[i]; r.sa[i] = P.sa[i]; r.off[i] = P.off[i];
        }
    }
};
template <> struct RobotRows<float> {
    static __device__ __forceinline__ void get(const DevPlan &P, RobotT<float> &r) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            r.a[i] = P.af[i]; r.d[i] = P.df[i]; r.ca[i] = P.caf[i]; r.sa[i] = P.saf[i]; r.off[i] = P.offf[i];
        }
    }
};

template <typename S, bool PRISM = true>
__device__ __forceinline__ RobotT<S> load_robot(const DevPlan &P) {
    RobotT<S> r;
    RobotRows<S>::get(P, r);
    if constexpr (PRISM) r.prism = (uint32_t)P.prism;
    return r;
}

__device__ __forceinline__ void dev_sincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void dev_sincos(double x, double *s, double *c) { sincos(x, s, c); }

// Kinematic chain of the standard DH convention, kept in registers.
// Frame columns X, Y, Z and origin p start at the identity; link i maps
//   X' = c X + s Y,  W = c Y - s X,  Y' = ca W + sa Z,  Z' = ca Z - sa W,
//   p' = p + a X' + d Z,
// which is the product with Rz(theta) Tz(d) Tx(a) Rx(alpha) written per
// column; theta = q + offset and d fixed for a revolute joint, theta = offset
// and d + q for a prismatic one.  With FRAMES the axis Z and origin p of
// joint i (before link i) are kept for the geometric Jacobian.
template <typename S>
__device__ __forceinline__ void chain_start(S X[3], S Y[3], S Z[3], S p[3]) {
    X[0] = 1; X[1] = 0; X[2] = 0;
    Y[0] = 0; Y[1] = 1; Y[2] = 0;
    Z[0] = 0; Z[1] = 0; Z[2] = 1;
    p[0] = 0; p[1] = 0; p[2] = 0;
}

// Link i of the chain: the frame before it becomes the frame after it.
// PRISM false: every joint revolute (the mask is not read).
template <typename S, bool PRISM = true>
__device__ __forceinline__ void dh_step(const RobotT<S> &rb, int i, S qi, S X[3], S Y[3], S Z[3], S p[3]) {
    if constexpr (!PRISM) {
        S s, c;
        dev_sincos(qi + rb.off[i], &s, &c);
        S nx[3], w[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            nx[r] = c * X[r] + s * Y[r];
            w[r] = c * Y[r] - s * X[r];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            p[r] = p[r] + rb.a[i] * nx[r] + rb.d[i] * Z[r];
            Y[r] = rb.ca[i] * w[r] + rb.sa[i] * Z[r];
            Z[r] = rb.ca[i] * Z[r] - rb.sa[i] * w[r];
            X[r] = nx[r];
        }
        return;
    }
    const bool pr = is_prismatic(rb.prism, i);
    S s, c;
    dev_sincos(pr ? rb.off[i] : qi + rb.off[i], &s, &c);
    const S di = pr ? rb.d[i] + qi : rb.d[i];
    S nx[3], w[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        nx[r] = c * X[r] + s * Y[r];
        w[r] = c * Y[r] - s * X[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        p[r] = p[r] + rb.a[i] * nx[r] + di * Z[r];
        Y[r] = rb.ca[i] * w[r] + rb.sa[i] * Z[r];
        Z[r] = rb.ca[i] * Z[r] - rb.sa[i] * w[r];
        X[r] = nx[r];
    }
}

// Column i of the geometric Jacobian at end-effector position p: a revolute
// joint gives [z x (p - o); z], a prismatic one [z; 0].
template <typename S>
__device__ __forceinline__ void jac_column(uint32_t prism, int i, const S z[3], const S o[3], const S p[3],
                                           S col[6]) {
    const bool pr = is_prismatic(prism, i);
    const S dx = p[0] - o[0], dy = p[1] - o[1], dz = p[2] - o[2];
    col[0] = pr ? z[0] : z[1] * dz - z[2] * dy;
    col[1] = pr ? z[1] : z[2] * dx - z[0] * dz;
    col[2] = pr ? z[2] : z[0] * dy - z[1] * dx;
    col[3] = pr ? S(0) : z[0];
    col[4] = pr ? S(0) : z[1];
    col[5] = pr ? S(0) : z[2];
}

template <typename S, bool FRAMES, bool PRISM = true>
__device__ __forceinline__ void chain(const RobotT<S> &rb, const S *q, S X[3], S Y[3], S Z[3],
                                      S p[3], S Zs[NJ][3], S Os[NJ][3]) {
    chain_start(X, Y, Z, p);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        if (FRAMES) {
#pragma unroll
            for (int r = 0; r < 3; ++r) { Zs[i][r] = Z[r]; Os[i][r] = p[r]; }
        }
        dh_step<S, PRISM>(rb, i, q[i], X, Y, Z, p);
    }
}

template <typename S> __device__ __forceinline__ S dev_atan2(S y, S x);
template <> __device__ __forceinline__ float dev_atan2<float>(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double dev_atan2<double>(double y, double x) { return atan2(y, x); }

// Rotation vector of E (row-major 3x3): angle atan2(|v|, (tr E - 1)/2) with
// v = vee(E - E^T)/2; series for the small-angle factor, and the axis of the
// symmetric part near pi.
template <typename S>
__device__ __forceinline__ void log_rot(const S E[9], S phi[3]) {
    const S v0 = S(0.5) * (E[7] - E[5]);
    const S v1 = S(0.5) * (E[2] - E[6]);
    const S v2 = S(0.5) * (E[3] - E[1]);
    const S sn = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const S cs = S(0.5) * (E[0] + E[4] + E[8] - S(1));
    const S th = dev_atan2<S>(sn, cs);
    if (th < S(1e-4)) {
        const S k = S(1) + th * th / S(6);
        phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
        return;
    }
    if (th > S(3.14159265358979323846) - S(1e-6)) {
        S B[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                B[r][c] = S(0.5) * (E[r * 3 + c] + E[c * 3 + r]) - (r == c ? cs : S(0));
        int i = 0;
        if (B[1][1] > B[i][i]) i = 1;
        if (B[2][2] > B[i][i]) i = 2;
        const S omc = S(1) - cs;
        const S ui = sqrt(B[i][i] / omc);
        S u[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[j] = B[i][j] / (omc * ui);
        u[i] = ui;
        if (u[0] * v0 + u[1] * v1 + u[2] * v2 < S(0)) { u[0] = -u[0]; u[1] = -u[1]; u[2] = -u[2]; }
        phi[0] = th * u[0]; phi[1] = th * u[1]; phi[2] = th * u[2];
        return;
    }
    const S k = th / sn;
    phi[0] = k * v0; phi[1] = k * v1; phi[2] = k * v2;
}

// Pose residual r = [p - p*; Log(R R*^T)] of one waypoint; R has columns
// X, Y, Z.  tgt is x y z then R* row-major (already in S).
template <typename S>
__device__ __forceinline__ void pose_residual(const S X[3], const S Y[3], const S Z[3], const S p[3],
                                              const S tgt[12], S r[6]) {
    r[0] = p[0] - tgt[0];
    r[1] = p[1] - tgt[1];
    r[2] = p[2] - tgt[2];
    S E[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)   // (R R*^T)_ij = sum_k R_ik R*_jk, R_ik = column k row i
            E[i * 3 + j] = X[i] * tgt[3 + j * 3 + 0] + Y[i] * tgt[3 + j * 3 + 1] + Z[i] * tgt[3 + j * 3 + 2];
    log_rot<S>(E, r + 3);
}

__host__ __device__ constexpr int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

// Storage of one cyclic-reduction level with n blocks (no = n / 2 odd
// blocks, ne = n - no even ones), in doubles: a general 7x7 block whole (49,
// row-major), a symmetric or triangular one as its packed lower triangle
// (28), a vector whole (7).  The sub-diagonal blocks E (49 n), the even
// blocks' diagonal block and right-hand side (28 ne + 7 ne), the solution
// (7 n), and per odd block the inverse Cholesky factor (28), the two
// coupling products (2 x 49), the two Schur contributions (2 x 28), the
// transformed right-hand side and its two contributions (3 x 7); the last
// level (n = 1) keeps its factor in the first odd slot.
__host__ __device__ inline size_t cr_level_doubles(int n) {
    const size_t no = (size_t)(n / 2), ne = (size_t)n - no, nod = no > 0 ? no : 1;
    return 56 * (size_t)n + 35 * ne + 203 * nod;
}

// All levels of a path of T waypoints (n halves, rounding up, down to 1).
__host__ __device__ inline size_t cr_doubles(int T) {
    size_t total = 0;
    int n = T;
    while (true) {
        total += cr_level_doubles(n);
        if (n <= 1) break;
        n = (n + 1) / 2;
    }
    return total;
}

}  // namespace cpf
