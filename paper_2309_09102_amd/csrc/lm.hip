// lm.hip -- Levenberg-Marquardt trajectory optimisation (Sec. III-C).
//
// Cost  C(xi) = w_p/2 sum_t |r_t|^2 + w_s/2 sum_t |xi_{t+1} - xi_t|^2 with the
// pose residual r_t = [p(q_t) - p*_t; Log(R(q_t) R*_t^T)] (Sec. II, III-C) and
// the differencing residual whose Jacobian is +I / -I.  Gauss-Newton with
// Levenberg damping gives a block-tridiagonal system
//   D_t = w_p J_t^T J_t + (w_s c_t + lambda) I,  off-diagonal blocks -w_s I,
//   g_t = w_p J_t^T r_t + w_s (c_t xi_t - xi_{t-1} - xi_{t+1}),
//   H delta = -g,
// with c_t the number of neighbours of waypoint t.  The step is clamped to
// the joint limits; lambda follows Nielsen's gain-ratio rule.
//
// One workgroup per plan runs all iterations without returning to the host.
// The residuals r_t, the cost and every cross-waypoint sum are FP64 in both
// arms; the arms differ in the Jacobian: S = float builds J_t from an FP32
// chain (the mixed arm), S = double from an FP64 one.  The Gram J^T J and the
// gradient J^T r accumulate in FP64.  This is the split of mixed-precision
// iterative refinement: the matrix of the linearised system only sets how
// fast the iteration converges, while the right-hand side (the residual and
// the gradient formed from it) and the accept test set the point it
// converges to, so those stay FP64.  The mixed arm keeps the FP64 residual
// of its current trajectory from the trial evaluation that accepted it, so
// each iteration still runs one chain per precision.  The solve is
// block cyclic reduction (a Cholesky factor per eliminated block, one lane
// per NJ x NJ block, log2 T levels), then FP64 iterative refinement against the
// same H reusing the stored factors.
#include <float.h>

#include "coll_device.h"
#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {
namespace CPF_JNS {

constexpr int LM_BS = 512;
// Fixed cost of an LM iteration in waypoints: an iteration of a plan of T
// waypoints takes about as long as T + LM_ITER_FIXED waypoints' worth of
// the per-waypoint work (the reduction rounds of the solve cost the same
// for any level size), measured on the one-workgroup kernel at T = 300 to
// 2000.
constexpr int LM_ITER_FIXED = 330;

// Workgroup sums (or maxima) of N values per thread, by a fixed tree: inside
// each wavefront by lane shuffles (offsets 32, 16, ..., 1, into lane 0),
// then the wavefronts' partial results in wavefront order, so that every run
// adds in the same order.  Two barriers for any N: after the partials are
// written, and before `red` may be written again.  `red` holds at least
// N * LM_BS / 64 doubles.
template <int N, bool MAX>
__device__ __forceinline__ void block_reduce_n(double v[N], double *red) {
    constexpr int NW = LM_BS / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double x = v[i];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            const double y = __shfl_down(x, s, 64);
            x = MAX ? fmax(x, y) : x + y;
        }
        if (lane == 0) red[wave * N + i] = x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double r = red[i];
#pragma unroll
        for (int w = 1; w < NW; ++w) r = MAX ? fmax(r, red[w * N + i]) : r + red[w * N + i];
        v[i] = r;
    }
    __syncthreads();
}
template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double *red) {
    double a[1] = {v};
    block_reduce_n<1, MAX>(a, red);
    return a[0];
}
__device__ __forceinline__ double block_sum(double v, double *red) { return block_reduce<false>(v, red); }
__device__ __forceinline__ double block_max(double v, double *red) { return block_reduce<true>(v, red); }

#ifdef CPF_PHASE_CYCLES
// Diagnostic build only: shader-clock totals of the iteration's phases, the
// solve's rounds and the steps of its one-wavefront levels, summed over a
// launch by thread 0 of each workgroup; workgroup 0 prints them at its end.
// All of it, the last clock readings included (one for the phases, one for
// the rounds and steps inside a solve), lives in LDS, so the marks hold no
// registers across the code they time.  Reading the clock waits for the
// wavefront's outstanding LDS operations.
__shared__ unsigned long long diag_last[2];
__shared__ unsigned long long diag_phase[8];
__shared__ unsigned long long diag_round[2][64];
__shared__ unsigned long long diag_tail[2][12];
#define DIAG_MARK(slot, clk)                           \
    do {                                               \
        if (threadIdx.x == 0) {                        \
            const unsigned long long now_ = clock64(); \
            (slot) += now_ - diag_last[clk];           \
            diag_last[clk] = now_;                     \
        }                                              \
    } while (0)
#else
#define DIAG_MARK(slot, clk) \
    do {                     \
    } while (0)
#endif

template <typename S>
__device__ __forceinline__ void load_target(const DevPlan &P, int T, int t, S tg[12]) {
#pragma unroll
    for (int e = 0; e < 12; ++e) tg[e] = (S)P.targets[(size_t)e * T + t];
}

// Pose residual of trajectory X ([NJ][T]) at waypoint t in FP64 (written to
// r) and its squared norm.  PR false throughout this file: a chain known to
// be all revolute (plans with collision capsules).
template <bool PR>
__device__ __forceinline__ double pose_res64(const DevPlan &P, const RobotT<double> &rb, const CPF_GLOBAL double *X,
                                             int T, int t, double r[6]) {
    double q[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = X[(size_t)j * T + t];
    double Xc[3], Yc[3], Zc[3], p[3], Zs[NJ][3], Os[NJ][3];
    chain<double, false, PR>(rb, q, Xc, Yc, Zc, p, Zs, Os);
    double tg[12];
    load_target<double>(P, T, t, tg);
    pose_residual<double>(Xc, Yc, Zc, p, tg, r);
    double s = r[0] * r[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) s += r[i] * r[i];
    return s;
}

// The plan's capsules in the kinematics precision.
template <typename S> struct CapsOf;
template <> struct CapsOf<double> {
    static __device__ __forceinline__ const double (*get(const DevPlan &P))[7] { return P.cap; }
};
template <> struct CapsOf<float> {
    static __device__ __forceinline__ const float (*get(const DevPlan &P))[7] { return P.capf; }
};

// The two collision residuals max(0, margin - d) of waypoint t of X and,
// with GRAD, their Jacobians (minus the distance gradients where positive).
template <typename S, bool GRAD, bool PR>
__device__ __forceinline__ void coll_residuals(const DevPlan &P, const RobotT<S> &rb, const S q[NJ], double rc[2],
                                               double Jc[2][NJ]) {
    S dm[2], g[2][NJ];
    coll_distances<S, GRAD, S, PR>(rb, CapsOf<S>::get(P), P.n_obs, P.obs, q, dm, g, (S)P.coll_margin);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double r = P.coll_margin - (double)dm[h];
        rc[h] = r > 0.0 ? r : 0.0;
        if (GRAD)
#pragma unroll
            for (int k = 0; k < NJ; ++k) Jc[h][k] = r > 0.0 ? -(double)g[h][k] : 0.0;
    }
}

// Cost of trajectory X in FP64: pose, smoothness and (wc != 0) collision
// parts, block-reduced.  With R non-null every waypoint's residual rows go
// to R ([RROWS][T]; the collision rows only when wc != 0).
template <bool PR>
__device__ __forceinline__ double plan_cost(const DevPlan &P, const CPF_GLOBAL double *X, int T, double *red,
                                            double wp, double ws, double wc, CPF_GLOBAL double *R,
                                            double *extra_sum = nullptr, double extra = 0.0) {
    const RobotT<double> rb = load_robot<double, PR>(P);
    double ps = 0.0, ss = 0.0, cs = 0.0;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double r[6];
        ps += pose_res64<PR>(P, rb, X, T, t, r);
        if (R) {
#pragma unroll
            for (int i = 0; i < 6; ++i) R[(size_t)i * T + t] = r[i];
        }
        if (t + 1 < T) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const double d = X[(size_t)j * T + t + 1] - X[(size_t)j * T + t];
                ss += d * d;
            }
        }
        if (wc != 0.0) {
            double q[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) q[j] = X[(size_t)j * T + t];
            double rc[2], Jc[2][NJ];
            coll_residuals<double, false, PR>(P, rb, q, rc, Jc);
            cs += rc[0] * rc[0] + rc[1] * rc[1];
            if (R) {
                R[(size_t)6 * T + t] = rc[0];
                R[(size_t)7 * T + t] = rc[1];
            }
        }
    }
    // one reduction for the three terms and the caller's extra per-thread
    // value (the trial's predicted reduction)
    double sums[4] = {ps, ss, cs, extra};
    block_reduce_n<4, false>(sums, red);
    if (extra_sum) *extra_sum = sums[3];
    const double coll_sum = wc != 0.0 ? sums[2] : 0.0;
    return 0.5 * wp * sums[0] + 0.5 * ws * sums[1] + 0.5 * wc * coll_sum;
}

// Linearise at xi: A_t = w_p J^T J (whole blocks), g_t; returns max |g|.
// S = double: J and the residual from one FP64 chain.  S = float (the mixed
// arm): J from an FP32 chain, the residual rows of xi in FP64 from P.rr,
// where the cost evaluation that produced xi left them.
template <typename S, bool PR>
__device__ __forceinline__ double linearise(const DevPlan &P, const RobotT<S> &rb, int T, double w_p, double w_s,
                                            double w_c) {
    constexpr bool F64 = sizeof(S) == sizeof(double);
    double gmax = 0.0;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double xq[NJ];
        S q[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            xq[j] = P.xi[(size_t)j * T + t];
            q[j] = (S)xq[j];
        }
        double r[6];
        if constexpr (!F64) {
#pragma unroll
            for (int i = 0; i < 6; ++i) r[i] = P.rr[(size_t)i * T + t];
        }
        S Xc[3], Yc[3], Zc[3], p[3], Zs[NJ][3], Os[NJ][3];
        chain<S, true, PR>(rb, q, Xc, Yc, Zc, p, Zs, Os);
        if constexpr (F64) {
            double tg[12];
            load_target<double>(P, T, t, tg);
            pose_residual<double>(Xc, Yc, Zc, p, tg, r);
        }
        S J[6][NJ];
        if constexpr (PR) {
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                S col[6];
                jac_column<S>(rb.prism, i, Zs[i], Os[i], p, col);
#pragma unroll
                for (int r = 0; r < 6; ++r) J[r][i] = col[r];
            }
        } else {
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const S dx = p[0] - Os[i][0], dy = p[1] - Os[i][1], dz = p[2] - Os[i][2];
                J[0][i] = Zs[i][1] * dz - Zs[i][2] * dy;
                J[1][i] = Zs[i][2] * dx - Zs[i][0] * dz;
                J[2][i] = Zs[i][0] * dy - Zs[i][1] * dx;
                J[3][i] = Zs[i][0];
                J[4][i] = Zs[i][1];
                J[5][i] = Zs[i][2];
            }
        }
        // The Gram matrix and the gradient J^T r of the (FP32 or FP64)
        // Jacobian and residual are accumulated in FP64.  Then the Gram is
        // positive semi-definite to FP64 rounding, so the damped block stays
        // positive definite for every lambda >= lambda_min also without a
        // smoothness term (the schedule's pose step), and the gradient lies
        // in J's row space to FP64 rounding: FP32 accumulation would leave a
        // component along J's null space (the self-motion direction) that a
        // pose-only step amplifies by 1 / lambda.
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double s = (double)J[0][i] * (double)J[0][j];
#pragma unroll
                for (int k = 1; k < 6; ++k) s += (double)J[k][i] * (double)J[k][j];
                P.A[(size_t)t * NTRI + tri_index(i, j)] = w_p * s;   // packed lower triangle
            }
        }
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            double s = (double)J[0][i] * r[0];
#pragma unroll
            for (int k = 1; k < 6; ++k) s += (double)J[k][i] * r[k];
            double gi = w_p * s;
            double sm = 0.0;
            if (t > 0) sm += xq[i] - P.xi[(size_t)i * T + t - 1];
            if (t + 1 < T) sm += xq[i] - P.xi[(size_t)i * T + t + 1];
            gi += w_s * sm;
            P.g[(size_t)i * T + t] = gi;
            gmax = fmax(gmax, fabs(gi));
        }
    }
    // Collision residuals (w_c != 0): w_c sum_h J_h J_h^T and w_c sum_h
    // J_h r_h added to the waypoint's block and gradient (a second pass, so
    // the pose pass keeps its registers).
    if (w_c != 0.0) {
        gmax = 0.0;
        for (int t = threadIdx.x; t < T; t += LM_BS) {
            S q[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) q[j] = (S)P.xi[(size_t)j * T + t];
            double rc[2], Jc[2][NJ];
            if constexpr (F64) {
                coll_residuals<S, true, PR>(P, rb, q, rc, Jc);
            } else {   // FP32 distance gradients; the FP64 residuals decide which are active
                S dm[2], gd[2][NJ];
                coll_distances<S, true, S, PR>(rb, CapsOf<S>::get(P), P.n_obs, P.obs, q, dm, gd, (S)P.coll_margin);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    rc[h] = P.rr[(size_t)(6 + h) * T + t];
#pragma unroll
                    for (int k = 0; k < NJ; ++k) Jc[h][k] = rc[h] > 0.0 ? -(double)gd[h][k] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    P.A[(size_t)t * NTRI + tri_index(i, j)] += w_c * (Jc[0][i] * Jc[0][j] + Jc[1][i] * Jc[1][j]);
                const double gi = P.g[(size_t)i * T + t] + w_c * (Jc[0][i] * rc[0] + Jc[1][i] * rc[1]);
                P.g[(size_t)i * T + t] = gi;
                gmax = fmax(gmax, fabs(gi));
            }
        }
    }
    return gmax;
}

// ---------------------------------------------------------------------------
// Block-tridiagonal solve by cyclic reduction.
//
// Level 0 is the LM system: diagonal blocks D_t, sub-diagonal blocks
// E_t = -w_s I.  A level with n blocks eliminates its odd blocks i:
//   L_i L_i^T = D_i (Cholesky), Li = L_i^{-1},
//   W_i = Li E_i,  V_i = Li E_{i+1}^T,
//   D'_{i-1} -= W_i^T W_i,  D'_{i+1} -= V_i^T V_i,
//   E'_{(i+1)/2} = -V_i^T W_i        (new coupling of blocks i+1 and i-1),
//   s_i = Li r_i,  r'_{i-1} -= W_i^T s_i,  r'_{i+1} -= V_i^T s_i,
// and its even blocks j form level l+1 as block j/2.  At the single block of
// the last level x = Li^T Li r; going back down, every odd block recovers
//   x_i = Li^T (s_i - W_i x_{i-1} - V_i x_{i+1}).
// At level 0 (E = -w I) this is W_i = V_i = -w Li, the Schur contribution
// w^2 Li^T Li on both neighbours and E' = -w^2 Li^T Li.  The factors of all
// levels stay in the plan's `cr` storage, so a further right-hand side (the
// refinement) costs only the right-hand-side and back-substitution rounds.
//
// Each round is one pass over a level followed by one workgroup barrier.
// Level 0 runs one lane per block.  Above it, NJ lanes share an odd block
// (lane c owns column c of W, V and of the products) and exchange columns
// through a per-group LDS area; LDS instructions of one wavefront complete
// in order, so a wave barrier is the only synchronisation the exchange
// needs.  Blocks are NJ x NJ row-major (NBLK doubles) one after another, so a
// lane reaches every element of its block, row or column from one per-lane
// address plus an instruction immediate.  Of the Gram blocks A_t, the
// diagonal blocks kept for the next level, the level-0 Schur contributions
// and the factors Li only the lower triangle is written: a reader takes a
// symmetric block's element (i, j) at (max, min) and a factor's upper part
// as zero, and the other readers use only the lower triangle.
// ---------------------------------------------------------------------------

constexpr int CR_GPW = 64 / NJ;                    // NJ-lane groups per wavefront
constexpr int CR_GL = CR_GPW * NJ;                 // lanes in groups (7 joints: lane 63 idles)
constexpr int CR_GROUPS = (LM_BS / 64) * CR_GPW;   // groups per workgroup
constexpr int CR_EX = 2 * NBLK;                    // LDS doubles per group

struct CRLevel {
    CPF_GLOBAL double *p;
    int n, no, ne, nod;
    // whole blocks: E, W, V; packed lower triangles: DE, Li, Z1, Z2
    __device__ CPF_GLOBAL double *E() const { return p; }
    __device__ CPF_GLOBAL double *DE() const { return p + NBLK * (size_t)n; }
    __device__ CPF_GLOBAL double *rE() const { return DE() + NTRI * (size_t)ne; }
    __device__ CPF_GLOBAL double *X() const { return rE() + NJ * (size_t)ne; }
    __device__ CPF_GLOBAL double *Li() const { return X() + NJ * (size_t)n; }
    __device__ CPF_GLOBAL double *W() const { return Li() + NTRI * (size_t)nod; }
    __device__ CPF_GLOBAL double *V() const { return W() + NBLK * (size_t)nod; }
    __device__ CPF_GLOBAL double *Z1() const { return V() + NBLK * (size_t)nod; }
    __device__ CPF_GLOBAL double *Z2() const { return Z1() + NTRI * (size_t)nod; }
    __device__ CPF_GLOBAL double *s() const { return Z2() + NTRI * (size_t)nod; }
    __device__ CPF_GLOBAL double *c1() const { return s() + NJ * (size_t)nod; }
    __device__ CPF_GLOBAL double *c2() const { return c1() + NJ * (size_t)nod; }
};

__device__ __forceinline__ CRLevel cr_level(CPF_GLOBAL double *base, int T, int lev) {
    int n = T;
    size_t off = 0;
    for (int l = 0; l < lev; ++l) {
        off += cr_level_doubles(n, NJ);
        n = (n + 1) / 2;
    }
    CRLevel L;
    L.p = base + off;
    L.n = n;
    L.no = n / 2;
    L.ne = n - L.no;
    L.nod = L.no > 0 ? L.no : 1;
    return L;
}

__device__ __forceinline__ int cr_top(int T) {
    int lev = 0;
    for (int n = T; n > 1; n = (n + 1) / 2) ++lev;
    return lev;
}

// Block `idx` of an array of whole blocks of `sz` doubles.
__device__ __forceinline__ CPF_GLOBAL double *blk(CPF_GLOBAL double *a, int idx, int sz) {
    return a + (size_t)idx * sz;
}
__device__ __forceinline__ const CPF_GLOBAL double *blk(const CPF_GLOBAL double *a, int idx, int sz) {
    return a + (size_t)idx * sz;
}

// In place: the packed lower triangle of an SPD block becomes the inverse of
// its Cholesky factor.  Reciprocal square roots: hardware estimate and two
// Newton steps.  ok becomes false on a pivot that is not positive.
__device__ __forceinline__ void chol_inverse(double a[NTRI], bool &ok) {
    double rd[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        double d = a[tri_index(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d = fma(-a[tri_index(j, k)], a[tri_index(j, k)], d);
        ok = ok && (d > 0.0);
        const double dd = d > 0.0 ? d : 1.0;
        double r = __builtin_amdgcn_rsq(dd);
        r = r * fma(-0.5 * dd, r * r, 1.5);
        r = r * fma(-0.5 * dd, r * r, 1.5);
        rd[j] = r;
#pragma unroll
        for (int i = j + 1; i < NJ; ++i) {
            double s = a[tri_index(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s = fma(-a[tri_index(i, k)], a[tri_index(j, k)], s);
            a[tri_index(i, j)] = s * r;
        }
    }
    // L^{-1}, column by column: M_jj = 1 / L_jj, M_ij = -(sum_{k=j}^{i-1} L_ik M_kj) / L_ii.
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        a[tri_index(j, j)] = rd[j];
#pragma unroll
        for (int i = j + 1; i < NJ; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) s = fma(a[tri_index(i, k)], a[tri_index(k, j)], s);
            a[tri_index(i, j)] = -s * rd[i];
        }
    }
}

// y = M x and y = M^T x for a packed lower-triangular M.
__device__ __forceinline__ void tri_mv(const double M[NTRI], const double x[NJ], double y[NJ]) {
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= a; ++k) s = fma(M[tri_index(a, k)], x[k], s);
        y[a] = s;
    }
}
__device__ __forceinline__ void tri_tmv(const double M[NTRI], const double x[NJ], double y[NJ]) {
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
        double s = 0.0;
#pragma unroll
        for (int k = a; k < NJ; ++k) s = fma(M[tri_index(k, a)], x[k], s);
        y[a] = s;
    }
}

// A symmetric or lower-triangular NJ x NJ block kept as its packed lower
// triangle (NTRI doubles, row by row): loaded, stored (scaled), and the
// position of element (i, j) of a symmetric one.
__device__ __forceinline__ void ld_packed(const CPF_GLOBAL double *b, double m[NTRI]) {
#pragma unroll
    for (int q = 0; q < NTRI; ++q) m[q] = b[q];
}
__device__ __forceinline__ void st_packed(CPF_GLOBAL double *b, const double m[NTRI], double scale) {
#pragma unroll
    for (int q = 0; q < NTRI; ++q) b[q] = scale * m[q];
}
__device__ __forceinline__ int sym_index(int i, int j) { return i >= j ? tri_index(i, j) : tri_index(j, i); }

// Level-0 diagonal block t (lower triangle): w_p J^T J + (w_s c_t + lambda) I.
__device__ __forceinline__ void level0_D(const DevPlan &P, int T, double lam, double ws, int t, double D[NTRI]) {
    ld_packed(blk(P.A, t, NTRI), D);
    const double dg = ws * ((t > 0) + (t + 1 < T)) + lam;
#pragma unroll
    for (int a = 0; a < NJ; ++a) D[tri_index(a, a)] += dg;
}

// Neighbour slots on level lev-1 of block j of level lev: the odd blocks
// 2j+1 (slot j) and 2j-1 (slot j-1); a missing one is read at a valid slot
// and masked, so that all loads of a block are issued together.
struct CRNbr {
    bool has_r, has_l;
    int jr, jl;
};
__device__ __forceinline__ CRNbr cr_nbr(const CRLevel &Lp, int j) {
    CRNbr q;
    q.has_r = 2 * j + 1 < Lp.n;
    q.has_l = j >= 1;
    q.jr = q.has_r ? j : 0;
    q.jl = q.has_l ? j - 1 : 0;
    return q;
}

// Block j of level lev >= 1 (one lane): lower triangle of its diagonal
// block and its right-hand side, formed from level lev-1.
__device__ __forceinline__ void cr_form_lane(const DevPlan &P, int T, double lam, double ws, const CRLevel &Lp, int lev, int j,
                                             bool factor, const CPF_GLOBAL double *rhs, double sgn, double D[NTRI],
                                             double r[NJ]) {
    const CRNbr q = cr_nbr(Lp, j);
    const CPF_GLOBAL double *Z2 = lev == 1 ? Lp.Z1() : Lp.Z2();   // level 0: Z1 = Z2
    const CPF_GLOBAL double *c2 = lev == 1 ? Lp.c1() : Lp.c2();
    if (factor) {
        if (lev == 1) level0_D(P, T, lam, ws, 2 * j, D);
        else ld_packed(blk(Lp.DE(), j, NTRI), D);
        const CPF_GLOBAL double *zr = blk(Lp.Z1(), q.jr, NTRI), *zl = blk(Z2, q.jl, NTRI);
#pragma unroll
        for (int a = 0; a < NJ; ++a)
#pragma unroll
            for (int k = 0; k <= a; ++k) {
                const double vr = zr[tri_index(a, k)], vl = zl[tri_index(a, k)];
                D[tri_index(a, k)] = D[tri_index(a, k)] - (q.has_r ? vr : 0.0) - (q.has_l ? vl : 0.0);
            }
    }
    const CPF_GLOBAL double *cr_ = blk(Lp.c1(), q.jr, NJ), *cl = blk(c2, q.jl, NJ);
    const CPF_GLOBAL double *rb = lev == 1 ? nullptr : blk(Lp.rE(), j, NJ);
#pragma unroll
    for (int e = 0; e < NJ; ++e) {
        const double r0 = lev == 1 ? sgn * rhs[(size_t)e * T + 2 * j] : rb[e];
        const double vr = cr_[e], vl = cl[e];
        r[e] = r0 - (q.has_r ? vr : 0.0) - (q.has_l ? vl : 0.0);
    }
}

// Column c of the diagonal block j of level lev >= 1 and entry c of its
// right-hand side (the share of lane c of a group).
__device__ __forceinline__ void cr_form_col(const DevPlan &P, int T, double lam, double ws, const CRLevel &Lp, int lev, int j,
                                            int c, bool factor, const CPF_GLOBAL double *rhs, double sgn,
                                            double d[NJ], double &rc) {
    const CRNbr q = cr_nbr(Lp, j);
    const CPF_GLOBAL double *Z2 = lev == 1 ? Lp.Z1() : Lp.Z2();
    const CPF_GLOBAL double *c2 = lev == 1 ? Lp.c1() : Lp.c2();
    if (factor) {
        const int t = 2 * j;
        const CPF_GLOBAL double *b0 = lev == 1 ? blk(P.A, t, NTRI) : blk(Lp.DE(), j, NTRI);
        const double dg = lev == 1 ? ws * ((t > 0) + (t + 1 < T)) + lam : 0.0;
        const CPF_GLOBAL double *zr = blk(Lp.Z1(), q.jr, NTRI), *zl = blk(Z2, q.jl, NTRI);
#pragma unroll
        for (int a = 0; a < NJ; ++a) {
            const int e = sym_index(a, c);
            const double v = b0[e] + (a == c ? dg : 0.0);
            const double vr = zr[e], vl = zl[e];
            d[a] = v - (q.has_r ? vr : 0.0) - (q.has_l ? vl : 0.0);
        }
    }
    const double r0 = lev == 1 ? sgn * rhs[(size_t)c * T + 2 * j] : blk(Lp.rE(), j, NJ)[c];
    const double vr = blk(Lp.c1(), q.jr, NJ)[c], vl = blk(c2, q.jl, NJ)[c];
    rc = r0 - (q.has_r ? vr : 0.0) - (q.has_l ? vl : 0.0);
}

// Column c of the coupling E_i of block i of level lev >= 1 (to block i-1)
// and row c of E_{i+1} (zero without a right neighbour).  Level 1's
// couplings are -Z1 of the odd blocks of level 0 between them: symmetric
// packed blocks, so row c equals column c.
__device__ __forceinline__ void cr_coupling_cols(const CRLevel &L, const CRLevel &Lp, int lev, int i, bool right, int c,
                                                 double e[NJ], double f[NJ]) {
    if (lev == 1) {
        const CPF_GLOBAL double *Zl = blk(Lp.Z1(), i - 1, NTRI), *Zr = blk(Lp.Z1(), right ? i : i - 1, NTRI);
#pragma unroll
        for (int k = 0; k < NJ; ++k) {
            const int q = sym_index(k, c);
            e[k] = -1.0 * Zl[q];
            const double fk = Zr[q];
            f[k] = right ? -1.0 * fk : 0.0;
        }
    } else {
        const CPF_GLOBAL double *Ei = blk(L.E(), i, NBLK) + c;
        const CPF_GLOBAL double *Er = blk(L.E(), right ? i + 1 : i, NBLK) + c * NJ;
#pragma unroll
        for (int k = 0; k < NJ; ++k) {
            e[k] = Ei[k * NJ];
            const double fk = Er[k];
            f[k] = right ? fk : 0.0;
        }
    }
}

// Odd block i = 2h+1 of level 0 (one lane): factor and Schur contribution
// (factor only), s and its contribution.
__device__ __forceinline__ void cr_odd_level0(const DevPlan &P, int T, double lam, double ws, const CRLevel &L0, int h,
                                              bool factor, const CPF_GLOBAL double *rhs, double sgn, bool &ok) {
    const int i = 2 * h + 1;
    const double w = ws;
    double Li[NTRI];
    if (factor) {
        level0_D(P, T, lam, ws, i, Li);
        chol_inverse(Li, ok);
        st_packed(blk(L0.Li(), h, NTRI), Li, 1.0);
        double Pm[NTRI];   // Li^T Li
#pragma unroll
        for (int a = 0; a < NJ; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                double s = 0.0;
#pragma unroll
                for (int k = a; k < NJ; ++k) s = fma(Li[tri_index(k, a)], Li[tri_index(k, b)], s);
                Pm[tri_index(a, b)] = s;
            }
        // Z1 = Z2 = w^2 Pm; the coupling E' = -Z1 of level 1 is not stored:
        // level 1 reads it from Z1
        st_packed(blk(L0.Z1(), h, NTRI), Pm, w * w);
    } else {
        ld_packed(blk(L0.Li(), h, NTRI), Li);
    }
    double r[NJ], s[NJ], c[NJ];
#pragma unroll
    for (int e = 0; e < NJ; ++e) r[e] = sgn * rhs[(size_t)e * T + i];
    tri_mv(Li, r, s);
    tri_tmv(Li, s, c);
    CPF_GLOBAL double *so = blk(L0.s(), h, NJ), *co = blk(L0.c1(), h, NJ);
#pragma unroll
    for (int e = 0; e < NJ; ++e) {
        so[e] = s[e];
        co[e] = -w * c[e];   // W^T s with W = -w Li
    }
}

// Even block j = 2 jj of level lev >= 1 (one lane): its diagonal block and
// right-hand side, kept for level lev+1 (as block jj).
__device__ __forceinline__ void cr_even(const DevPlan &P, int T, double lam, double ws, const CRLevel &Lp, const CRLevel &L,
                                        int lev, int jj, bool factor, const CPF_GLOBAL double *rhs, double sgn) {
    double D[NTRI], r[NJ];
    cr_form_lane(P, T, lam, ws, Lp, lev, 2 * jj, factor, rhs, sgn, D, r);
    if (factor) st_packed(blk(L.DE(), jj, NTRI), D, 1.0);
    CPF_GLOBAL double *ro = blk(L.rE(), jj, NJ);
#pragma unroll
    for (int e = 0; e < NJ; ++e) ro[e] = r[e];
}

// Last level (one block, one lane): factor (or reuse) and x = Li^T Li r.
__device__ __forceinline__ void cr_top_solve(const DevPlan &P, int T, double lam, double ws, const CRLevel &Lp,
                                             const CRLevel &L, int lev, bool factor, const CPF_GLOBAL double *rhs,
                                             double sgn, CPF_GLOBAL double *out, bool &ok) {
    double Li[NTRI], r[NJ], s[NJ], x[NJ];
    if (lev == 0) {   // a single waypoint
        if (factor) level0_D(P, T, lam, ws, 0, Li);
#pragma unroll
        for (int e = 0; e < NJ; ++e) r[e] = sgn * rhs[(size_t)e * T];
    } else {
        cr_form_lane(P, T, lam, ws, Lp, lev, 0, factor, rhs, sgn, Li, r);
    }
    if (factor) {
        chol_inverse(Li, ok);
        st_packed(blk(L.Li(), 0, NTRI), Li, 1.0);
    } else {
        ld_packed(blk(L.Li(), 0, NTRI), Li);
    }
    tri_mv(Li, r, s);
    tri_tmv(Li, s, x);
#pragma unroll
    for (int e = 0; e < NJ; ++e) {
        if (lev == 0) out[(size_t)e * T] = x[e];
        else blk(L.X(), 0, NJ)[e] = x[e];
    }
}

__device__ __forceinline__ void group_sync() { __builtin_amdgcn_wave_barrier(); }

// Odd block i = 2h+1 of level lev >= 1, factor round (group, lane c).
__device__ __forceinline__ void cr_odd_factor(const DevPlan &P, int T, double lam, double ws, const CRLevel &Lp,
                                              const CRLevel &L, const CRLevel &Ln, int lev, int h, int c,
                                              const CPF_GLOBAL double *rhs, double sgn, double *ex, bool &ok) {
    const int i = 2 * h + 1;
    const bool right = i + 1 < L.n;
    // column c of E_i and row c of E_{i+1}, loaded first (used after the
    // factor); on level 1, E_i = -Z1 of odd block i-1 of level 0 (symmetric)
    double e[NJ], f[NJ];
    cr_coupling_cols(L, Lp, lev, i, right, c, e, f);
    // the group forms D_i and r_i column by column and shares them
    {
        double d[NJ], rc;
        cr_form_col(P, T, lam, ws, Lp, lev, i, c, true, rhs, sgn, d, rc);
#pragma unroll
        for (int a = 0; a < NJ; ++a) ex[a * NJ + c] = d[a];
        ex[NBLK + c] = rc;
    }
    group_sync();
    double Li[NTRI], r[NJ], s[NJ];
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) Li[tri_index(a, b)] = ex[a * NJ + b];
        r[a] = ex[NBLK + a];
    }
    group_sync();   // ex is rewritten below
    chol_inverse(Li, ok);
    tri_mv(Li, r, s);
    // column c of W = Li E_i and of V = Li E_{i+1}^T (row c of E_{i+1})
    double w[NJ], v[NJ];
    tri_mv(Li, e, w);
    tri_mv(Li, f, v);
    CPF_GLOBAL double *Wc = blk(L.W(), h, NBLK) + c, *Vc = blk(L.V(), h, NBLK) + c;
    double c1 = 0.0, c2 = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        c1 = fma(w[k], s[k], c1);
        c2 = fma(v[k], s[k], c2);
        Wc[k * NJ] = w[k];
        Vc[k * NJ] = v[k];
        ex[k * NJ + c] = w[k];
        ex[NBLK + k * NJ + c] = v[k];
    }
    blk(L.c1(), h, NJ)[c] = c1;
    blk(L.c2(), h, NJ)[c] = c2;
    // Li (packed lower triangle) column c and s_c by lane c, picked out of
    // the registers every lane of the group holds
    CPF_GLOBAL double *Lo = blk(L.Li(), h, NTRI) + c;
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
        double lv = Li[tri_index(a, 0)];
#pragma unroll
        for (int b = 1; b <= a; ++b) lv = c == b ? Li[tri_index(a, b)] : lv;
        if (a >= c) Lo[tri_index(a, 0)] = lv;
    }
    double sc = s[0];
#pragma unroll
    for (int a = 1; a < NJ; ++a) sc = c == a ? s[a] : sc;
    blk(L.s(), h, NJ)[c] = sc;
    group_sync();
    // column c of W^T W, V^T V (symmetric: rows a >= c, packed) and -V^T W
    // (the coupling of level lev+1, whole)
    CPF_GLOBAL double *Z1c = blk(L.Z1(), h, NTRI) + c, *Z2c = blk(L.Z2(), h, NTRI) + c;
    CPF_GLOBAL double *Enc = blk(Ln.E(), right ? (i + 1) / 2 : 0, NBLK) + c;
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
        double z1 = 0.0, z2 = 0.0, en = 0.0;
#pragma unroll
        for (int k = 0; k < NJ; ++k) {
            const double wa = ex[k * NJ + a], va = ex[NBLK + k * NJ + a];
            z1 = fma(wa, w[k], z1);
            z2 = fma(va, v[k], z2);
            en = fma(va, w[k], en);
        }
        if (a >= c) {
            Z1c[tri_index(a, 0)] = z1;
            Z2c[tri_index(a, 0)] = z2;
        }
        if (right) Enc[a * NJ] = -en;
    }
    group_sync();   // ex is rewritten by the group's next block
}

// Odd block i = 2h+1 of level lev >= 1 for a further right-hand side
// (group, lane c): s = Li r and its contributions through W and V.
__device__ __forceinline__ void cr_odd_rhs(const DevPlan &P, int T, const CRLevel &Lp, const CRLevel &L, int lev,
                                           int h, int c, const CPF_GLOBAL double *rhs, double sgn, double *ex) {
    const int i = 2 * h + 1;
    // row c of Li and column c of W and V, loaded with the right-hand side
    // (Li packed: its row c starts at tri_index(c, 0); the loads past the
    // diagonal stay inside the block and are replaced by zero)
    const CPF_GLOBAL double *Lr = blk(L.Li(), h, NTRI) + tri_index(c, 0);
    const CPF_GLOBAL double *Wc = blk(L.W(), h, NBLK) + c, *Vc = blk(L.V(), h, NBLK) + c;
    double lr[NJ], wc[NJ], vc[NJ];
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const double l = Lr[k];
        lr[k] = k <= c ? l : 0.0;   // zero above the diagonal
        wc[k] = Wc[k * NJ];
        vc[k] = Vc[k * NJ];
    }
    double d[NJ], rc;
    cr_form_col(P, T, 0.0, 0.0, Lp, lev, i, c, false, rhs, sgn, d, rc);
    ex[c] = rc;
    group_sync();
    double sc = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) sc = fma(lr[k], ex[k], sc);
    group_sync();
    ex[c] = sc;
    blk(L.s(), h, NJ)[c] = sc;
    group_sync();
    double c1 = 0.0, c2 = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const double sk = ex[k];
        c1 = fma(wc[k], sk, c1);
        c2 = fma(vc[k], sk, c2);
    }
    blk(L.c1(), h, NJ)[c] = c1;
    blk(L.c2(), h, NJ)[c] = c2;
    group_sync();
}

// Back-substitution of odd block i = 2h+1 of level lev >= 1 (group, lane c):
// y_c = s_c - (W x_{i-1})_c - (V x_{i+1})_c, then x_c = (Li^T y)_c.
__device__ __forceinline__ void cr_back_group(const CRLevel &L, const CRLevel &Ln, int h, int c, double *ex) {
    const int i = 2 * h + 1;
    const bool right = i + 1 < L.n;
    const CPF_GLOBAL double *xl = blk(Ln.X(), (i - 1) / 2, NJ), *xr = blk(Ln.X(), right ? (i + 1) / 2 : 0, NJ);
    const CPF_GLOBAL double *Wr = blk(L.W(), h, NBLK) + c * NJ, *Vr = blk(L.V(), h, NBLK) + c * NJ;
    // column c of Li (packed; the loads above the diagonal stay inside the
    // block and are replaced by zero)
    const CPF_GLOBAL double *Lc = blk(L.Li(), h, NTRI) + c;
    double lc[NJ];
#pragma unroll
    for (int a = 0; a < NJ; ++a) {
        const double l = Lc[tri_index(a, 0)];
        lc[a] = a >= c ? l : 0.0;   // zero above the diagonal
    }
    double acc = blk(L.s(), h, NJ)[c];
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const double vr = xr[k];
        acc = fma(-Wr[k], xl[k], acc);
        acc = fma(-Vr[k], right ? vr : 0.0, acc);
    }
    ex[c] = acc;
    group_sync();
    double x = 0.0;
#pragma unroll
    for (int a = 0; a < NJ; ++a) x = fma(lc[a], ex[a], x);
    blk(L.X(), i, NJ)[c] = x;
    group_sync();
}

// Back-substitution, one lane per block: odd blocks of level 0,
// x_i = Li^T (s_i + w Li (x_{i-1} + x_{i+1})), and the even blocks of any
// level (copied from the level above).
__device__ __forceinline__ void cr_back_lane(const DevPlan &P, int T, double ws, const CRLevel &L, const CRLevel &Ln, int lev,
                                             int x, CPF_GLOBAL double *out) {
    double xv[NJ];
    if (lev == 0 && (x & 1)) {
        const int i = x, h = (i - 1) / 2;
        const bool right = i + 1 < L.n;
        const CPF_GLOBAL double *xl = blk(Ln.X(), (i - 1) / 2, NJ), *xr = blk(Ln.X(), right ? (i + 1) / 2 : 0, NJ);
        const CPF_GLOBAL double *so = blk(L.s(), h, NJ);
        double u[NJ], v[NJ], y[NJ], Li[NTRI];
#pragma unroll
        for (int e = 0; e < NJ; ++e) {
            const double vr = xr[e];
            u[e] = xl[e] + (right ? vr : 0.0);
        }
        ld_packed(blk(L.Li(), h, NTRI), Li);
        tri_mv(Li, u, v);
#pragma unroll
        for (int e = 0; e < NJ; ++e) y[e] = fma(ws, v[e], so[e]);
        tri_tmv(Li, y, xv);
    } else {
        const CPF_GLOBAL double *xs = blk(Ln.X(), x / 2, NJ);
#pragma unroll
        for (int e = 0; e < NJ; ++e) xv[e] = xs[e];
    }
#pragma unroll
    for (int e = 0; e < NJ; ++e) {
        if (lev == 0) out[(size_t)e * T + x] = xv[e];
        else blk(L.X(), x, NJ)[e] = xv[e];
    }
}

// ---------------------------------------------------------------------------
// The small levels in one wavefront.
//
// From the first level of at most CR_TAIL_N = 2 CR_GPW + 1 blocks on (level
// 1 at the earliest), every level's odd blocks fit the groups of a single
// wavefront.  Wavefront 0 then runs all the remaining levels, forward and
// back, with the blocks in LDS and wave barriers between the steps, while
// the other wavefronts wait at the workgroup barrier after it.  The
// arithmetic is that of the rounds above, operation for operation.  Blocks
// are updated in place: block b of the k-th level of the tail lives in slot
// b 2^k of the entry level's arrays, so an even block is already where the
// next level looks for it, and the two Schur contributions to an even block
// are subtracted in two steps (first from its right odd neighbour, then from
// its left one, as the rounds above form it).  The factored blocks (Li, W,
// V whole and s) stay in LDS for further right-hand sides; a level's x goes
// back to global memory only at the entry level, for the rounds below.
// ---------------------------------------------------------------------------

constexpr int CR_TAIL_N = 2 * CR_GPW + 1;      // blocks of the entry level, at most
constexpr int CR_TAIL_FB = 3 * NBLK + NJ;      // LDS doubles per factored block: Li, W, V, s
constexpr int CR_TAIL_FS = CR_TAIL_N * CR_TAIL_FB;
constexpr int CR_TAIL_WK = CR_TAIL_N * (2 * NBLK + 2 * NJ);   // D, E, r, x of the entry level

// First level of the tail: the first with at most CR_TAIL_N blocks, and at
// least 1 (level 0 has its own one-lane-per-block round).
__device__ __forceinline__ int cr_tail_level(int T) {
    int lev = 0;
    for (int n = T; n > CR_TAIL_N; n = (n + 1) / 2) ++lev;
    return lev > 0 ? lev : 1;
}

// Steps of the one-wavefront levels (diagnostic build with CPF_TAIL_STEPS as
// well; the marks change how the compiler schedules these steps): 0 block
// loads, 1 Cholesky and inverse, 2 products with Li and the W, V stores, 3
// Li and s stores, 4 Z columns, 5 left update, 6 right update; 8 entry, 9
// top, 10 back levels, 11 exit.
#ifdef CPF_TAIL_STEPS
#define CR_TAIL_MARK(k) DIAG_MARK(diag_tail[factor ? 0 : 1][k], 1)
#else
#define CR_TAIL_MARK(k) \
    do {                \
    } while (0)
#endif

// The entry level of the tail: the blocks of level lw formed from level
// lw-1 (column c by lane c of a group) into the tail's LDS arrays, by all
// the workgroup's groups at once (a level of at most CR_TAIL_N blocks is one
// round of them); the caller's barrier then hands the arrays to wavefront 0.
__device__ void cr_tail_entry(const DevPlan &P, int T, double lam, double ws, bool factor,
                              const CPF_GLOBAL double *rhs, double sgn, CPF_GLOBAL double *base, int lw, int gid,
                              int c, double *wk) {
    double *D = wk, *E = D + CR_TAIL_N * NBLK, *R = E + CR_TAIL_N * NBLK;
    const CRLevel Lp = cr_level(base, T, lw - 1), L = cr_level(base, T, lw);
    if (gid < 0) return;
    for (int j = gid; j < L.n; j += CR_GROUPS) {
        double d[NJ], rc;
        cr_form_col(P, T, lam, ws, Lp, lw, j, c, factor, rhs, sgn, d, rc);
        R[j * NJ + c] = rc;
        if (factor) {
#pragma unroll
            for (int a = 0; a < NJ; ++a) D[j * NBLK + a * NJ + c] = d[a];
            if (j >= 1) {   // E_j, column c
                double e[NJ], f[NJ];
                cr_coupling_cols(L, Lp, lw, j, false, c, e, f);
#pragma unroll
                for (int k = 0; k < NJ; ++k) E[j * NBLK + k * NJ + c] = e[k];
            }
        }
    }
}

// Wavefront 0 only (lanes in groups of NJ; with 7 joints lane 63 idles).  Solves
// levels lw..top of the system whose levels below lw are in `base`,
// factoring them first (factor) or reusing the factored blocks in fs; the
// entry level's blocks are in wk already (cr_tail_entry).
__device__ void cr_tail(const DevPlan &P, int T, double lam, double ws, bool factor, const CPF_GLOBAL double *rhs,
                        double sgn, CPF_GLOBAL double *base, int lw, double *fs, double *wk, bool &ok) {
    const int lane = threadIdx.x & 63;
    const int g = lane < CR_GL ? lane / NJ : CR_GPW;   // an idle lane: a group that never has a block
    const int c = lane < CR_GL ? lane % NJ : 0;
    double *D = wk, *E = D + CR_TAIL_N * NBLK, *R = E + CR_TAIL_N * NBLK, *X = R + CR_TAIL_N * NJ;
    const CRLevel L = cr_level(base, T, lw);
    const int n = L.n;

    group_sync();
    CR_TAIL_MARK(8);

    // Forward: level by level up to the single top block.
    int nk = n, st = 1, fb = 0;
    for (; nk > 1; fb += nk / 2, nk = (nk + 1) / 2, st *= 2) {
        const int no = nk / 2;
        const int i = 2 * g + 1;
        const bool mine = g < no, right = i + 1 < nk;
        const int pi = i * st, pl = (i - 1) * st, pr = right ? (i + 1) * st : pi;
        double *F = fs + (size_t)(fb + (mine ? g : 0)) * CR_TAIL_FB;
        double *Fl = F, *Fw = F + NBLK, *Fv = F + 2 * NBLK, *Fs = F + 3 * NBLK;
        double z1[NJ], z2[NJ], en[NJ], c1 = 0.0, c2 = 0.0;
        if (mine) {
            if (factor) {
                double Li[NTRI], rv[NJ], e[NJ], f[NJ], s[NJ], w[NJ], v[NJ];
#pragma unroll
                for (int a = 0; a < NJ; ++a) {
#pragma unroll
                    for (int b = 0; b <= a; ++b) Li[tri_index(a, b)] = D[pi * NBLK + a * NJ + b];
                    rv[a] = R[pi * NJ + a];
                }
#pragma unroll
                for (int k = 0; k < NJ; ++k) {
                    e[k] = E[pi * NBLK + k * NJ + c];
                    const double fk = E[pr * NBLK + c * NJ + k];
                    f[k] = right ? fk : 0.0;
                }
                CR_TAIL_MARK(0);
                chol_inverse(Li, ok);
                CR_TAIL_MARK(1);
                tri_mv(Li, rv, s);
                tri_mv(Li, e, w);
                tri_mv(Li, f, v);
#pragma unroll
                for (int k = 0; k < NJ; ++k) {
                    c1 = fma(w[k], s[k], c1);
                    c2 = fma(v[k], s[k], c2);
                    Fw[k * NJ + c] = w[k];
                    Fv[k * NJ + c] = v[k];
                }
                CR_TAIL_MARK(2);
                // the lower triangle of Li and s, the same values from every
                // lane of the group
#pragma unroll
                for (int a = 0; a < NJ; ++a) {
#pragma unroll
                    for (int b = 0; b <= a; ++b) Fl[a * NJ + b] = Li[tri_index(a, b)];
                    Fs[a] = s[a];
                }
                group_sync();
                CR_TAIL_MARK(3);
                // column c of W^T W, V^T V and -V^T W
#pragma unroll
                for (int a = 0; a < NJ; ++a) {
                    double x1 = 0.0, x2 = 0.0, x3 = 0.0;
#pragma unroll
                    for (int k = 0; k < NJ; ++k) {
                        const double wa = Fw[k * NJ + a], va = Fv[k * NJ + a];
                        x1 = fma(wa, w[k], x1);
                        x2 = fma(va, v[k], x2);
                        x3 = fma(va, w[k], x3);
                    }
                    z1[a] = x1;
                    z2[a] = x2;
                    en[a] = x3;
                }
                CR_TAIL_MARK(4);
            } else {
                // s = Li r_i (row c of Li), shared through Fs, then W^T s and V^T s
                double sc = 0.0;
#pragma unroll
                for (int k = 0; k < NJ; ++k) {
                    const double l = Fl[c * NJ + k];
                    sc = fma(k <= c ? l : 0.0, R[pi * NJ + k], sc);
                }
                group_sync();
                Fs[c] = sc;
                group_sync();
#pragma unroll
                for (int k = 0; k < NJ; ++k) {
                    const double sk = Fs[k];
                    c1 = fma(Fw[k * NJ + c], sk, c1);
                    c2 = fma(Fv[k * NJ + c], sk, c2);
                }
            }
            // left even neighbour: the contribution of its right odd neighbour
            if (factor)
#pragma unroll
                for (int a = 0; a < NJ; ++a) D[pl * NBLK + a * NJ + c] -= z1[a];
            R[pl * NJ + c] -= c1;
        }
        group_sync();
        CR_TAIL_MARK(5);
        if (mine && right) {   // right even neighbour: the contribution of its left odd neighbour
            if (factor)
#pragma unroll
                for (int a = 0; a < NJ; ++a) {
                    D[pr * NBLK + a * NJ + c] -= z2[a];
                    E[pr * NBLK + a * NJ + c] = -en[a];   // coupling of level k+1 (slot of block i+1)
                }
            R[pr * NJ + c] -= c2;
        }
        group_sync();
        CR_TAIL_MARK(6);
    }

    // Top block (slot 0): x = Li^T Li r, by group 0.
    if (g == 0) {
        double *Fl = fs + (size_t)fb * CR_TAIL_FB;
        double Li[NTRI], rv[NJ], s[NJ], x[NJ];
#pragma unroll
        for (int a = 0; a < NJ; ++a) rv[a] = R[a];
        if (factor) {
#pragma unroll
            for (int a = 0; a < NJ; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) Li[tri_index(a, b)] = D[a * NJ + b];
            chol_inverse(Li, ok);
#pragma unroll
            for (int a = 0; a < NJ; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) Fl[a * NJ + b] = Li[tri_index(a, b)];
        } else {
#pragma unroll
            for (int a = 0; a < NJ; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) Li[tri_index(a, b)] = Fl[a * NJ + b];
        }
        tri_mv(Li, rv, s);
        tri_tmv(Li, s, x);
#pragma unroll
        for (int a = 0; a < NJ; ++a) X[a] = x[a];
    }
    group_sync();
    CR_TAIL_MARK(9);

    // Back: x_i = Li^T (s_i - W x_{i-1} - V x_{i+1}) for the odd blocks, from
    // the level below the top down to the entry level.
    while (st > 1) {
        st /= 2;
        // the level with slot stride st: its block count and first factored block
        int m = n, f0 = 0;
        for (int s2 = 1; s2 < st; s2 *= 2) {
            f0 += m / 2;
            m = (m + 1) / 2;
        }
        const int i = 2 * g + 1;
        if (g < m / 2) {
            const bool right = i + 1 < m;
            const int pi = i * st, pl = (i - 1) * st, pr = right ? (i + 1) * st : pl;
            const double *F = fs + (size_t)(f0 + g) * CR_TAIL_FB;
            const double *Fl = F, *Fw = F + NBLK, *Fv = F + 2 * NBLK, *Fs = F + 3 * NBLK;
            double acc = Fs[c];
#pragma unroll
            for (int k = 0; k < NJ; ++k) {
                const double xr = X[pr * NJ + k];
                acc = fma(-Fw[c * NJ + k], X[pl * NJ + k], acc);
                acc = fma(-Fv[c * NJ + k], right ? xr : 0.0, acc);
            }
            X[pi * NJ + c] = acc;
            group_sync();
            double x = 0.0;
#pragma unroll
            for (int a = 0; a < NJ; ++a) {
                const double l = Fl[a * NJ + c];
                x = fma(a >= c ? l : 0.0, X[pi * NJ + a], x);
            }
            group_sync();
            X[pi * NJ + c] = x;
        }
        group_sync();
        CR_TAIL_MARK(10);
    }

    // x of the entry level for the back-substitution rounds below it
    if (g < CR_GPW)
        for (int j = g; j < n; j += CR_GPW) blk(L.X(), j, NJ)[c] = X[j * NJ + c];
    CR_TAIL_MARK(11);
}

#define CR_ROUND_MARK(kind, r) DIAG_MARK(diag_round[kind][(r) & 63], 1)

// Solve H x = sgn * rhs ([NJ][T]), factoring H first (factor = true) or
// reusing the stored factors; x goes to out ([NJ][T], may alias rhs: the
// right-hand side is read only in the first two forward rounds).  Returns
// false on a pivot that is not positive.  All threads of the workgroup;
// exch: CR_GROUPS x CR_EX doubles of LDS; tfs, twk: CR_TAIL_FS and
// CR_TAIL_WK doubles of LDS for the small levels (tfs kept between the
// factoring solve and the further right-hand sides).
__device__ __forceinline__ bool cr_solve(const DevPlan &P, int T, double lam, double ws, bool factor,
                                         const CPF_GLOBAL double *rhs, double sgn, CPF_GLOBAL double *out,
                                         int *bad, double *exch, double *tfs, double *twk) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int gid = lane < CR_GL ? (tid >> 6) * CR_GPW + lane / NJ : -1;
    const int gc = lane < CR_GL ? lane % NJ : 0;
    double *ex = exch + (size_t)(gid >= 0 ? gid : 0) * CR_EX;
    const int top = cr_top(T);
    // levels below lw run as workgroup rounds, lw..top in wavefront 0
    // (a single waypoint: level 0 is the top, solved by one lane)
    const int lw = top >= 1 ? cr_tail_level(T) : 1;
    CPF_GLOBAL double *base = P.cr;
    bool ok = true;
    if (tid == 0) *bad = 0;
    DIAG_MARK(diag_phase[7], 1);   // (restarts the rounds' clock)
    // forward rounds
    for (int lev = 0; lev < lw; ++lev) {
        const CRLevel L = cr_level(base, T, lev);
        const CRLevel Lp = cr_level(base, T, lev > 0 ? lev - 1 : 0);
        if (lev == top) {
            if (tid == 0) cr_top_solve(P, T, lam, ws, Lp, L, lev, factor, rhs, sgn, out, ok);
        } else if (lev == 0) {
            for (int h = tid; h < L.no; h += LM_BS) cr_odd_level0(P, T, lam, ws, L, h, factor, rhs, sgn, ok);
        } else {
            const CRLevel Ln = cr_level(base, T, lev + 1);
            if (gid >= 0) {
                for (int h = gid; h < L.no; h += CR_GROUPS) {
                    if (factor) cr_odd_factor(P, T, lam, ws, Lp, L, Ln, lev, h, gc, rhs, sgn, ex, ok);
                    else cr_odd_rhs(P, T, Lp, L, lev, h, gc, rhs, sgn, ex);
                }
            }
            // even blocks from the last wavefronts down, so that on small levels
            // they run beside the groups (which start at the first wavefront)
            for (int x = LM_BS - 1 - tid; x < L.ne; x += LM_BS) cr_even(P, T, lam, ws, Lp, L, lev, x, factor, rhs, sgn);
        }
        __syncthreads();
        CR_ROUND_MARK(factor ? 0 : 1, lev);
    }
    if (top >= 1) {
        cr_tail_entry(P, T, lam, ws, factor, rhs, sgn, base, lw, gid, gc, twk);
        __syncthreads();
        if (tid < 64) cr_tail(P, T, lam, ws, factor, rhs, sgn, base, lw, tfs, twk, ok);
        __syncthreads();
        CR_ROUND_MARK(factor ? 0 : 1, 31);
    }
    if (!ok) *bad = 1;
    // back-substitution rounds below the tail
    for (int lev = top >= 1 ? lw - 1 : -1; lev >= 0; --lev) {
        const CRLevel L = cr_level(base, T, lev);
        const CRLevel Ln = cr_level(base, T, lev + 1);
        if (lev == 0) {
            for (int x = tid; x < L.n; x += LM_BS) cr_back_lane(P, T, ws, L, Ln, 0, x, out);
        } else {
            if (gid >= 0)
                for (int h = gid; h < L.no; h += CR_GROUPS) cr_back_group(L, Ln, h, gc, ex);
            for (int x = 2 * (LM_BS - 1 - tid); x < L.n; x += 2 * LM_BS) cr_back_lane(P, T, ws, L, Ln, lev, x, out);
        }
        __syncthreads();
        CR_ROUND_MARK(factor ? 0 : 1, 32 + lev);
    }
    __syncthreads();
    return *bad == 0;
}

// Block-diagonal case (no differencing term, w_s = 0: the schedule's pose
// step, Sec. III-C): each waypoint solves D_t x_t = sgn rhs_t on its own,
// one lane per waypoint, refactoring for every right-hand side (an NJ x NJ
// Cholesky is cheaper than storing and reloading it).  out may alias rhs.
// Returns false on a pivot that is not positive.  All threads.
__device__ __forceinline__ bool diag_solve(const DevPlan &P, int T, double lam, const CPF_GLOBAL double *rhs,
                                           double sgn, CPF_GLOBAL double *out, int *bad) {
    if (threadIdx.x == 0) *bad = 0;
    __syncthreads();
    bool ok = true;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double D[NTRI], b[NJ], y[NJ], x[NJ];
        level0_D(P, T, lam, 0.0, t, D);
        chol_inverse(D, ok);
#pragma unroll
        for (int j = 0; j < NJ; ++j) b[j] = sgn * rhs[(size_t)j * T + t];
        tri_mv(D, b, y);
        tri_tmv(D, y, x);
#pragma unroll
        for (int j = 0; j < NJ; ++j) out[(size_t)j * T + t] = x[j];
    }
    if (!ok) *bad = 1;
    __syncthreads();
    return *bad == 0;
}

// rb_t = -g_t - (H dx)_t  for every waypoint (all lanes).
__device__ __forceinline__ void refine_residual(const DevPlan &P, int T, double lam, double ws) {
    const double w = ws;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double d[NJ], A[NTRI];
#pragma unroll
        for (int c = 0; c < NJ; ++c) d[c] = P.dx[(size_t)c * T + t];
        ld_packed(blk(P.A, t, NTRI), A);
        const int ct = (t > 0) + (t + 1 < T);
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
            double h = 0.0;
#pragma unroll
            for (int c = 0; c < NJ; ++c) {
                double v = A[sym_index(r, c)];   // element (r, c) of D_t = A_t + (w_s c_t + lambda) I
                if (r == c) v += ws * ct + lam;
                h += v * d[c];
            }
            if (t > 0) h -= w * P.dx[(size_t)r * T + t - 1];
            if (t + 1 < T) h -= w * P.dx[(size_t)r * T + t + 1];
            P.rb[(size_t)r * T + t] = -P.g[(size_t)r * T + t] - h;
        }
    }
}

// FP64 pose errors of waypoint t of X against its target (the Sec. II
// metrics): position distance and geodesic rotation angle.
template <bool PR>
__device__ __forceinline__ void pose_err_fp64(const DevPlan &P, const RobotT<double> &rb,
                                              const CPF_GLOBAL double *X, int T, int t, double *ep,
                                              double *er) {
    double q[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = X[(size_t)j * T + t];
    double Xc[3], Yc[3], Zc[3], p[3], Zs[NJ][3], Os[NJ][3];
    chain<double, false, PR>(rb, q, Xc, Yc, Zc, p, Zs, Os);
    double tg[12];
    load_target<double>(P, T, t, tg);
    const double dx = p[0] - tg[0], dy = p[1] - tg[1], dz = p[2] - tg[2];
    *ep = sqrt(dx * dx + dy * dy + dz * dz);
    // E = R R*^T; angle from its skew part and trace
    double E[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            E[a * 3 + b] = Xc[a] * tg[3 + b * 3 + 0] + Yc[a] * tg[3 + b * 3 + 1] + Zc[a] * tg[3 + b * 3 + 2];
    const double v0 = 0.5 * (E[7] - E[5]), v1 = 0.5 * (E[2] - E[6]), v2 = 0.5 * (E[3] - E[1]);
    *er = atan2(sqrt(v0 * v0 + v1 * v1 + v2 * v2), 0.5 * (E[0] + E[4] + E[8] - 1.0));
}

// Validity check of the alternating schedule (Sec. III-C's anytime result
// under the Sec. II thresholds), FP64 kinematics: every waypoint within the
// position and rotation thresholds, no joint step above the step threshold of
// its joint type and, with collision geometry, no capsule distance below
// zero (Sec. II
// collision avoidance).  A trajectory that passes is copied to xv and
// counted.  Returns
// the next step's objective to all lanes: 1 (differencing) when the pose
// thresholds hold, else 0 (pose).
template <bool COLL, bool PR>
__device__ int schedule_check(const DevPlan &P, LMState *st, int T, double *red) {
    const RobotT<double> rb = load_robot<double, PR>(P);
    // mj: for an all-revolute chain the largest step; with a prismatic joint
    // 1 when some joint steps beyond the threshold of its type, else 0
    double ep = 0.0, er = 0.0, mj = 0.0, len = 0.0, pen = 0.0;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double a, b;
        pose_err_fp64<PR>(P, rb, P.xi, T, t, &a, &b);
        ep = fmax(ep, a);
        er = fmax(er, b);
        if (COLL) {   // deepest penetration, as a positive number
            double q[NJ], dm[2], g[2][NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) q[j] = P.xi[(size_t)j * T + t];
            coll_distances<double, false, double, PR>(rb, P.cap, P.n_obs, P.obs, q, dm, g);
            pen = fmax(pen, fmax(-dm[0], -dm[1]));
        }
        if (t + 1 < T)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const double d = fabs(P.xi[(size_t)j * T + t + 1] - P.xi[(size_t)j * T + t]);
                if constexpr (!PR) mj = fmax(mj, d);
                else if (d > P.vtol[is_prismatic(rb.prism, j) ? 3 : 2]) mj = 1.0;
                len += d;
            }
    }
    double mx[4] = {ep, er, mj, pen};
    block_reduce_n<4, true>(mx, red);
    ep = mx[0];
    er = mx[1];
    mj = mx[2];
    if (COLL) pen = mx[3];
    len = block_sum(len, red);
    const bool pose_ok = ep <= P.vtol[0] && er <= P.vtol[1];
    if constexpr (!PR) {
        if (pose_ok && mj <= P.vtol[2] && pen <= 0.0) {
            for (int e = threadIdx.x; e < NJ * T; e += LM_BS) P.xv[e] = P.xi[e];
            if (threadIdx.x == 0) {
                st->n_valid += 1;
                if (st->first_valid < 0) st->first_valid = st->iters_done;
                st->valid_length = len;
            }
        }
    } else {
        if (pose_ok && mj == 0.0 && pen <= 0.0) {
            for (int e = threadIdx.x; e < NJ * T; e += LM_BS) P.xv[e] = P.xi[e];
            if (threadIdx.x == 0) {
                st->n_valid += 1;
                if (st->first_valid < 0) st->first_valid = st->iters_done;
                st->valid_length = len;
            }
        }
    }
    return pose_ok ? 1 : 0;
}

// One instance per precision, objective kind (the weighted sum, or the
// alternating schedule) and geometry (an all-revolute chain, collision
// capsules, a chain with a prismatic joint), so that the schedule's state,
// the collision terms and the joint-type selects add nothing to the plain
// iteration.  Plans with capsules are all-revolute (COLL implies !PR).
template <typename S, bool SCHED, bool COLL, bool PR>
__global__ __launch_bounds__(LM_BS) void lm_kernel(const DevPlan *__restrict__ plans, int iters, int tick_budget) {
    static_assert(!(COLL && PR), "plans with capsules are all-revolute");
    constexpr int PREC = sizeof(S) == sizeof(double) ? 1 : 0;
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T;
    // empty slot, or a plan of another precision, objective kind, geometry or
    // chain length
    if (T <= 0 || P.prec != PREC || (P.schedule != 0) != SCHED || (P.has_coll != 0) != COLL ||
        (!COLL && (P.prism != 0) != PR) || P.dof != NJ)
        return;
    {
        const LMState *s0 = P.st;
        if (s0->seeded && s0->iters_target > 0 && s0->iters_done >= s0->iters_target) return;
    }
    __shared__ double red[LM_BS];
    __shared__ double sh_lam, sh_nu, sh_cost;
    __shared__ int sh_flags[4];   // 0 need_lin, 1 status, 2 accept, 3 pivot failure
    __shared__ int sh_sched[3];   // 0 checked, 1 next objective, 2 objective of the last step
    const int tid = threadIdx.x;
    constexpr bool sched = SCHED;
    LMState *st = P.st;
    const double wc_all = COLL ? P.w_coll : 0.0;   // weight of the collision residuals
    // the mixed arm keeps the FP64 residual rows of xi (and of the trial point)
    constexpr bool keep_r = sizeof(S) != sizeof(double);

    if (tid == 0) sh_flags[2] = st->seeded;
    __syncthreads();
    if (sh_flags[2] == 0) {   // first call after the search: clamp, initial cost
        for (int t = tid; t < T; t += LM_BS)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                double v = P.xi[(size_t)j * T + t];
                v = v < P.lo[j] ? P.lo[j] : v;
                v = v > P.hi[j] ? P.hi[j] : v;
                P.xi[(size_t)j * T + t] = v;
            }
        __syncthreads();
        const double c0 = plan_cost<PR>(P, P.xi, T, red, P.w_p, P.w_s, wc_all, keep_r ? P.rr : nullptr);
        if (tid == 0) {
            st->nu = 2.0;
            st->cost = c0;
            st->cost0 = c0;
            st->n_acc = 0;
            st->iters_done = 0;
            st->status = 0;
            st->need_lin = 1;
            st->seeded = 1;
            st->grad_inf = 0.0;
            st->valid_length = 0.0;
            st->checked = 0;
            st->mode = 0;
            st->last_mode = -1;
            st->n_valid = 0;
            st->first_valid = -1;
            st->pose_steps = 0;
            st->diff_steps = 0;
        }
        __syncthreads();
    }
    if (tid == 0) {
        sh_lam = st->lambda;
        sh_nu = st->nu;
        sh_cost = st->cost;
        sh_sched[0] = st->checked;
        sh_sched[1] = st->mode;
        sh_sched[2] = st->last_mode;
        sh_flags[0] = st->need_lin;
        sh_flags[1] = st->status;
        // iterations this launch: at most what the plan still has to do and,
        // with a tick budget (serving), about tick_budget / (T + LM_ITER_FIXED)
        // (at least one): a serving tick then takes about as long for a plan
        // of any length, so short plans are not held back by long ones
        const int left = st->iters_target > 0 ? st->iters_target - st->iters_done : iters;
        int n = left < iters ? (left > 0 ? left : 0) : iters;
        if (tick_budget > 0) {
            const int cap = tick_budget / (T + LM_ITER_FIXED);
            n = n < (cap > 1 ? cap : 1) ? n : (cap > 1 ? cap : 1);
        }
        sh_flags[2] = n;
    }
    __syncthreads();
    const int n_it = sh_flags[2];

    __shared__ int sh_bad;
    __shared__ double exch[CR_GROUPS * CR_EX];
    __shared__ double tail_fs[CR_TAIL_FS], tail_wk[CR_TAIL_WK];
#ifdef CPF_PHASE_CYCLES
    if (tid == 0) {
        for (int r = 0; r < 64; ++r) diag_round[0][r] = diag_round[1][r] = 0;
        for (int r = 0; r < 12; ++r) diag_tail[0][r] = diag_tail[1][r] = 0;
        for (int r = 0; r < 8; ++r) diag_phase[r] = 0;
        diag_last[0] = diag_last[1] = clock64();
    }
    __syncthreads();
#endif
#define PHASE_MARK(k) DIAG_MARK(diag_phase[k], 0)
    for (int it = 0; it < n_it; ++it) {
        if (sh_flags[1] != 0) break;
        // Objective of this step: the weighted sum, or under the schedule the
        // pose term alone until the pose thresholds hold, then the
        // differencing term alone (re-decided by a check before every step).
        // The differencing step keeps the fixed damping lambda0: its
        // objective is quadratic, so the gain-ratio rule would only drive
        // lambda to its floor and one step would then flatten the path.
        int m = 0;
        double wp = P.w_p, ws = P.w_s, wc = wc_all;
        if (sched) {
            if (!sh_sched[0]) {
                const int nm = schedule_check<COLL, PR>(P, st, T, red);
                if (tid == 0) {
                    sh_sched[0] = 1;
                    sh_sched[1] = nm;
                }
                __syncthreads();
            }
            m = sh_sched[1];
            wp = m ? 0.0 : P.w_p;
            ws = m ? P.w_s : 0.0;
            wc = m ? wc_all : 0.0;
            if (m != sh_sched[2]) {   // new objective: its cost and linearisation
                // (the barriers inside plan_cost order every lane's read of
                // sh_sched[2] before lane 0 rewrites it)
                const double c = plan_cost<PR>(P, P.xi, T, red, wp, ws, wc, keep_r ? P.rr : nullptr);
                if (tid == 0) {
                    sh_cost = c;
                    sh_flags[0] = 1;
                    sh_sched[2] = m;
                }
                __syncthreads();
            }
        }
        const double lam = m ? P.lam0 : sh_lam;
        if (sh_flags[0]) {
            const double gm = linearise<S, PR>(P, load_robot<S, PR>(P), T, wp, ws, wc);
            const double gmax = block_max(gm, red);
            if (tid == 0) st->grad_inf = gmax;
        }
        __syncthreads();
        PHASE_MARK(0);
        // Solve 0 factors H and solves H dx = -g; each further solve takes
        // the FP64 residual rb = -g - H dx and adds the correction H^-1 rb
        // (one call site, so the solver is inlined once).
        for (int rs = 0; rs <= P.refine_steps; ++rs) {
            const bool first = rs == 0;
            if (!first) {
                refine_residual(P, T, lam, ws);
                __syncthreads();
                PHASE_MARK(3);
            }
            const bool ok = (SCHED && ws == 0.0)
                                ? diag_solve(P, T, lam, first ? P.g : P.rb, first ? -1.0 : 1.0,
                                             first ? P.dx : P.rb, &sh_bad)
                                : cr_solve(P, T, lam, ws, first, first ? P.g : P.rb, first ? -1.0 : 1.0,
                                           first ? P.dx : P.rb, &sh_bad, exch, tail_fs, tail_wk);
            if (first) {
                if (tid == 0) sh_flags[3] = ok ? 0 : 1;
                PHASE_MARK(1);
                __syncthreads();
                if (sh_flags[3]) break;
            } else {
                for (int t = tid; t < T; t += LM_BS)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) P.dx[(size_t)j * T + t] += P.rb[(size_t)j * T + t];
                __syncthreads();
                PHASE_MARK(4);
            }
        }
        if (sh_flags[3]) {
            if (tid == 0) sh_flags[1] = CPF_STATUS_NUMERIC;
            __syncthreads();
            break;
        }
        // Trial point, its cost and the predicted reduction.
        double pr = 0.0;
        for (int t = tid; t < T; t += LM_BS)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const size_t e = (size_t)j * T + t;
                const double dl = P.dx[e];
                double v = P.xi[e] + dl;
                v = v < P.lo[j] ? P.lo[j] : v;
                v = v > P.hi[j] ? P.hi[j] : v;
                P.xt[e] = v;
                pr += dl * (lam * dl - P.g[e]);
            }
        __syncthreads();
        double pr_sum;
        const double cn = plan_cost<PR>(P, P.xt, T, red, wp, ws, wc, keep_r ? P.rt : nullptr, &pr_sum, pr);
        const double pred = 0.5 * pr_sum;
        PHASE_MARK(5);
        if (tid == 0) {
            const double c = sh_cost;
            double l = sh_lam, nu = sh_nu;
            const int acc = cn < c;
            if (m) {
                // differencing step: accept iff it lowers its objective; the
                // pose objective's damping is left as it is
                if (acc) {
                    sh_cost = cn;
                    st->n_acc += 1;
                }
            } else if (acc) {
                const double rho = (c - cn) / pred;
                const double u = 2.0 * rho - 1.0;
                double f = 1.0 - u * u * u;
                if (f < 1.0 / 3.0) f = 1.0 / 3.0;
                l *= f;
                nu = 2.0;
                sh_cost = cn;
                st->n_acc += 1;
            } else {
                l *= nu;
                nu *= 2.0;
            }
            if (l < P.lam_min) l = P.lam_min;
            if (l > P.lam_max) l = P.lam_max;
            if (!m) {
                sh_lam = l;
                sh_nu = nu;
            }
            sh_flags[0] = acc;
            sh_flags[2] = acc;
            st->iters_done += 1;
            if (sched) {
                sh_sched[0] = 0;
                if (m) st->diff_steps += 1;
                else st->pose_steps += 1;
            }
        }
        __syncthreads();
        if (sh_flags[2]) {
            for (int t = tid; t < T; t += LM_BS) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) P.xi[(size_t)j * T + t] = P.xt[(size_t)j * T + t];
                if (keep_r) {
                    const int rows = wc != 0.0 ? RROWS : 6;
                    for (int i = 0; i < rows; ++i) P.rr[(size_t)i * T + t] = P.rt[(size_t)i * T + t];
                }
            }
        }
        __syncthreads();
        PHASE_MARK(6);
    }
#ifdef CPF_PHASE_CYCLES
    if (tid == 0 && blockIdx.x == 0)
        printf("lm phase cycles T=%d iters=%d: lin %llu factor %llu solve %llu refres %llu "
               "refsub %llu trial %llu accept %llu\n",
               T, n_it, diag_phase[0], diag_phase[1], diag_phase[2], diag_phase[3], diag_phase[4],
               diag_phase[5], diag_phase[6]);
#endif
#ifdef CPF_PHASE_CYCLES
    if (tid == 0 && blockIdx.x == 0) {
        for (int k = 0; k < 2; ++k) {
            printf("cr rounds %s:", k ? "rhs" : "factor");
            for (int r = 0; r < 64; ++r)
                if (diag_round[k][r] && r == 31) printf(" tail=%llu", diag_round[k][r]);
                else if (diag_round[k][r]) printf(" %s%d=%llu", r >= 32 ? "b" : "f", r & 31, diag_round[k][r]);
            printf("\n");
        }
        for (int k = 0; k < 2; ++k) {
            printf("tail steps %s:", k ? "rhs" : "factor");
            for (int r = 0; r < 12; ++r)
                if (diag_tail[k][r]) printf(" s%d=%llu", r, diag_tail[k][r]);
            printf("\n");
        }
    }
#endif
#undef PHASE_MARK
    // The check after the last step of the call (the next call's first step
    // then reuses its decision).
    if (sched && sh_flags[1] == 0 && !sh_sched[0]) {
        const int nm = schedule_check<COLL, PR>(P, st, T, red);
        if (tid == 0) {
            sh_sched[0] = 1;
            sh_sched[1] = nm;
        }
    }
    __syncthreads();
    if (tid == 0) {
        st->lambda = sh_lam;
        st->nu = sh_nu;
        st->cost = sh_cost;
        st->need_lin = sh_flags[0];
        st->status = sh_flags[1];
        st->checked = sh_sched[0];
        st->mode = sh_sched[1];
        st->last_mode = sh_sched[2];
    }
}

// Report: FP64 pose error of xi vs the targets and mjac (Sec. II metrics)
// and, with collision geometry, the smallest self and environment distances
// along xi (+inf without).
template <bool COLL, bool PR>
__global__ __launch_bounds__(LM_BS) void eval_kernel(const DevPlan *__restrict__ plans,
                                                     int only_finished) {
    static_assert(!(COLL && PR), "plans with capsules are all-revolute");
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T;
    if (T <= 0 || (P.has_coll != 0) != COLL || (!COLL && (P.prism != 0) != PR) || P.dof != NJ) return;
    if (only_finished) {
        const LMState *s0 = P.st;
        const bool finished = s0->status != 0 ||
                              (s0->iters_target > 0 && s0->iters_done >= s0->iters_target);
        if (!finished || s0->reported) return;
    }
    __shared__ double red[LM_BS];
    const RobotT<double> rb = load_robot<double, PR>(P);
    double ep = 0.0, er = 0.0, mj = 0.0, ns = -__builtin_inf(), ne = -__builtin_inf();
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double a, b;
        pose_err_fp64<PR>(P, rb, P.xi, T, t, &a, &b);
        ep = fmax(ep, a);
        er = fmax(er, b);
        if (t + 1 < T)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                mj = fmax(mj, fabs(P.xi[(size_t)j * T + t + 1] - P.xi[(size_t)j * T + t]));
        if (COLL) {
            double q[NJ], dm[2], g[2][NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) q[j] = P.xi[(size_t)j * T + t];
            coll_distances<double, false, double, PR>(rb, P.cap, P.n_obs, P.obs, q, dm, g);
            ns = fmax(ns, -dm[0]);
            ne = fmax(ne, -dm[1]);
        }
    }
    double mx[5] = {ep, er, mj, ns, ne};
    block_reduce_n<5, true>(mx, red);
    ep = mx[0];
    er = mx[1];
    mj = mx[2];
    if (COLL) {
        ns = mx[3];
        ne = mx[4];
    }
    if (threadIdx.x == 0) {
        P.report[0] = ep;
        P.report[1] = er;
        P.report[2] = mj;
        P.report[3] = -ns;
        P.report[4] = -ne;
        if (only_finished) P.st->reported = 1;
    }
}

template <typename S, bool SCHED>
static void lm_launch_geo(const DevPlan *d_plans, int nplans, int geo, int iters, int budget, hipStream_t s) {
    const dim3 g(nplans), b(LM_BS);
    if (geo == GEO_COLL)
        hipLaunchKernelGGL((lm_kernel<S, SCHED, true, false>), g, b, 0, s, d_plans, iters, budget);
    else if (geo == GEO_PRISM)
        hipLaunchKernelGGL((lm_kernel<S, SCHED, false, true>), g, b, 0, s, d_plans, iters, budget);
    else
        hipLaunchKernelGGL((lm_kernel<S, SCHED, false, false>), g, b, 0, s, d_plans, iters, budget);
}

hipError_t lm_launch(const DevPlan *d_plans, int nplans, int prec, int sched, int geo, int iters, hipStream_t s,
                     int tick_budget) {
    if (nplans <= 0) return hipSuccess;
    if (geo < 0 || geo >= GEO_KINDS) return hipErrorInvalidValue;
    if (prec == 1 && sched)
        lm_launch_geo<double, true>(d_plans, nplans, geo, iters, tick_budget, s);
    else if (prec == 1)
        lm_launch_geo<double, false>(d_plans, nplans, geo, iters, tick_budget, s);
    else if (sched)
        lm_launch_geo<float, true>(d_plans, nplans, geo, iters, tick_budget, s);
    else
        lm_launch_geo<float, false>(d_plans, nplans, geo, iters, tick_budget, s);
    return hipGetLastError();
}

hipError_t eval_launch(const DevPlan *d_plans, int nplans, int only_finished, int geo, hipStream_t s) {
    if (nplans <= 0) return hipSuccess;
    if (geo < 0 || geo >= GEO_KINDS) return hipErrorInvalidValue;
    const dim3 g(nplans), b(LM_BS);
    if (geo == GEO_COLL)
        hipLaunchKernelGGL((eval_kernel<true, false>), g, b, 0, s, d_plans, only_finished);
    else if (geo == GEO_PRISM)
        hipLaunchKernelGGL((eval_kernel<false, true>), g, b, 0, s, d_plans, only_finished);
    else
        hipLaunchKernelGGL((eval_kernel<false, false>), g, b, 0, s, d_plans, only_finished);
    return hipGetLastError();
}

}  // namespace CPF_JNS
}  // namespace cpf
