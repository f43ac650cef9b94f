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
// Kinematics (FK, J, residuals, J^T J) run in S = float or double; the
// assembly, the solve and every cross-waypoint sum are FP64.  The solve is a
// block LDL^T sweep  S_t = D_t - w^2 S_{t-1}^{-1}  on one wavefront (lane
// i*7+j holds element (i, j); 7x7 inverses by Gauss-Jordan), then forward /
// backward substitution, then FP64 iterative refinement against the same H.
#include <float.h>

#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {

constexpr int LM_BS = 512;

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = LM_BS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = LM_BS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <typename S>
__device__ __forceinline__ void load_target(const DevPlan &P, int T, int t, S tg[12]) {
#pragma unroll
    for (int e = 0; e < 12; ++e) tg[e] = (S)P.targets[(size_t)e * T + t];
}

// Squared pose residual of trajectory X ([7][T]) at waypoint t.
template <typename S>
__device__ __forceinline__ double pose_sq(const DevPlan &P, const RobotT<S> &rb, const double *X,
                                          int T, int t) {
    S q[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = (S)X[(size_t)j * T + t];
    S Xc[3], Yc[3], Zc[3], p[3], Zs[NJ][3], Os[NJ][3];
    chain<S, false>(rb, q, Xc, Yc, Zc, p, Zs, Os);
    S tg[12], r[6];
    load_target<S>(P, T, t, tg);
    pose_residual<S>(Xc, Yc, Zc, p, tg, r);
    S s = r[0] * r[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) s += r[i] * r[i];
    return (double)s;
}

// Cost of trajectory X: pose part and smoothness part, block-reduced.
template <typename S>
__device__ __forceinline__ double plan_cost(const DevPlan &P, const RobotT<S> &rb, const double *X,
                                            int T, double *red) {
    double ps = 0.0, ss = 0.0;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        ps += pose_sq<S>(P, rb, X, T, t);
        if (t + 1 < T) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const double d = X[(size_t)j * T + t + 1] - X[(size_t)j * T + t];
                ss += d * d;
            }
        }
    }
    const double pose_sum = block_sum(ps, red);
    const double diff_sum = block_sum(ss, red);
    return 0.5 * P.w_p * pose_sum + 0.5 * P.w_s * diff_sum;
}

// Linearise at xi: A_t = w_p J^T J (packed lower), g_t; returns max |g|.
template <typename S>
__device__ __forceinline__ double linearise(const DevPlan &P, const RobotT<S> &rb, int T) {
    double gmax = 0.0;
    const double w_p = P.w_p, w_s = P.w_s;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double xq[NJ];
        S q[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            xq[j] = P.xi[(size_t)j * T + t];
            q[j] = (S)xq[j];
        }
        S Xc[3], Yc[3], Zc[3], p[3], Zs[NJ][3], Os[NJ][3];
        chain<S, true>(rb, q, Xc, Yc, Zc, p, Zs, Os);
        S tg[12], r[6];
        load_target<S>(P, T, t, tg);
        pose_residual<S>(Xc, Yc, Zc, p, tg, r);
        S J[6][NJ];
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
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                S s = J[0][i] * J[0][j];
#pragma unroll
                for (int k = 1; k < 6; ++k) s += J[k][i] * J[k][j];
                P.A[(size_t)tri_index(i, j) * T + t] = w_p * (double)s;
            }
        }
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            S s = J[0][i] * r[0];
#pragma unroll
            for (int k = 1; k < 6; ++k) s += J[k][i] * r[k];
            double gi = w_p * (double)s;
            double sm = 0.0;
            if (t > 0) sm += xq[i] - P.xi[(size_t)i * T + t - 1];
            if (t + 1 < T) sm += xq[i] - P.xi[(size_t)i * T + t + 1];
            gi += w_s * sm;
            P.g[(size_t)i * T + t] = gi;
            gmax = fmax(gmax, fabs(gi));
        }
    }
    return gmax;
}

// Element (i, j) of D_t = A_t + (w_s c_t + lambda) I.
__device__ __forceinline__ double d_elem(const DevPlan &P, int T, int t, int i, int j, double lam) {
    const int hi = i > j ? i : j, lo = i > j ? j : i;
    double v = P.A[(size_t)tri_index(hi, lo) * T + t];
    if (i == j) {
        const int ct = (t > 0) + (t + 1 < T);
        v += P.w_s * ct + lam;
    }
    return v;
}

// In-place Gauss-Jordan inverse of a symmetric positive definite 7x7 matrix
// spread over a wavefront (lane i*7+j holds element (i, j); lanes >= 49
// carry copies and are ignored).  ok becomes false on a non-positive pivot.
__device__ __forceinline__ double gj_inverse7(double a, int i, int j, bool &ok) {
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const double akk = __shfl(a, k * NJ + k);
        const double aik = __shfl(a, i * NJ + k);
        const double akj = __shfl(a, k * NJ + j);
        ok = ok && (akk > 0.0);
        const double r = 1.0 / akk;
        double na;
        if (i == k) na = (j == k) ? r : akj * r;
        else if (j == k) na = -aik * r;
        else na = a - aik * (akj * r);
        a = na;
    }
    return a;
}

// Product of a lane-distributed 7x7 block (lane r*7+c holds M(r, c)) with a
// vector held in lanes 0..6: lane r < 7 returns (M v)_r.  `col` is the
// lane's column index c; the row sum gathered by lane r is over lanes
// r*7 .. r*7+6.
__device__ __forceinline__ double matvec7(double m, double v, int lane, int col) {
    const double prod = m * __shfl(v, col);
    const int r = lane < NJ ? lane : 0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NJ; ++c) s += __shfl(prod, r * NJ + c);
    return s;
}

// Solve H x = rhs with the stored inverse Schur blocks P[49][T]:
// forward y_t = sign*rhs_t + w P_{t-1} y_{t-1}; backward x_t = P_t (y_t + w x_{t+1}).
// Wave 0 only.  rhs, out are [7][T] (may alias); y is scratch.
__device__ void substitute(const DevPlan &P, int T, const double *rhs, double sign, double *out,
                           int lane) {
    const int j = lane < NBLK ? lane % NJ : 0;
    const int l = lane < NBLK ? lane : 0;
    const double w = P.w_s;
    double yprev = 0.0;
    for (int t = 0; t < T; ++t) {
        double y = lane < NJ ? sign * rhs[(size_t)lane * T + t] : 0.0;
        if (t > 0) {
            const double pm = P.P[(size_t)l * T + t - 1];
            y += w * matvec7(pm, yprev, lane, j);
        }
        if (lane < NJ) P.y[(size_t)lane * T + t] = y;
        yprev = y;
    }
    double xnext = 0.0;
    for (int t = T - 1; t >= 0; --t) {
        const double pm = P.P[(size_t)l * T + t];
        double v = lane < NJ ? P.y[(size_t)lane * T + t] : 0.0;
        if (t + 1 < T) v += w * xnext;
        const double x = matvec7(pm, v, lane, j);
        if (lane < NJ) out[(size_t)lane * T + t] = x;
        xnext = x;
    }
}

// Factor sweep: P_t = (D_t - w^2 P_{t-1})^{-1}, then substitution for -g.
// Wave 0 only.  Returns false on a non-positive pivot.
__device__ bool factor_and_solve(const DevPlan &P, int T, double lam, int lane) {
    const int i = lane < NBLK ? lane / NJ : 0, j = lane < NBLK ? lane % NJ : 0;
    const double w = P.w_s, w2 = w * w;
    bool ok = true;
    double pprev = 0.0;
    double dnext = d_elem(P, T, 0, i, j, lam);
    for (int t = 0; t < T; ++t) {
        const double dcur = dnext;
        if (t + 1 < T) dnext = d_elem(P, T, t + 1, i, j, lam);
        const double s = (t > 0) ? dcur - w2 * pprev : dcur;
        const double pinv = gj_inverse7(s, i, j, ok);
        if (lane < NBLK) P.P[(size_t)lane * T + t] = pinv;
        pprev = pinv;
    }
    substitute(P, T, P.g, -1.0, P.dx, lane);   // right-hand side -g
    return ok;
}

// ---------------------------------------------------------------------------
// Partitioned solve.  The waypoints are split into C contiguous chunks
// [s_c, e_c], one per wavefront.  Within a chunk, block Gaussian elimination
// from s_c onwards treats the previous chunk's last block z_{c-1} = x_{e_{c-1}}
// as an external unknown:
//   S_t x_t - w x_{t+1} = y_t + F_t z_{c-1},  S_t = D_t - w^2 P_{t-1},
//   P_t = S_t^{-1},  y_t = b_t + w P_{t-1} y_{t-1},  F_t = w P_{t-1} F_{t-1},
//   F_{s_c} = w I (zero for the first chunk).
// Back-substituting from the chunk's last block z_c gives, at its first block,
//   x_{s_c} = a_c + G_c z_{c-1} + (F_{e_c}^T / w) z_c,
//   a: a_t = P_t (y_t + w a_{t+1}),  G: G_t = P_t (F_t + w G_{t+1}),  a_e = G_e = 0.
// The last rows of the chunks then form a symmetric block-tridiagonal system
// in z_0 .. z_{C-1} (the Schur complement on the chunk ends):
//   M_c = S_{e_c} - w G_{c+1},  sub-diagonal -F_{e_c},  r_c = y_{e_c} + w a_{c+1},
// solved by one wavefront with the same LDL^T sweep, after which every chunk
// recovers its interior: x_t = P_t (y_t + F_t z_{c-1} + w x_{t+1}).
// ---------------------------------------------------------------------------

constexpr int MAX_CHUNKS = LM_BS / 64;

struct ChunkShared {
    double S[MAX_CHUNKS][NBLK];    // S_{e_c}, then M_c, then Pi_c = Sigma_c^{-1}
    double G[MAX_CHUNKS][NBLK];    // G_c at the chunk's first block
    double y[MAX_CHUNKS][8];       // y_{e_c}, then r_c, then rho_c
    double a[MAX_CHUNKS][8];       // a_c at the chunk's first block
    double z[MAX_CHUNKS][8];       // chunk-end solution z_c
    int bad;
};

__device__ __forceinline__ double matmul7(double A, double B, int i, int j) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) s += __shfl(A, i * NJ + k) * __shfl(B, k * NJ + j);
    return s;
}

__device__ __forceinline__ void chunk_bounds(int T, int C, int c, int &s, int &e) {
    s = (int)(((long long)c * T) / C);
    e = (int)(((long long)(c + 1) * T) / C) - 1;
}

// Factorisation of the partitioned system (all waves; wave c owns chunk c).
// Stores P_t (t < e_c) and F_t for every t, and Pi_c for the chunk ends.
// Returns false on a non-positive pivot (flag in sh.bad).
__device__ bool chunk_factor(const DevPlan &P, int T, int C, double lam, ChunkShared &sh) {
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int i = lane < NBLK ? lane / NJ : 0, j = lane < NBLK ? lane % NJ : 0;
    const int l = lane < NBLK ? lane : 0;
    const double w = P.w_s, w2 = w * w;
    if (threadIdx.x == 0) sh.bad = 0;
    __syncthreads();
    bool ok = true;
    if (c < C) {
        int s, e;
        chunk_bounds(T, C, c, s, e);
        double pprev = 0.0, fprev = 0.0;
        for (int t = s; t <= e; ++t) {
            const double d = d_elem(P, T, t, i, j, lam);
            const double S = (t > s) ? d - w2 * pprev : d;
            double F;
            if (t == s) F = (c > 0 && i == j) ? w : 0.0;
            else F = w * matmul7(pprev, fprev, i, j);
            if (lane < NBLK) P.F[(size_t)lane * T + t] = F;
            if (t == e) {
                if (lane < NBLK) sh.S[c][lane] = S;
            } else {
                const double pinv = gj_inverse7(S, i, j, ok);
                if (lane < NBLK) P.P[(size_t)lane * T + t] = pinv;
                pprev = pinv;
            }
            fprev = F;
        }
        // G at the first block: G_t = P_t (F_t + w G_{t+1}), G_e = 0.
        double G = 0.0;
        for (int t = e - 1; t >= s; --t) {
            const double pm = P.P[(size_t)l * T + t];
            const double f = P.F[(size_t)l * T + t];
            G = matmul7(pm, f + w * G, i, j);
        }
        if (lane < NBLK) sh.G[c][lane] = G;
        if (!ok) sh.bad = 1;
    }
    __syncthreads();
    // Reduced system on the chunk ends (wave 0).
    if (c == 0) {
        double pi_prev = 0.0;
        for (int cc = 0; cc < C; ++cc) {
            int s, e;
            chunk_bounds(T, C, cc, s, e);
            double M = sh.S[cc][l];
            if (cc + 1 < C) M -= w * sh.G[cc + 1][l];
            if (cc > 0) {
                const double Fe = P.F[(size_t)l * T + e];
                const double FePi = matmul7(Fe, pi_prev, i, j);
                M -= matmul7(FePi, __shfl(Fe, j * NJ + i), i, j);   // F Pi F^T
            }
            const double pi = gj_inverse7(M, i, j, ok);
            if (lane < NBLK) sh.S[cc][lane] = pi;
            pi_prev = pi;
        }
        if (!ok) sh.bad = 1;
    }
    __syncthreads();
    return sh.bad == 0;
}

// Solve with the partitioned factors for right-hand side sign*rhs ([7][T]);
// writes out ([7][T], may alias rhs).  All waves.
__device__ void chunk_substitute(const DevPlan &P, int T, int C, const double *rhs, double sign,
                                 double *out, ChunkShared &sh) {
    const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
    const int j = lane < NBLK ? lane % NJ : 0;
    const int l = lane < NBLK ? lane : 0;
    const double w = P.w_s;
    if (c < C) {
        int s, e;
        chunk_bounds(T, C, c, s, e);
        // forward: y_t = b_t + w P_{t-1} y_{t-1} within the chunk
        double yprev = 0.0;
        for (int t = s; t <= e; ++t) {
            double y = lane < NJ ? sign * rhs[(size_t)lane * T + t] : 0.0;
            if (t > s) y += w * matvec7(P.P[(size_t)l * T + t - 1], yprev, lane, j);
            if (lane < NJ) P.y[(size_t)lane * T + t] = y;
            yprev = y;
        }
        if (lane < NJ) sh.y[c][lane] = yprev;
        // backward: a_t = P_t (y_t + w a_{t+1}), a_e = 0
        double a = 0.0;
        for (int t = e - 1; t >= s; --t) {
            const double v = (lane < NJ ? P.y[(size_t)lane * T + t] : 0.0) + w * a;
            a = matvec7(P.P[(size_t)l * T + t], v, lane, j);
        }
        if (lane < NJ) sh.a[c][lane] = a;
    }
    __syncthreads();
    if (c == 0) {
        // rho_c = r_c + F_{e_c} Pi_{c-1} rho_{c-1};  z_c = Pi_c (rho_c + F_{e_{c+1}}^T z_{c+1})
        double rho_prev = 0.0;
        for (int cc = 0; cc < C; ++cc) {
            int s, e;
            chunk_bounds(T, C, cc, s, e);
            double r = lane < NJ ? sh.y[cc][lane] : 0.0;
            if (cc + 1 < C && lane < NJ) r += w * sh.a[cc + 1][lane];
            if (cc > 0) {
                const double v = matvec7(sh.S[cc - 1][l], rho_prev, lane, j);
                r += matvec7(P.F[(size_t)l * T + e], v, lane, j);
            }
            if (lane < NJ) sh.y[cc][lane] = r;
            rho_prev = r;
        }
        double znext = 0.0;
        for (int cc = C - 1; cc >= 0; --cc) {
            double v = lane < NJ ? sh.y[cc][lane] : 0.0;
            if (cc + 1 < C) {
                int s1, e1;
                chunk_bounds(T, C, cc + 1, s1, e1);
                const double Fe = P.F[(size_t)l * T + e1];
                v += matvec7(__shfl(Fe, j * NJ + (lane < NBLK ? lane / NJ : 0)), znext, lane, j);
            }
            const double z = matvec7(sh.S[cc][l], v, lane, j);
            if (lane < NJ) sh.z[cc][lane] = z;
            znext = z;
        }
    }
    __syncthreads();
    if (c < C) {
        int s, e;
        chunk_bounds(T, C, c, s, e);
        const double zl = (c > 0 && lane < NJ) ? sh.z[c - 1][lane] : 0.0;
        double x = lane < NJ ? sh.z[c][lane] : 0.0;
        if (lane < NJ) out[(size_t)lane * T + e] = x;
        for (int t = e - 1; t >= s; --t) {
            double v = (lane < NJ ? P.y[(size_t)lane * T + t] : 0.0) + w * x;
            if (c > 0) v += matvec7(P.F[(size_t)l * T + t], zl, lane, j);
            x = matvec7(P.P[(size_t)l * T + t], v, lane, j);
            if (lane < NJ) out[(size_t)lane * T + t] = x;
        }
    }
    __syncthreads();
}

// rb_t = -g_t - (H dx)_t  for every waypoint (all lanes).
__device__ void refine_residual(const DevPlan &P, int T, double lam) {
    const double w = P.w_s;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double d[NJ];
#pragma unroll
        for (int c = 0; c < NJ; ++c) d[c] = P.dx[(size_t)c * T + t];
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
            double h = 0.0;
#pragma unroll
            for (int c = 0; c < NJ; ++c) h += d_elem(P, T, t, r, c, lam) * d[c];
            if (t > 0) h -= w * P.dx[(size_t)r * T + t - 1];
            if (t + 1 < T) h -= w * P.dx[(size_t)r * T + t + 1];
            P.rb[(size_t)r * T + t] = -P.g[(size_t)r * T + t] - h;
        }
    }
}

template <typename S>
__global__ __launch_bounds__(LM_BS) void lm_kernel(const DevPlan *__restrict__ plans, int iters) {
    constexpr int PREC = sizeof(S) == sizeof(double) ? 1 : 0;
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T;
    if (T <= 0 || P.prec != PREC) return;   // empty slot or the other precision's plan
    {
        const LMState *s0 = P.st;
        if (s0->seeded && s0->iters_target > 0 && s0->iters_done >= s0->iters_target) return;
    }
    __shared__ double red[LM_BS];
    __shared__ double sh_lam, sh_nu, sh_cost;
    __shared__ int sh_flags[4];   // 0 need_lin, 1 status, 2 accept, 3 pivot failure
    const int tid = threadIdx.x;
    const RobotT<S> rb = load_robot<S>(P);
    LMState *st = P.st;

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
        const double c0 = plan_cost<S>(P, rb, P.xi, T, red);
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
        }
        __syncthreads();
    }
    if (tid == 0) {
        sh_lam = st->lambda;
        sh_nu = st->nu;
        sh_cost = st->cost;
        sh_flags[0] = st->need_lin;
        sh_flags[1] = st->status;
        // iterations this launch: at most what the plan still has to do
        const int left = st->iters_target > 0 ? st->iters_target - st->iters_done : iters;
        sh_flags[2] = left < iters ? (left > 0 ? left : 0) : iters;
    }
    __syncthreads();
    const int n_it = sh_flags[2];

    const int lane = tid & 63;
    const bool wave0 = tid < 64;
    __shared__ ChunkShared chs;
    // Chunks of at least 8 waypoints, one per wavefront; short paths use the
    // single-wavefront sweep.
    const int C = min(MAX_CHUNKS, T / 8) >= 2 ? min(MAX_CHUNKS, T / 8) : 1;
    for (int it = 0; it < n_it; ++it) {
        if (sh_flags[1] != 0) break;
        const double lam = sh_lam;
        if (sh_flags[0]) {
            const double gm = linearise<S>(P, rb, T);
            const double gmax = block_max(gm, red);
            if (tid == 0) st->grad_inf = gmax;
        }
        __syncthreads();
        if (C > 1) {
            const bool ok = chunk_factor(P, T, C, lam, chs);
            if (tid == 0) sh_flags[3] = ok ? 0 : 1;
            if (ok) chunk_substitute(P, T, C, P.g, -1.0, P.dx, chs);   // right-hand side -g
        } else if (wave0) {
            const bool ok = factor_and_solve(P, T, lam, lane);
            if (lane == 0) sh_flags[3] = ok ? 0 : 1;
        }
        __syncthreads();
        if (sh_flags[3]) {
            if (tid == 0) sh_flags[1] = CPF_STATUS_NUMERIC;
            __syncthreads();
            break;
        }
        for (int rs = 0; rs < P.refine_steps; ++rs) {
            refine_residual(P, T, lam);
            __syncthreads();
            if (C > 1) {
                chunk_substitute(P, T, C, P.rb, 1.0, P.rb, chs);   // correction in place
            } else if (wave0) {
                substitute(P, T, P.rb, 1.0, P.rb, lane);
            }
            __syncthreads();
            for (int t = tid; t < T; t += LM_BS)
#pragma unroll
                for (int j = 0; j < NJ; ++j) P.dx[(size_t)j * T + t] += P.rb[(size_t)j * T + t];
            __syncthreads();
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
        const double cn = plan_cost<S>(P, rb, P.xt, T, red);
        const double pred = 0.5 * block_sum(pr, red);
        if (tid == 0) {
            const double c = sh_cost;
            double l = sh_lam, nu = sh_nu;
            const int acc = cn < c;
            if (acc) {
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
            sh_lam = l;
            sh_nu = nu;
            sh_flags[0] = acc;
            sh_flags[2] = acc;
            st->iters_done += 1;
        }
        __syncthreads();
        if (sh_flags[2]) {
            for (int t = tid; t < T; t += LM_BS)
#pragma unroll
                for (int j = 0; j < NJ; ++j) P.xi[(size_t)j * T + t] = P.xt[(size_t)j * T + t];
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->lambda = sh_lam;
        st->nu = sh_nu;
        st->cost = sh_cost;
        st->need_lin = sh_flags[0];
        st->status = sh_flags[1];
    }
}

// Report: FP64 pose error of xi vs the targets and mjac (Sec. II metrics).
__global__ __launch_bounds__(LM_BS) void eval_kernel(const DevPlan *__restrict__ plans,
                                                     int only_finished) {
    const DevPlan &P = plans[blockIdx.x];
    const int T = P.T;
    if (T <= 0) return;
    if (only_finished) {
        const LMState *s0 = P.st;
        const bool finished = s0->status != 0 ||
                              (s0->iters_target > 0 && s0->iters_done >= s0->iters_target);
        if (!finished || s0->reported) return;
    }
    __shared__ double red[LM_BS];
    const RobotT<double> rb = load_robot<double>(P);
    double ep = 0.0, er = 0.0, mj = 0.0;
    for (int t = threadIdx.x; t < T; t += LM_BS) {
        double q[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) q[j] = P.xi[(size_t)j * T + t];
        double X[3], Y[3], Z[3], p[3], Zs[NJ][3], Os[NJ][3];
        chain<double, false>(rb, q, X, Y, Z, p, Zs, Os);
        double tg[12];
        load_target<double>(P, T, t, tg);
        const double dx = p[0] - tg[0], dy = p[1] - tg[1], dz = p[2] - tg[2];
        ep = fmax(ep, sqrt(dx * dx + dy * dy + dz * dz));
        double E[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                E[a * 3 + b] = X[a] * tg[3 + b * 3 + 0] + Y[a] * tg[3 + b * 3 + 1] + Z[a] * tg[3 + b * 3 + 2];
        const double v0 = 0.5 * (E[7] - E[5]), v1 = 0.5 * (E[2] - E[6]), v2 = 0.5 * (E[3] - E[1]);
        er = fmax(er, atan2(sqrt(v0 * v0 + v1 * v1 + v2 * v2), 0.5 * (E[0] + E[4] + E[8] - 1.0)));
        if (t + 1 < T)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                mj = fmax(mj, fabs(P.xi[(size_t)j * T + t + 1] - q[j]));
    }
    ep = block_max(ep, red);
    er = block_max(er, red);
    mj = block_max(mj, red);
    if (threadIdx.x == 0) {
        P.report[0] = ep;
        P.report[1] = er;
        P.report[2] = mj;
        if (only_finished) P.st->reported = 1;
    }
}

hipError_t lm_launch(const DevPlan *d_plans, int nplans, int prec, int iters, hipStream_t s) {
    if (nplans <= 0) return hipSuccess;
    if (prec == 1)
        hipLaunchKernelGGL((lm_kernel<double>), dim3(nplans), dim3(LM_BS), 0, s, d_plans, iters);
    else
        hipLaunchKernelGGL((lm_kernel<float>), dim3(nplans), dim3(LM_BS), 0, s, d_plans, iters);
    return hipGetLastError();
}

hipError_t eval_launch(const DevPlan *d_plans, int nplans, int only_finished, hipStream_t s) {
    if (nplans <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_kernel, dim3(nplans), dim3(LM_BS), 0, s, d_plans, only_finished);
    return hipGetLastError();
}

}  // namespace cpf
