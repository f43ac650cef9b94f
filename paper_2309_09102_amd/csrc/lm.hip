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
// block LDL^T sweep  S_t = D_t - w^2 S_{t-1}^{-1}, partitioned over the
// wavefronts of the workgroup (7x7 blocks one element per lane, inverses by
// Gauss-Jordan), then FP64 iterative refinement against the same H.
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
__device__ __forceinline__ double pose_sq(const DevPlan &P, const RobotT<S> &rb, const CPF_GLOBAL double *X,
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
__device__ __forceinline__ double plan_cost(const DevPlan &P, const RobotT<S> &rb, const CPF_GLOBAL double *X,
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

// ---------------------------------------------------------------------------
// 7x7 blocks on a wavefront: lane l < 49 holds element (l / 7, l % 7); lanes
// 49..63 hold nothing and never write.  A vector is held in lanes 0..6.
// Block products exchange operands through a per-wavefront LDS scratch (one
// write of the block, then each lane reads its row and column); LDS
// instructions of one wavefront execute in program order, so no barrier is
// needed.  Blocks live in HBM as [T][7][8] doubles.
// ---------------------------------------------------------------------------

struct Lane {
    int l, i, j, r;   // lane, element row / column, vector index
    bool el;          // lane holds an element
};

__device__ __forceinline__ Lane lane_info() {
    Lane L;
    L.l = threadIdx.x & 63;
    L.el = L.l < NBLK;
    L.i = L.el ? L.l / NJ : NJ - 1;
    L.j = L.el ? L.l % NJ : NJ - 1;
    L.r = L.l < NJ ? L.l : NJ - 1;
    return L;
}

struct WaveScratch {
    double m0[64], m1[64], v[8];
};

// The wave barriers keep the compiler from moving scratch reads of the
// previous product past this write, or this product's reads before it.
__device__ __forceinline__ void put(double *buf, const Lane &L, double x) {
    __builtin_amdgcn_wave_barrier();
    if (L.el) buf[L.i * 8 + L.j] = x;
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void put_vec(double *buf, const Lane &L, double x) {
    __builtin_amdgcn_wave_barrier();
    if (L.l < NJ) buf[L.l] = x;
    __builtin_amdgcn_wave_barrier();
}

// element (i, j) of A B
__device__ __forceinline__ double mm(double A, double B, const Lane &L, WaveScratch &ws) {
    put(ws.m0, L, A);
    put(ws.m1, L, B);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) s += ws.m0[L.i * 8 + k] * ws.m1[k * 8 + L.j];
    return s;
}

// element (i, j) of A B^T
__device__ __forceinline__ double mm_bt(double A, double B, const Lane &L, WaveScratch &ws) {
    put(ws.m0, L, A);
    put(ws.m1, L, B);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) s += ws.m0[L.i * 8 + k] * ws.m1[L.j * 8 + k];
    return s;
}

// (M v)_r in lane r < 7
__device__ __forceinline__ double mv(double M, double v, const Lane &L, WaveScratch &ws) {
    put(ws.m0, L, M);
    put_vec(ws.v, L, v);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) s += ws.m0[L.r * 8 + k] * ws.v[k];
    return s;
}

// (M^T v)_r in lane r < 7
__device__ __forceinline__ double mtv(double M, double v, const Lane &L, WaveScratch &ws) {
    put(ws.m0, L, M);
    put_vec(ws.v, L, v);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NJ; ++k) s += ws.m0[k * 8 + L.r] * ws.v[k];
    return s;
}

// In-place Gauss-Jordan inverse of a symmetric positive definite block.
// Pivot k: a_kk, the lane's a_ik and a_kj are read back from the scratch.
// ok becomes false on a non-positive pivot.
__device__ __forceinline__ double gj_inverse(double a, const Lane &L, WaveScratch &ws, bool &ok) {
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        put(ws.m0, L, a);
        const double akk = ws.m0[k * 9];
        const double aik = ws.m0[L.i * 8 + k];
        const double akj = ws.m0[k * 8 + L.j];
        ok = ok && (akk > 0.0);
        // reciprocal: hardware estimate refined by one Newton step
        double rc = __builtin_amdgcn_rcp(akk);
        rc = fma(rc, fma(-akk, rc, 1.0), rc);
        double na;
        if (L.i == k) na = (L.j == k) ? rc : akj * rc;
        else if (L.j == k) na = -aik * rc;
        else na = a - aik * (akj * rc);
        a = na;
    }
    return a;
}

__device__ __forceinline__ double blk_ld(const CPF_GLOBAL double *base, int t, const Lane &L, int lo, int hi) {
    return (t >= lo && t <= hi && L.el) ? base[(size_t)t * 56 + L.i * 8 + L.j] : 0.0;
}

__device__ __forceinline__ void blk_st(CPF_GLOBAL double *base, int t, const Lane &L, double x) {
    if (L.el) base[(size_t)t * 56 + L.i * 8 + L.j] = x;
}

__device__ __forceinline__ double vec_ld(const CPF_GLOBAL double *base, int T, const Lane &L, int t, int lo,
                                         int hi) {
    return (t >= lo && t <= hi) ? base[(size_t)L.r * T + t] : 0.0;
}

__device__ __forceinline__ double d_ld(const DevPlan &P, int T, int t, const Lane &L, int lo, int hi,
                                       double lam) {
    return (t >= lo && t <= hi) ? d_elem(P, T, t, L.i, L.j, lam) : 0.0;
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
//   a_t = P_t (y_t + w a_{t+1}),  G_t = P_t (F_t + w G_{t+1}),  a_e = G_e = 0.
// The last rows of the chunks then form a symmetric block-tridiagonal system
// in z_0 .. z_{C-1} (the Schur complement on the chunk ends):
//   M_c = S_{e_c} - w G_{c+1},  sub-diagonal -F_{e_c},  r_c = y_{e_c} + w a_{c+1},
// solved by one wavefront with the same LDL^T sweep, after which every chunk
// recovers its interior: x_t = P_t (y_t + F_t z_{c-1} + w x_{t+1}).
// With C = 1 this is the plain block LDL^T sweep over the whole path.
// ---------------------------------------------------------------------------

constexpr int MAX_CHUNKS = LM_BS / 64;

struct ChunkShared {
    double Pi[MAX_CHUNKS][64];   // S_{e_c}, then Pi_c = Sigma_c^{-1}
    double G[MAX_CHUNKS][64];    // G_c at the chunk's first block
    double y[MAX_CHUNKS][8];     // y_{e_c}, then rho_c
    double a[MAX_CHUNKS][8];     // a_c at the chunk's first block
    double z[MAX_CHUNKS][8];     // chunk-end solution z_c
    WaveScratch ws[MAX_CHUNKS];
    int bad;
};

__device__ __forceinline__ void chunk_bounds(int T, int C, int c, int &s, int &e) {
    s = (int)(((long long)c * T) / C);
    e = (int)(((long long)(c + 1) * T) / C) - 1;
}

// Reduced system on the chunk ends (wave 0).  With `factor`, Sigma_c =
// M_c - F_{e_c} Pi_{c-1} F_{e_c}^T is factored (Pi_c kept in sh.Pi); then
// rho / z are solved from sh.y (y_{e_c}) and sh.a (a_c).
__device__ __forceinline__ void reduced_solve(const DevPlan &P, int T, int C, bool factor, ChunkShared &sh,
                              bool &ok) {
    const Lane L = lane_info();
    WaveScratch &ws = sh.ws[0];
    const double w = P.w_s;
    const int ij = L.i * 8 + L.j;
    double pi_prev = 0.0, rho_prev = 0.0;
    for (int cc = 0; cc < C; ++cc) {
        int s, e;
        chunk_bounds(T, C, cc, s, e);
        const double Fe = cc > 0 ? blk_ld(P.F, e, L, 0, T - 1) : 0.0;   // F_{e_c}
        double pi;
        if (factor) {
            double M = sh.Pi[cc][ij];
            if (cc + 1 < C) M -= w * sh.G[cc + 1][ij];
            if (cc > 0) M -= mm_bt(mm(Fe, pi_prev, L, ws), Fe, L, ws);   // F Pi F^T
            pi = gj_inverse(M, L, ws, ok);
            if (L.el) sh.Pi[cc][ij] = pi;
        } else {
            pi = sh.Pi[cc][ij];
        }
        double r = sh.y[cc][L.r];
        if (cc + 1 < C) r += w * sh.a[cc + 1][L.r];
        if (cc > 0) r += mv(Fe, mv(pi_prev, rho_prev, L, ws), L, ws);
        if (L.l < NJ) sh.y[cc][L.r] = r;
        rho_prev = r;
        pi_prev = pi;
    }
    double znext = 0.0;
    for (int cc = C - 1; cc >= 0; --cc) {
        double v = sh.y[cc][L.r];
        if (cc + 1 < C) {
            int s1, e1;
            chunk_bounds(T, C, cc + 1, s1, e1);
            v += mtv(blk_ld(P.F, e1, L, 0, T - 1), znext, L, ws);   // F_{e_{c+1}}^T z_{c+1}
        }
        const double z = mv(sh.Pi[cc][ij], v, L, ws);
        if (L.l < NJ) sh.z[cc][L.r] = z;
        znext = z;
    }
}

// Interior of chunk c: x_t = P_t (y_t + F_t z_{c-1} + w x_{t+1}), x_e = z_c.
__device__ __forceinline__ void chunk_interior(const DevPlan &P, int T, int c, int s, int e,
                                               CPF_GLOBAL double *out, ChunkShared &sh) {
    const Lane L = lane_info();
    WaveScratch &ws = sh.ws[c];
    const double w = P.w_s;
    const double zl = c > 0 ? sh.z[c - 1][L.r] : 0.0;
    double x = sh.z[c][L.r];
    if (L.l < NJ) out[(size_t)L.r * T + e] = x;
    double p0 = blk_ld(P.P, e - 1, L, s, e - 1), p1 = blk_ld(P.P, e - 2, L, s, e - 1);
    double f0 = blk_ld(P.F, e - 1, L, s, e - 1), f1 = blk_ld(P.F, e - 2, L, s, e - 1);
    double y0 = vec_ld(P.y, T, L, e - 1, s, e - 1), y1 = vec_ld(P.y, T, L, e - 2, s, e - 1);
    for (int t = e - 1; t >= s; --t) {
        const double pm = p0, fm = f0, ym = y0;
        p0 = p1; f0 = f1; y0 = y1;
        p1 = blk_ld(P.P, t - 2, L, s, e - 1);
        f1 = blk_ld(P.F, t - 2, L, s, e - 1);
        y1 = vec_ld(P.y, T, L, t - 2, s, e - 1);
        double v = ym + w * x;
        if (c > 0) v += mv(fm, zl, L, ws);
        x = mv(pm, v, L, ws);
        if (L.l < NJ) out[(size_t)L.r * T + t] = x;
    }
}

// Factorisation of the partitioned system fused with the solve for the
// right-hand side -g (all waves; wave c owns chunk c).  Stores P_t (t < e_c),
// F_t and y_t, Pi_c for the chunk ends, and the step in P.dx.  Returns false
// on a non-positive pivot.
__device__ __forceinline__ bool chunk_factor_solve(const DevPlan &P, int T, int C, double lam,
                                                   ChunkShared &sh) {
    const int c = threadIdx.x >> 6;
    const Lane L = lane_info();
    const double w = P.w_s, w2 = w * w;
    if (threadIdx.x == 0) sh.bad = 0;
    __syncthreads();
    bool ok = true;
    int s = 0, e = -1;
    if (c < C) {
        WaveScratch &ws = sh.ws[c];
        chunk_bounds(T, C, c, s, e);
        double d0 = d_ld(P, T, s, L, s, e, lam), d1 = d_ld(P, T, s + 1, L, s, e, lam);
        double b0 = -vec_ld(P.g, T, L, s, s, e), b1 = -vec_ld(P.g, T, L, s + 1, s, e);
        double pprev = 0.0, fprev = 0.0, yprev = 0.0;
        for (int t = s; t <= e; ++t) {
            const double d = d0, b = b0;
            d0 = d1;
            b0 = b1;
            d1 = d_ld(P, T, t + 2, L, s, e, lam);
            b1 = -vec_ld(P.g, T, L, t + 2, s, e);
            double S = d, F, y = b;
            if (t == s) {
                F = (c > 0 && L.el && L.i == L.j) ? w : 0.0;
            } else {
                S -= w2 * pprev;
                F = w * mm(pprev, fprev, L, ws);
                y += w * mv(pprev, yprev, L, ws);
            }
            if (C > 1) blk_st(P.F, t, L, F);
            if (L.l < NJ) P.y[(size_t)L.r * T + t] = y;
            if (t == e) {
                if (L.el) sh.Pi[c][L.i * 8 + L.j] = S;
                if (L.l < NJ) sh.y[c][L.r] = y;
            } else {
                pprev = gj_inverse(S, L, ws, ok);
                blk_st(P.P, t, L, pprev);
            }
            fprev = F;
            yprev = y;
        }
        // backward (chunks that have a predecessor): G and a at the first block
        double G = 0.0, a = 0.0;
        if (c > 0) {
            double p0 = blk_ld(P.P, e - 1, L, s, e - 1), p1 = blk_ld(P.P, e - 2, L, s, e - 1);
            double f0 = blk_ld(P.F, e - 1, L, s, e - 1), f1 = blk_ld(P.F, e - 2, L, s, e - 1);
            double y0 = vec_ld(P.y, T, L, e - 1, s, e - 1), y1 = vec_ld(P.y, T, L, e - 2, s, e - 1);
            for (int t = e - 1; t >= s; --t) {
                const double pm = p0, fm = f0, ym = y0;
                p0 = p1; f0 = f1; y0 = y1;
                p1 = blk_ld(P.P, t - 2, L, s, e - 1);
                f1 = blk_ld(P.F, t - 2, L, s, e - 1);
                y1 = vec_ld(P.y, T, L, t - 2, s, e - 1);
                G = mm(pm, fm + w * G, L, ws);
                a = mv(pm, ym + w * a, L, ws);
            }
        }
        if (L.el) sh.G[c][L.i * 8 + L.j] = G;
        if (L.l < NJ) sh.a[c][L.r] = a;
        if (!ok) sh.bad = 1;
    }
    __syncthreads();
    if (c == 0) {
        reduced_solve(P, T, C, true, sh, ok);
        if (!ok) sh.bad = 1;
    }
    __syncthreads();
    if (sh.bad) return false;
    if (c < C) chunk_interior(P, T, c, s, e, P.dx, sh);
    __syncthreads();
    return true;
}

// Solve with the partitioned factors for right-hand side sign*rhs ([7][T]);
// writes out ([7][T], may alias rhs).  All waves.
__device__ __forceinline__ void chunk_substitute(const DevPlan &P, int T, int C,
                                                 const CPF_GLOBAL double *rhs,
                                 double sign, CPF_GLOBAL double *out, ChunkShared &sh) {
    const int c = threadIdx.x >> 6;
    const Lane L = lane_info();
    const double w = P.w_s;
    int s = 0, e = -1;
    if (c < C) {
        WaveScratch &ws = sh.ws[c];
        chunk_bounds(T, C, c, s, e);
        // forward: y_t = b_t + w P_{t-1} y_{t-1} within the chunk
        double yprev = 0.0, pprev = 0.0;
        double p0 = blk_ld(P.P, s, L, s, e - 1), p1 = blk_ld(P.P, s + 1, L, s, e - 1);
        double r0 = vec_ld(rhs, T, L, s, s, e), r1 = vec_ld(rhs, T, L, s + 1, s, e);
        for (int t = s; t <= e; ++t) {
            const double pm = p0, rm = r0;
            p0 = p1; r0 = r1;
            p1 = blk_ld(P.P, t + 2, L, s, e - 1);
            r1 = vec_ld(rhs, T, L, t + 2, s, e);
            double y = sign * rm;
            if (t > s) y += w * mv(pprev, yprev, L, ws);
            if (L.l < NJ) P.y[(size_t)L.r * T + t] = y;
            yprev = y;
            pprev = pm;
        }
        if (L.l < NJ) sh.y[c][L.r] = yprev;
        // backward: a_t = P_t (y_t + w a_{t+1}), a_e = 0
        double a = 0.0;
        if (c > 0) {
            double q0 = blk_ld(P.P, e - 1, L, s, e - 1), q1 = blk_ld(P.P, e - 2, L, s, e - 1);
            double y0 = vec_ld(P.y, T, L, e - 1, s, e - 1), y1 = vec_ld(P.y, T, L, e - 2, s, e - 1);
            for (int t = e - 1; t >= s; --t) {
                const double pm = q0, ym = y0;
                q0 = q1; y0 = y1;
                q1 = blk_ld(P.P, t - 2, L, s, e - 1);
                y1 = vec_ld(P.y, T, L, t - 2, s, e - 1);
                a = mv(pm, ym + w * a, L, ws);
            }
        }
        if (L.l < NJ) sh.a[c][L.r] = a;
    }
    __syncthreads();
    if (c == 0) {
        bool ok = true;
        reduced_solve(P, T, C, false, sh, ok);
    }
    __syncthreads();
    if (c < C) chunk_interior(P, T, c, s, e, out, sh);
    __syncthreads();
}

// rb_t = -g_t - (H dx)_t  for every waypoint (all lanes).
__device__ __forceinline__ void refine_residual(const DevPlan &P, int T, double lam) {
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

    __shared__ ChunkShared chs;
    // Chunks of at least 8 waypoints, one per wavefront (C = 1: plain sweep).
    const int C = max(1, min(MAX_CHUNKS, T / 8));
#ifdef CPF_PHASE_CYCLES
    // Diagnostic build only: per-phase shader-clock totals printed by thread 0.
    uint64_t ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t ph_last = clock64();
#define PHASE_MARK(k)                                  \
    do {                                               \
        if (tid == 0) {                                \
            const uint64_t now_ = clock64();           \
            ph[k] += now_ - ph_last;                   \
            ph_last = now_;                            \
        }                                              \
    } while (0)
#else
#define PHASE_MARK(k) \
    do {              \
    } while (0)
#endif
    for (int it = 0; it < n_it; ++it) {
        if (sh_flags[1] != 0) break;
        const double lam = sh_lam;
        if (sh_flags[0]) {
            const double gm = linearise<S>(P, rb, T);
            const double gmax = block_max(gm, red);
            if (tid == 0) st->grad_inf = gmax;
        }
        __syncthreads();
        PHASE_MARK(0);
        {
            const bool ok = chunk_factor_solve(P, T, C, lam, chs);   // right-hand side -g
            if (tid == 0) sh_flags[3] = ok ? 0 : 1;
            PHASE_MARK(1);
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
            PHASE_MARK(3);
            chunk_substitute(P, T, C, P.rb, 1.0, P.rb, chs);   // correction in place
            __syncthreads();
            for (int t = tid; t < T; t += LM_BS)
#pragma unroll
                for (int j = 0; j < NJ; ++j) P.dx[(size_t)j * T + t] += P.rb[(size_t)j * T + t];
            __syncthreads();
            PHASE_MARK(4);
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
        PHASE_MARK(5);
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
        PHASE_MARK(6);
    }
#ifdef CPF_PHASE_CYCLES
    if (tid == 0 && blockIdx.x == 0)
        printf("lm phase cycles T=%d C=%d iters=%d: lin %llu factor %llu solve %llu refres %llu "
               "refsub %llu trial %llu accept %llu\n",
               T, C, n_it, (unsigned long long)ph[0], (unsigned long long)ph[1],
               (unsigned long long)ph[2], (unsigned long long)ph[3], (unsigned long long)ph[4],
               (unsigned long long)ph[5], (unsigned long long)ph[6]);
#endif
#undef PHASE_MARK
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
