// fk.hip -- batched forward kinematics and geometric Jacobian (Sec. II; the
// kinematic Jacobian of Sec. III-C).  One lane per configuration; the chain
// lives in registers; q, pose and J are SoA so every load and store of a
// wavefront is one contiguous 256-byte (float) or 512-byte (double) run.
#include "coll_device.h"
#include "cpf_device.h"
#include "cpf_internal.h"

namespace cpf {
namespace CPF_JNS {

template <typename S, bool WANT_J>
__global__ __launch_bounds__(256) void fk_batch_kernel(RobotT<S> rb, int64_t M,
                                                       const S *__restrict__ q,
                                                       S *__restrict__ pose,
                                                       S *__restrict__ J) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    S qq[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qq[j] = q[(int64_t)j * M + m];
    S X[3], Y[3], Z[3], p[3], Zs[NJ][3], Os[NJ][3];
    chain<S, WANT_J>(rb, qq, X, Y, Z, p, Zs, Os);
    const S out[12] = {p[0], p[1], p[2], X[0], Y[0], Z[0], X[1], Y[1], Z[1], X[2], Y[2], Z[2]};
#pragma unroll
    for (int e = 0; e < 12; ++e) pose[(int64_t)e * M + m] = out[e];
    if (WANT_J) {
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            S col[6];
            jac_column<S>(rb.prism, i, Zs[i], Os[i], p, col);
#pragma unroll
            for (int r = 0; r < 6; ++r) J[((int64_t)r * NJ + i) * M + m] = col[r];
        }
    }
}

template <typename S>
static hipError_t launch_fk(const RobotT<S> &rb, int64_t M, const void *q, void *pose, void *J,
                            hipStream_t s) {
    if (M == 0) return hipSuccess;
    const dim3 grid((unsigned)((M + 255) / 256));
    if (J)
        hipLaunchKernelGGL((fk_batch_kernel<S, true>), grid, dim3(256), 0, s, rb, M,
                           (const S *)q, (S *)pose, (S *)J);
    else
        hipLaunchKernelGGL((fk_batch_kernel<S, false>), grid, dim3(256), 0, s, rb, M,
                           (const S *)q, (S *)pose, (S *)nullptr);
    return hipGetLastError();
}

hipError_t fk_batch_launch(const HostRobot &hr, int64_t M, int prec, const void *q, void *pose,
                           void *J, hipStream_t s) {
    if (prec == 1) {
        RobotT<double> rb;
        for (int i = 0; i < NJ; ++i) {
            rb.a[i] = hr.a[i]; rb.d[i] = hr.d[i]; rb.ca[i] = hr.ca[i]; rb.sa[i] = hr.sa[i];
            rb.off[i] = hr.off[i];
        }
        rb.prism = hr.prism;
        return launch_fk<double>(rb, M, q, pose, J, s);
    }
    RobotT<float> rb;
    for (int i = 0; i < NJ; ++i) {
        rb.a[i] = (float)hr.a[i]; rb.d[i] = (float)hr.d[i]; rb.ca[i] = (float)hr.ca[i];
        rb.sa[i] = (float)hr.sa[i]; rb.off[i] = (float)hr.off[i];
    }
    rb.prism = hr.prism;
    return launch_fk<float>(rb, M, q, pose, J, s);
}

// Collision distances of M configurations (the checker of Sec. III-B and the
// distances of Sec. III-C): dist [2][M] (self, environment), optionally the
// gradients grad [2 * NJ][M] (row h * NJ + k).  One lane per configuration.
template <typename S, bool GRAD>
__global__ __launch_bounds__(256) void coll_batch_kernel(RobotT<S> rb, HostCaps caps, int n_obs,
                                                         const double *__restrict__ obs, int64_t M,
                                                         const S *__restrict__ q, S *__restrict__ dist,
                                                         S *__restrict__ grad) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    S qq[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qq[j] = q[(int64_t)j * M + m];
    S dm[2], g[2][NJ];
    coll_distances<S, GRAD>(rb, caps.v, n_obs, (const CPF_GLOBAL double *)obs, qq, dm, g);
    dist[m] = dm[0];
    dist[M + m] = dm[1];
    if (GRAD) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < NJ; ++k) grad[((int64_t)h * NJ + k) * M + m] = g[h][k];
    }
}

template <typename S>
static hipError_t launch_coll(const RobotT<S> &rb, const HostCaps &caps, int n_obs, const double *obs, int64_t M,
                              const void *q, void *dist, void *grad, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const dim3 grid((unsigned)((M + 255) / 256));
    if (grad)
        hipLaunchKernelGGL((coll_batch_kernel<S, true>), grid, dim3(256), 0, s, rb, caps, n_obs, obs, M,
                           (const S *)q, (S *)dist, (S *)grad);
    else
        hipLaunchKernelGGL((coll_batch_kernel<S, false>), grid, dim3(256), 0, s, rb, caps, n_obs, obs, M,
                           (const S *)q, (S *)dist, (S *)nullptr);
    return hipGetLastError();
}

hipError_t coll_batch_launch(const HostRobot &hr, const HostCaps &caps, int n_obs, const double *obs, int64_t M,
                             int prec, const void *q, void *dist, void *grad, hipStream_t s) {
    if (prec == 1) {
        RobotT<double> rb;
        for (int i = 0; i < NJ; ++i) {
            rb.a[i] = hr.a[i]; rb.d[i] = hr.d[i]; rb.ca[i] = hr.ca[i]; rb.sa[i] = hr.sa[i];
            rb.off[i] = hr.off[i];
        }
        rb.prism = hr.prism;
        return launch_coll<double>(rb, caps, n_obs, obs, M, q, dist, grad, s);
    }
    RobotT<float> rb;
    for (int i = 0; i < NJ; ++i) {
        rb.a[i] = (float)hr.a[i]; rb.d[i] = (float)hr.d[i]; rb.ca[i] = (float)hr.ca[i];
        rb.sa[i] = (float)hr.sa[i]; rb.off[i] = (float)hr.off[i];
    }
    rb.prism = hr.prism;
    return launch_coll<float>(rb, caps, n_obs, obs, M, q, dist, grad, s);
}

// One thread per (waypoint, candidate) pair, candidates fastest, so the
// float stores of a joint row are contiguous; the last T threads transpose
// the targets.  Candidates arrive as [K][T][NJ] doubles or floats.  With bad
// non-null (inputs the host could not check), a value that is not finite
// (also a double beyond the float range) is stored as 0 and sets *bad.
template <typename C>
__global__ __launch_bounds__(256) void stage_kernel(const C *__restrict__ cand_in, const double *__restrict__ tg_in,
                                                    int T, int K, float *__restrict__ cand,
                                                    double *__restrict__ targets, int *__restrict__ bad) {
    const long long n = (long long)T * K;
    const long long x = (long long)blockIdx.x * 256 + threadIdx.x;
    bool ok = true;
    if (x < n) {
        const int t = (int)(x / K), k = (int)(x % K);
        const C *q = cand_in + ((size_t)k * T + t) * NJ;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            float v = (float)q[j];
            if (bad && !isfinite(v)) {
                v = 0.0f;
                ok = false;
            }
            cand[((size_t)t * NJ + j) * K + k] = v;
        }
    } else if (x < n + T) {
        const int t = (int)(x - n);
        const double *tg = tg_in + (size_t)t * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double v = tg[c];
            if (bad && !isfinite(v)) {
                v = 0.0;
                ok = false;
            }
            targets[(size_t)c * T + t] = v;
        }
    }
    if (!ok) atomicOr(bad, 1);
}

// Appended candidates: raw [K_add][T][NJ] doubles into columns
// k_off .. k_off + K_add - 1 of the float [T][NJ][K] candidate array.
__global__ __launch_bounds__(256) void stage_append_kernel(const double *__restrict__ raw, int T, int K_add,
                                                           int K, int k_off, float *__restrict__ cand) {
    const long long x = (long long)blockIdx.x * 256 + threadIdx.x;
    if (x >= (long long)T * K_add) return;
    const int t = (int)(x / K_add), k = (int)(x % K_add);
    const double *q = raw + ((size_t)k * T + t) * NJ;
#pragma unroll
    for (int j = 0; j < NJ; ++j) cand[((size_t)t * NJ + j) * K + k_off + k] = (float)q[j];
}

hipError_t stage_append_launch(const double *raw, int T, int K_add, int K, int k_off, float *cand,
                               hipStream_t s) {
    const long long n = (long long)T * K_add;
    if (n <= 0) return hipSuccess;
    if (k_off < 0 || k_off + K_add > K) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stage_append_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, raw, T, K_add,
                       K, k_off, cand);
    return hipGetLastError();
}

hipError_t stage_launch(const void *cand_in, bool cand_f32, const double *tg_in, int T, int K, float *cand,
                        double *targets, int *bad, hipStream_t s) {
    const long long n = (long long)T * K + T;
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (cand_f32)
        hipLaunchKernelGGL(stage_kernel<float>, g, b, 0, s, (const float *)cand_in, tg_in, T, K, cand, targets, bad);
    else
        hipLaunchKernelGGL(stage_kernel<double>, g, b, 0, s, (const double *)cand_in, tg_in, T, K, cand, targets,
                           bad);
    return hipGetLastError();
}

// A [NJ][T] trajectory (one row per joint) into [T][NJ] rows, one thread per
// element of the output.
__global__ __launch_bounds__(256) void soa_rows_kernel(const double *__restrict__ soa, int T,
                                                       double *__restrict__ rows) {
    const long long x = (long long)blockIdx.x * 256 + threadIdx.x;
    if (x >= (long long)T * NJ) return;
    const int t = (int)(x / NJ), j = (int)(x % NJ);
    rows[x] = soa[(size_t)j * T + t];
}

hipError_t soa_rows_launch(const double *soa, int T, double *rows, hipStream_t s) {
    const long long n = (long long)T * NJ;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(soa_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, soa, T, rows);
    return hipGetLastError();
}

}  // namespace CPF_JNS
}  // namespace cpf
