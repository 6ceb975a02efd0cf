// N-link planar robot (gfx950): the robot of the paper's convex-solver and
// EMPC experiments (Sec. IV-F setup, Sec. VI-A), M(q) qdd + C(q, qd) + b qd
// = tau, in a plane perpendicular to gravity, point masses at the link ends.
// EMPC runs on a linear model (eq. 2) relinearized at the current state
// every control tick; these kernels produce that model on the device and
// simulate the robot itself:
//  - nlink_linearize_kernel: the exact Jacobians of f(x, tau) = [qd; qdd] at
//    (x, u), the affine offset, and the zero-order hold over dt
//    (A_d, B_d, w_d from the exponential of [[A, B, w], [0, 0, 0]] dt);
//  - nlink_step_kernel: classical RK4 substeps of the nonlinear dynamics.
// Inverse dynamics come from a recursive Newton-Euler pass over the chain
// (O(N) per call): accelerations of the mass points outward, the force and
// moment carried by each joint inward.  M(q) is N such passes with qd = 0 and
// qdd = e_j, C(q, qd) one pass with qdd = 0, and the Jacobian of the forward
// dynamics follows from differentiating RNEA(q, qd, qdd(q, qd, tau)) =
// tau - b qd: dqdd/dx_s = M^-1 (d(tau - b qd)/dx_s - dRNEA/dx_s |qdd fixed),
// the last term a forward-mode dual-number pass per direction.  Everything
// runs in FP64 (the model is tiny); outputs are written in the problem dtype.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace empc {

namespace {

struct Dual {
    double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ inline Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ inline void sincos_d(Dual a, Dual *s, Dual *c) {
    double sv, cv;
    sincos(a.v, &sv, &cv);
    *s = {sv, cv * a.d};
    *c = {cv, -sv * a.d};
}
__device__ inline void sincos_d(double a, double *s, double *c) { sincos(a, s, c); }
template <typename S>
__device__ inline S make(double v, double d);
template <>
__device__ inline double make<double>(double v, double) { return v; }
template <>
__device__ inline Dual make<Dual>(double v, double d) { return {v, d}; }

// Inverse dynamics of the planar chain without gravity: joint torques that
// produce accelerations qdd at (q, qd), the viscous damping excluded.
// Mass point i moves with a_i = a_{i-1} + l_i (alpha_i u_i^perp - omega_i^2
// u_i), u_i = (cos phi_i, sin phi_i), phi/omega/alpha the absolute angle,
// rate and acceleration of link i; joint i carries the force f_i =
// sum_{j>=i} m_j a_j and the moment tau_i = tau_{i+1} + l_i u_i x f_i.
template <typename S>
__device__ void rnea(int N, const double *mass, const double *len, const S *q, const S *qd,
                     const S *qdd, S *tau) {
    S ux[NLINK_MAX], uy[NLINK_MAX], ax[NLINK_MAX], ay[NLINK_MAX];
    S phi = make<S>(0, 0), om = make<S>(0, 0), al = make<S>(0, 0);
    S px = make<S>(0, 0), py = make<S>(0, 0);
    for (int i = 0; i < N; ++i) {
        phi = phi + q[i];
        om = om + qd[i];
        al = al + qdd[i];
        S s, c;
        sincos_d(phi, &s, &c);
        const S w2 = om * om;
        px = px + len[i] * (make<S>(0, 0) - al * s - w2 * c);
        py = py + len[i] * (al * c - w2 * s);
        ux[i] = c;
        uy[i] = s;
        ax[i] = px;
        ay[i] = py;
    }
    S fx = make<S>(0, 0), fy = make<S>(0, 0), t = make<S>(0, 0);
    for (int i = N - 1; i >= 0; --i) {
        fx = fx + mass[i] * ax[i];
        fy = fy + mass[i] * ay[i];
        t = t + len[i] * (ux[i] * fy - uy[i] * fx);
        tau[i] = t;
    }
}

// In-place Cholesky factor (lower) of the N x N matrix A (row-major); one
// thread.
__device__ void cholesky(int N, double *A) {
    for (int j = 0; j < N; ++j) {
        double s = A[j * N + j];
        for (int k = 0; k < j; ++k) s -= A[j * N + k] * A[j * N + k];
        const double d = sqrt(s);
        A[j * N + j] = d;
        for (int i = j + 1; i < N; ++i) {
            double t = A[i * N + j];
            for (int k = 0; k < j; ++k) t -= A[i * N + k] * A[j * N + k];
            A[i * N + j] = t / d;
        }
    }
}
// y = (L L^T)^-1 r, in place on y (holding r on entry)
__device__ void chol_solve(int N, const double *L, double *y) {
    for (int i = 0; i < N; ++i) {
        double s = y[i];
        for (int k = 0; k < i; ++k) s -= L[i * N + k] * y[k];
        y[i] = s / L[i * N + i];
    }
    for (int i = N - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < N; ++k) s -= L[k * N + i] * y[k];
        y[i] = s / L[i * N + i];
    }
}

// Forward dynamics qdd = M^-1 (tau - C - b qd) at (q, qd) by threads
// 0..N of the workgroup (M's columns and C in parallel, the factorisation on
// thread 0).  Msh: N*N doubles of LDS, qdd: N doubles of LDS (the result).
// Must be reached by every thread of the workgroup.
__device__ void forward_dynamics(int N, const double *mass, const double *len, double b,
                                 const double *q, const double *qd, const double *tau,
                                 double *Msh, double *qdd) {
    const int tid = threadIdx.x;
    double zero[NLINK_MAX], col[NLINK_MAX];
    for (int i = 0; i < N; ++i) zero[i] = 0.0;
    if (tid < N) {
        double e[NLINK_MAX];
        for (int i = 0; i < N; ++i) e[i] = i == tid ? 1.0 : 0.0;
        rnea<double>(N, mass, len, q, zero, e, col);
        for (int i = 0; i < N; ++i) Msh[i * N + tid] = col[i];
    } else if (tid == N) {
        rnea<double>(N, mass, len, q, qd, zero, col);
        for (int i = 0; i < N; ++i) qdd[i] = tau[i] - col[i] - b * qd[i];
    }
    __syncthreads();
    if (tid == 0) {
        cholesky(N, Msh);
        chol_solve(N, Msh, qdd);
    }
    __syncthreads();
}

constexpr int LIN_THREADS = 256;
constexpr int ZMAX = 3 * NLINK_MAX + 1;  // n + m + 1 of the augmented hold matrix

// C = A B (D x D, row-major, LDS), all threads
__device__ void matmul_lds(int D, const double *A, const double *B, double *C) {
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
        const int i = e / D, j = e % D;
        double s = 0.0;
        for (int k = 0; k < D; ++k) s += A[i * D + k] * B[k * D + j];
        C[e] = s;
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(LIN_THREADS) void nlink_linearize_kernel(
    int N, const T *__restrict__ mass_in, const T *__restrict__ len_in, double b, double dt,
    const T *__restrict__ x_in, const T *__restrict__ u_in, T *__restrict__ Ad,
    T *__restrict__ Bd, T *__restrict__ wd) {
    __shared__ double mass[NLINK_MAX], len[NLINK_MAX], x[2 * NLINK_MAX], u[NLINK_MAX];
    __shared__ double Msh[NLINK_MAX * NLINK_MAX], qdd0[NLINK_MAX];
    __shared__ double J[3 * NLINK_MAX][NLINK_MAX];  // dqdd / d(q, qd, tau), column s
    __shared__ double Z[ZMAX * ZMAX], E[ZMAX * ZMAX], W[ZMAX * ZMAX];
    __shared__ int s_scale;
    const int tid = threadIdx.x, n = 2 * N, m = N, D = n + m + 1;
    if (tid < N) {
        mass[tid] = (double)mass_in[tid];
        len[tid] = (double)len_in[tid];
        u[tid] = (double)u_in[tid];
    }
    if (tid < n) x[tid] = (double)x_in[tid];
    __syncthreads();
    forward_dynamics(N, mass, len, b, x, x + N, u, Msh, qdd0);
    // direction s < 2N: state x_s; 2N <= s < 3N: torque s - 2N
    if (tid < 3 * N) {
        double y[NLINK_MAX];
        if (tid < n) {
            Dual q[NLINK_MAX], qd[NLINK_MAX], a[NLINK_MAX], t[NLINK_MAX];
            for (int i = 0; i < N; ++i) {
                q[i] = {x[i], i == tid ? 1.0 : 0.0};
                qd[i] = {x[N + i], N + i == tid ? 1.0 : 0.0};
                a[i] = {qdd0[i], 0.0};
            }
            rnea<Dual>(N, mass, len, q, qd, a, t);
            for (int i = 0; i < N; ++i) y[i] = -t[i].d - (N + i == tid ? b : 0.0);
        } else {
            for (int i = 0; i < N; ++i) y[i] = i == tid - n ? 1.0 : 0.0;
        }
        chol_solve(N, Msh, y);
        for (int i = 0; i < N; ++i) J[tid][i] = y[i];
    }
    __syncthreads();
    // Z = dt [[A, B, w], [0, 0, 0]]: position rows [0 I | 0 | 0] (their
    // offset qd - qd is 0), velocity rows from J and the offset
    // w = qdd0 - A x - B u
    for (int e = tid; e < D * D; e += blockDim.x) {
        const int i = e / D, j = e % D;
        double v = 0.0;
        if (i < N) {
            v = (j == N + i) ? 1.0 : 0.0;
        } else if (i < n) {
            const int k = i - N;
            if (j < n + m) {
                v = J[j][k];
            } else {
                double w = qdd0[k];
                for (int s = 0; s < n; ++s) w -= J[s][k] * x[s];
                for (int s = 0; s < m; ++s) w -= J[n + s][k] * u[s];
                v = w;
            }
        }
        Z[e] = v * dt;
    }
    __syncthreads();
    // scaling and squaring: Y = Z / 2^s with |Y|_1 <= 1/4, exp(Y) by the
    // degree-16 Taylor polynomial in Horner form (truncation below 1e-26 of
    // |exp(Y)|), then s squarings
    if (tid == 0) {
        double nrm = 0.0;
        for (int j = 0; j < D; ++j) {
            double c = 0.0;
            for (int i = 0; i < D; ++i) c += fabs(Z[i * D + j]);
            nrm = c > nrm ? c : nrm;
        }
        int s = 0;
        while (nrm > 0.25 && s < 64) {
            nrm *= 0.5;
            ++s;
        }
        s_scale = s;
    }
    __syncthreads();
    const double sc = ldexp(1.0, -s_scale);
    for (int e = tid; e < D * D; e += blockDim.x) {
        Z[e] *= sc;
        E[e] = (e / D == e % D ? 1.0 : 0.0) + Z[e] / 16.0;
    }
    __syncthreads();
    for (int k = 15; k >= 1; --k) {
        matmul_lds(D, Z, E, W);  // W = Y E
        for (int e = tid; e < D * D; e += blockDim.x)
            E[e] = (e / D == e % D ? 1.0 : 0.0) + W[e] / (double)k;
        __syncthreads();
    }
    for (int r = 0; r < s_scale; ++r) {
        matmul_lds(D, E, E, W);
        for (int e = tid; e < D * D; e += blockDim.x) E[e] = W[e];
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += blockDim.x) Ad[e] = (T)E[(e / n) * D + e % n];
    for (int e = tid; e < n * m; e += blockDim.x) Bd[e] = (T)E[(e / m) * D + n + e % m];
    if (tid < n) wd[tid] = (T)E[tid * D + n + m];
}

constexpr int STEP_THREADS = 64;

// Classical RK4 over dt in `sub` substeps, tau held; one wavefront.
template <typename T>
__global__ __launch_bounds__(STEP_THREADS) void nlink_step_kernel(
    int N, const T *__restrict__ mass_in, const T *__restrict__ len_in, double b, double dt,
    int sub, const T *x_in, const T *__restrict__ u_in, T *x_out) {
    __shared__ double mass[NLINK_MAX], len[NLINK_MAX], tau[NLINK_MAX];
    __shared__ double y[2 * NLINK_MAX], st[2 * NLINK_MAX], acc[2 * NLINK_MAX];
    __shared__ double Msh[NLINK_MAX * NLINK_MAX], qdd[NLINK_MAX];
    const int tid = threadIdx.x, n = 2 * N;
    if (tid < N) {
        mass[tid] = (double)mass_in[tid];
        len[tid] = (double)len_in[tid];
        tau[tid] = (double)u_in[tid];
    }
    if (tid < n) y[tid] = (double)x_in[tid];
    __syncthreads();
    const double h = dt / sub;
    const double wt[4] = {1.0, 2.0, 2.0, 1.0}, off[4] = {0.0, 0.5, 0.5, 1.0};
    for (int s = 0; s < sub; ++s) {
        if (tid < n) {
            st[tid] = y[tid];
            acc[tid] = 0.0;
        }
        __syncthreads();
        for (int stage = 0; stage < 4; ++stage) {
            forward_dynamics(N, mass, len, b, st, st + N, tau, Msh, qdd);
            // k = [qd; qdd] at the stage state; next stage state y + off h k
            double k = 0.0;
            if (tid < n) {
                k = tid < N ? st[N + tid] : qdd[tid - N];
                acc[tid] += wt[stage] * k;
            }
            __syncthreads();
            if (tid < n && stage < 3) st[tid] = y[tid] + off[stage + 1] * h * k;
            __syncthreads();
        }
        if (tid < n) y[tid] += h / 6.0 * acc[tid];
        __syncthreads();
    }
    if (tid < n) x_out[tid] = (T)y[tid];
}

}  // namespace

template <typename T>
hipError_t launch_nlink_linearize(int N, const T *mass, const T *len, double b, double dt,
                                  const T *x, const T *u, T *Ad, T *Bd, T *wd, hipStream_t s) {
    hipLaunchKernelGGL(nlink_linearize_kernel<T>, dim3(1), dim3(LIN_THREADS), 0, s, N, mass, len,
                       b, dt, x, u, Ad, Bd, wd);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_nlink_step(int N, const T *mass, const T *len, double b, double dt, int sub,
                             const T *x, const T *u, T *x_next, hipStream_t s) {
    hipLaunchKernelGGL(nlink_step_kernel<T>, dim3(1), dim3(STEP_THREADS), 0, s, N, mass, len, b,
                       dt, sub, x, u, x_next);
    return hipGetLastError();
}
template hipError_t launch_nlink_linearize<float>(int, const float *, const float *, double,
                                                  double, const float *, const float *, float *,
                                                  float *, float *, hipStream_t);
template hipError_t launch_nlink_linearize<double>(int, const double *, const double *, double,
                                                   double, const double *, const double *,
                                                   double *, double *, double *, hipStream_t);
template hipError_t launch_nlink_step<float>(int, const float *, const float *, double, double, int,
                                             const float *, const float *, float *, hipStream_t);
template hipError_t launch_nlink_step<double>(int, const double *, const double *, double, double,
                                              int, const double *, const double *, double *,
                                              hipStream_t);

}  // namespace empc

using namespace empc;

empc_status empc_fail_internal(empc_status s, const char *msg);

namespace {

empc_status check_robot(const empc_nlink *R, double dt) {
    if (!R) return empc_fail_internal(EMPC_EINVAL, "robot is NULL");
    if (R->dtype != EMPC_F32 && R->dtype != EMPC_F64)
        return empc_fail_internal(EMPC_EINVAL, "unknown dtype");
    if (R->links < 1) return empc_fail_internal(EMPC_EINVAL, "links must be >= 1");
    if (R->links > NLINK_MAX)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "more links than this build supports (16)");
    if (!R->mass || !R->length) return empc_fail_internal(EMPC_EINVAL, "mass and length are required");
    if (!isfinite(R->damping)) return empc_fail_internal(EMPC_EINVAL, "damping must be finite");
    if (!(dt > 0.0) || !isfinite(dt)) return empc_fail_internal(EMPC_EINVAL, "dt must be finite and > 0");
    return EMPC_OK;
}

empc_status launched(hipError_t e) {
    if (e == hipSuccess) return EMPC_OK;
    return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

empc_status empc_nlink_linearize(const empc_nlink *robot, double dt, const void *x,
                                 const void *u, void *Ad, void *Bd, void *wd, void *stream) {
    empc_status st = check_robot(robot, dt);
    if (st) return st;
    if (!x || !u || !Ad || !Bd || !wd)
        return empc_fail_internal(EMPC_EINVAL, "x, u, Ad, Bd and wd are required");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return launched(e);
    hipStream_t s = (hipStream_t)stream;
    const int N = robot->links;
    if (robot->dtype == EMPC_F32)
        e = launch_nlink_linearize<float>(N, (const float *)robot->mass, (const float *)robot->length,
                                          robot->damping, dt, (const float *)x, (const float *)u,
                                          (float *)Ad, (float *)Bd, (float *)wd, s);
    else
        e = launch_nlink_linearize<double>(N, (const double *)robot->mass,
                                           (const double *)robot->length, robot->damping, dt,
                                           (const double *)x, (const double *)u, (double *)Ad,
                                           (double *)Bd, (double *)wd, s);
    return launched(e);
}

empc_status empc_nlink_step(const empc_nlink *robot, double dt, int32_t substeps, const void *x,
                            const void *u, void *x_next, void *stream) {
    empc_status st = check_robot(robot, dt);
    if (st) return st;
    if (substeps < 1 || substeps > 1000000)
        return empc_fail_internal(EMPC_EINVAL, "substeps outside [1, 10^6]");
    if (!x || !u || !x_next) return empc_fail_internal(EMPC_EINVAL, "x, u and x_next are required");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return launched(e);
    hipStream_t s = (hipStream_t)stream;
    const int N = robot->links;
    if (robot->dtype == EMPC_F32)
        e = launch_nlink_step<float>(N, (const float *)robot->mass, (const float *)robot->length,
                                     robot->damping, dt, substeps, (const float *)x,
                                     (const float *)u, (float *)x_next, s);
    else
        e = launch_nlink_step<double>(N, (const double *)robot->mass, (const double *)robot->length,
                                      robot->damping, dt, substeps, (const double *)x,
                                      (const double *)u, (double *)x_next, s);
    return launched(e);
}

}  // extern "C"
