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
// qdd = e_j (one per thread), C(q, qd) one pass with qdd = 0, M is factored
// by Cholesky across the workgroup, and the Jacobian of the forward dynamics
// follows from differentiating RNEA(q, qd, qdd(q, qd, tau)) = tau - b qd:
// dqdd/dx_s = M^-1 (d(tau - b qd)/dx_s - dRNEA/dx_s |qdd fixed), the last
// term a forward-mode dual-number pass per direction (one per thread).  The
// zero-order hold works on the n x n state block (Phi and its integral)
// rather than on the augmented matrix.  Everything runs in FP64 (the model
// is tiny); outputs are written in the problem dtype.
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
// sine and cosine of an angle whose value's sine and cosine are known
__device__ inline void sincos_at(double, double s0, double c0, double *s, double *c) {
    *s = s0;
    *c = c0;
}
__device__ inline void sincos_at(Dual a, double s0, double c0, Dual *s, Dual *c) {
    *s = {s0, c0 * a.d};
    *c = {c0, -s0 * a.d};
}
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
// Loops run to NLINK_MAX with the links past N skipped, so that the
// per-link arrays live in registers (every index a compile-time constant).
// sphi, cphi: sine and cosine of the absolute angles at q (a table shared
// by all passes at the same q); a dual q carries its directional part into
// them by the chain rule.
template <typename S, typename QV, typename DV, typename AV>
__device__ __forceinline__ void rnea(int N, const double *mass, const double *len,
                                     const double *sphi, const double *cphi, const QV &q,
                                     const DV &qd, const AV &qdd, S *tau) {
    S ux[NLINK_MAX], uy[NLINK_MAX], ax[NLINK_MAX], ay[NLINK_MAX];
    S phi = make<S>(0, 0), om = make<S>(0, 0), al = make<S>(0, 0);
    S px = make<S>(0, 0), py = make<S>(0, 0);
#pragma unroll
    for (int i = 0; i < NLINK_MAX; ++i) {
        if (i < N) {
            phi = phi + q(i);
            om = om + qd(i);
            al = al + qdd(i);
            S sn, c;
            sincos_at(phi, sphi[i], cphi[i], &sn, &c);
            const S w2 = om * om;
            px = px + len[i] * (make<S>(0, 0) - al * sn - w2 * c);
            py = py + len[i] * (al * c - w2 * sn);
            ux[i] = c;
            uy[i] = sn;
            ax[i] = px;
            ay[i] = py;
        }
    }
    S fx = make<S>(0, 0), fy = make<S>(0, 0), t = make<S>(0, 0);
#pragma unroll
    for (int i = NLINK_MAX - 1; i >= 0; --i) {
        if (i < N) {
            fx = fx + mass[i] * ax[i];
            fy = fy + mass[i] * ay[i];
            t = t + len[i] * (ux[i] * fy - uy[i] * fx);
            tau[i] = t;
        }
    }
}

// Cholesky factor of the N x N matrix A (row-major, LDS) by every thread of
// the workgroup: column j is scaled by the threads of its rows, then the
// trailing block is updated in parallel; the strictly lower part of A
// receives L, dg the diagonal of L.  Must be reached by every thread.
__device__ void cholesky_par(int N, double *A, double *dg) {
    const int t = threadIdx.x;
    for (int j = 0; j < N; ++j) {
        const double d = sqrt(A[j * N + j]);
        if (t == j) dg[j] = d;
        if (t > j && t < N) A[t * N + j] /= d;
        __syncthreads();
        const int rem = N - j - 1;
        for (int e = t; e < rem * rem; e += blockDim.x) {
            const int i = j + 1 + e / rem, k = j + 1 + e % rem;
            if (k <= i) A[i * N + k] -= A[i * N + j] * A[k * N + j];
        }
        __syncthreads();
    }
}

// (L L^T)^-1 r with thread t < N holding r_t in yt (returned as y_t); each
// step's pivot goes through sh (N doubles of LDS).  Every thread.
__device__ double chol_solve_par(int N, const double *L, const double *dg, double yt,
                                 double *sh) {
    const int t = threadIdx.x;
    for (int j = 0; j < N; ++j) {  // L z = r
        if (t == j) {
            yt /= dg[j];
            sh[j] = yt;
        }
        __syncthreads();
        if (t > j && t < N) yt -= L[t * N + j] * sh[j];
    }
    for (int j = N - 1; j >= 0; --j) {  // L^T y = z
        if (t == j) {
            yt /= dg[j];
            sh[j] = yt;
        }
        __syncthreads();
        if (t < j) yt -= L[j * N + t] * sh[j];
    }
    return yt;
}

// (L L^T)^-1 r for one right-hand side held in registers by one thread (L,
// dg in LDS, read by every thread at the same address).
__device__ __forceinline__ void chol_solve_regs(int N, const double *L, const double *dg,
                                                double *y) {
#pragma unroll
    for (int i = 0; i < NLINK_MAX; ++i) {
        if (i < N) {
            double s = y[i];
#pragma unroll
            for (int k = 0; k < NLINK_MAX; ++k)
                if (k < i) s -= L[i * N + k] * y[k];
            y[i] = s / dg[i];
        }
    }
#pragma unroll
    for (int i = NLINK_MAX - 1; i >= 0; --i) {
        if (i < N) {
            double s = y[i];
#pragma unroll
            for (int k = 0; k < NLINK_MAX; ++k)
                if (k > i && k < N) s -= L[k * N + i] * y[k];
            y[i] = s / dg[i];
        }
    }
}

// Forward dynamics qdd = M^-1 (tau - C - b qd) at (q, qd) (LDS arrays) by the
// workgroup: threads 0..N-1 build M's columns, thread N the bias C, all of
// them factor M; the result qdd (LDS, N doubles) and the factor (Msh, dg)
// are left for the caller.  Must be reached by every thread.
// Sine and cosine of the absolute angles q_0 + .. + q_i, thread i (LDS).
// Must be reached by every thread.
__device__ void angle_table(int N, const double *q, double *sphi, double *cphi) {
    const int t = threadIdx.x;
    if (t < N) {
        double phi = 0.0;
        for (int i = 0; i <= t; ++i) phi += q[i];
        sincos(phi, &sphi[t], &cphi[t]);
    }
    __syncthreads();
}

// (inlined into its callers, so that its LDS arrays are addressed as LDS)
__device__ __forceinline__ void forward_dynamics(int N, const double *mass, const double *len,
                                                 double b,
                                 const double *q, const double *qd, const double *tau,
                                 double *Msh, double *dg, double *sh, double *sphi,
                                 double *cphi, double *qdd) {
    const int tid = threadIdx.x;
    auto zero = [](int) { return 0.0; };
    auto qv = [&](int i) { return q[i]; };
    double rhs = 0.0;
    angle_table(N, q, sphi, cphi);
    if (tid < N) {
        double col[NLINK_MAX];
        rnea<double>(N, mass, len, sphi, cphi, qv, zero,
                     [&](int i) { return i == tid ? 1.0 : 0.0; }, col);
#pragma unroll
        for (int i = 0; i < NLINK_MAX; ++i)
            if (i < N) Msh[i * N + tid] = col[i];
    } else if (tid == N) {
        double col[NLINK_MAX];
        rnea<double>(N, mass, len, sphi, cphi, qv, [&](int i) { return qd[i]; }, zero, col);
#pragma unroll
        for (int i = 0; i < NLINK_MAX; ++i)
            if (i < N) qdd[i] = tau[i] - col[i] - b * qd[i];
    }
    __syncthreads();
    if (tid < N) rhs = qdd[tid];
    cholesky_par(N, Msh, dg);
    rhs = chol_solve_par(N, Msh, dg, rhs, sh);
    __syncthreads();  // every read of sh done before qdd (maybe the same caller buffer) changes
    if (tid < N) qdd[tid] = rhs;
    __syncthreads();
}

constexpr int LIN_THREADS = 256;

// C = A B for n x n matrices in LDS (row-major, leading dimension n), all
// threads, a 2 x 2 block of C per thread
__device__ void matmul_lds(int n, const double *A, const double *B, double *C) {
    const int h = (n + 1) / 2;
    for (int e = threadIdx.x; e < h * h; e += blockDim.x) {
        const int i = 2 * (e / h), j = 2 * (e % h);
        const bool i1 = i + 1 < n, j1 = j + 1 < n;
        double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
        for (int k = 0; k < n; ++k) {
            const double a0 = A[i * n + k], a1 = i1 ? A[(i + 1) * n + k] : 0.0;
            const double b0 = B[k * n + j], b1 = j1 ? B[k * n + j + 1] : 0.0;
            c00 += a0 * b0;
            c01 += a0 * b1;
            c10 += a1 * b0;
            c11 += a1 * b1;
        }
        C[i * n + j] = c00;
        if (j1) C[i * n + j + 1] = c01;
        if (i1) C[(i + 1) * n + j] = c10;
        if (i1 && j1) C[(i + 1) * n + j + 1] = c11;
    }
    __syncthreads();
}

constexpr int NS_MAX = 2 * NLINK_MAX;  // states

template <typename T>
__global__ __launch_bounds__(LIN_THREADS) void nlink_linearize_kernel(
    int N, const T *__restrict__ mass_in, const T *__restrict__ len_in, double b, double dt,
    const T *__restrict__ x_in, const T *__restrict__ u_in, T *__restrict__ Ad,
    T *__restrict__ Bd, T *__restrict__ wd) {
    __shared__ double mass[NLINK_MAX], len[NLINK_MAX], x[NS_MAX], u[NLINK_MAX];
    __shared__ double Msh[NLINK_MAX * NLINK_MAX], dg[NLINK_MAX], sh[NLINK_MAX];
    __shared__ double sphi[NLINK_MAX], cphi[NLINK_MAX], qdd0[NLINK_MAX];
    __shared__ double J[3 * NLINK_MAX][NLINK_MAX];  // dqdd / d(q, qd, tau), column s
    __shared__ double Y[NS_MAX * NS_MAX], G[NS_MAX * NS_MAX], W[NS_MAX * NS_MAX];
    __shared__ double Ph[NS_MAX * NS_MAX], F[NS_MAX * (NLINK_MAX + 1)];
    __shared__ int s_scale;
    const int tid = threadIdx.x, n = 2 * N, m = N;
    if (tid < N) {
        mass[tid] = (double)mass_in[tid];
        len[tid] = (double)len_in[tid];
        u[tid] = (double)u_in[tid];
    }
    if (tid < n) x[tid] = (double)x_in[tid];
    __syncthreads();
    forward_dynamics(N, mass, len, b, x, x + N, u, Msh, dg, sh, sphi, cphi, qdd0);
    // direction s < 2N: state x_s; 2N <= s < 3N: torque s - 2N.  The
    // Jacobian of RNEA(q, qd, qdd0) in direction s by one dual-number pass.
    if (tid < 3 * N) {
        double y[NLINK_MAX];
        if (tid < n) {
            Dual t[NLINK_MAX];
            rnea<Dual>(
                N, mass, len, sphi, cphi, [&](int i) { return Dual{x[i], i == tid ? 1.0 : 0.0}; },
                [&](int i) { return Dual{x[N + i], N + i == tid ? 1.0 : 0.0}; },
                [&](int i) { return Dual{qdd0[i], 0.0}; }, t);
#pragma unroll
            for (int i = 0; i < NLINK_MAX; ++i)
                if (i < N) y[i] = -t[i].d - (N + i == tid ? b : 0.0);
        } else {
#pragma unroll
            for (int i = 0; i < NLINK_MAX; ++i) y[i] = i == tid - n ? 1.0 : 0.0;
        }
        chol_solve_regs(N, Msh, dg, y);
#pragma unroll
        for (int i = 0; i < NLINK_MAX; ++i)
            if (i < N) J[tid][i] = y[i];
    }
    __syncthreads();
    // f(x, u) ~ f0 + A (x' - x) + B (u' - u): A = [[0, I], [Jq, Jqd]],
    // B = [[0], [Ju]], offset w = f0 - A x - B u (position rows: 0).
    // F holds [B | w] (n x (m + 1)); Y = A dt first, scaled below.
    const int m1 = m + 1;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        Y[e] = (i < N ? (j == N + i ? 1.0 : 0.0) : J[j][i - N]) * dt;
    }
    for (int e = tid; e < n * m1; e += blockDim.x) {
        const int i = e / m1, j = e % m1;
        double v = 0.0;
        if (i >= N) {
            const int k = i - N;
            if (j < m) {
                v = J[n + j][k];
            } else {
                v = qdd0[k];
                for (int s2 = 0; s2 < n; ++s2) v -= J[s2][k] * x[s2];
                for (int s2 = 0; s2 < m; ++s2) v -= J[n + s2][k] * u[s2];
            }
        }
        F[e] = v;
    }
    __syncthreads();
    // Zero-order hold: Phi = exp(A dt), Gamma = int_0^dt exp(A s) ds, then
    // A_d = Phi, [B_d w_d] = Gamma [B w].  Scaling and squaring on
    // h = dt / 2^s with |A h|_1 <= 1/4: G = sum_k (A h)^k / (k+1)! by a
    // degree-14 Horner scheme (truncation below 1e-20), Phi(h) = I + A h G,
    // Gamma(h) = h G; each squaring Gamma <- Gamma + Phi Gamma,
    // Phi <- Phi Phi.  The column sums of |Y| and their maximum by the first
    // wavefront.
    if (tid < 64) {
        double c = 0.0;
        if (tid < n)
            for (int i = 0; i < n; ++i) c += fabs(Y[i * n + tid]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) c = fmax(c, __shfl_xor(c, o, 64));
        if (tid == 0) {
            int sc = 0;
            while (c > 0.25 && sc < 64) {
                c *= 0.5;
                ++sc;
            }
            s_scale = sc;
        }
    }
    __syncthreads();
    const int sc = s_scale;
    const double scl = ldexp(1.0, -sc), h = dt * scl;
    for (int e = tid; e < n * n; e += blockDim.x) {
        Y[e] *= scl;
        G[e] = (e / n == e % n ? 1.0 : 0.0) + Y[e] / 15.0;
    }
    __syncthreads();
    for (int k = 13; k >= 1; --k) {  // G <- I + Y G / (k + 1)
        matmul_lds(n, Y, G, W);
        for (int e = tid; e < n * n; e += blockDim.x)
            G[e] = (e / n == e % n ? 1.0 : 0.0) + W[e] / (double)(k + 1);
        __syncthreads();
    }
    matmul_lds(n, Y, G, W);
    for (int e = tid; e < n * n; e += blockDim.x) {
        Ph[e] = (e / n == e % n ? 1.0 : 0.0) + W[e];
        G[e] *= h;
    }
    __syncthreads();
    for (int r = 0; r < sc; ++r) {
        matmul_lds(n, Ph, G, W);  // Phi Gamma
        for (int e = tid; e < n * n; e += blockDim.x) G[e] += W[e];
        __syncthreads();
        matmul_lds(n, Ph, Ph, W);
        for (int e = tid; e < n * n; e += blockDim.x) Ph[e] = W[e];
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += blockDim.x) Ad[e] = (T)Ph[e];
    for (int e = tid; e < n * m1; e += blockDim.x) {
        const int i = e / m1, j = e % m1;
        double v = 0.0;
        for (int k = 0; k < n; ++k) v += G[i * n + k] * F[k * m1 + j];
        if (j < m)
            Bd[i * m + j] = (T)v;
        else
            wd[i] = (T)v;
    }
}

constexpr int STEP_THREADS = 64;

// Classical RK4 over dt in `sub` substeps, tau held; one wavefront.
template <typename T>
__global__ __launch_bounds__(STEP_THREADS) void nlink_step_kernel(
    int N, const T *__restrict__ mass_in, const T *__restrict__ len_in, double b, double dt,
    int sub, const T *x_in, const T *__restrict__ u_in, T *x_out) {
    __shared__ double mass[NLINK_MAX], len[NLINK_MAX], tau[NLINK_MAX];
    __shared__ double st[NS_MAX];
    __shared__ double Msh[NLINK_MAX * NLINK_MAX], dg[NLINK_MAX], sh[NLINK_MAX], qdd[NLINK_MAX];
    __shared__ double sphi[NLINK_MAX], cphi[NLINK_MAX];
    const int tid = threadIdx.x, n = 2 * N;
    if (tid < N) {
        mass[tid] = (double)mass_in[tid];
        len[tid] = (double)len_in[tid];
        tau[tid] = (double)u_in[tid];
    }
    // thread i < n keeps state i (y), its RK4 sum (acc) in registers
    double y = tid < n ? (double)x_in[tid] : 0.0;
    const double hs = dt / sub;
    for (int s = 0; s < sub; ++s) {
        double acc = 0.0;
        if (tid < n) st[tid] = y;
        __syncthreads();
        // the four stages share one inlined copy of the dynamics; weights
        // 1, 2, 2, 1 and next-stage offsets 0.5, 0.5, 1
#pragma unroll 1
        for (int stage = 0; stage < 4; ++stage) {
            forward_dynamics(N, mass, len, b, st, st + N, tau, Msh, dg, sh, sphi, cphi, qdd);
            // k = [qd; qdd] at the stage state; next stage state y + off h k
            double k = 0.0;
            if (tid < n) {
                k = tid < N ? st[N + tid] : qdd[tid - N];
                acc += (stage == 0 || stage == 3 ? 1.0 : 2.0) * k;
            }
            __syncthreads();
            if (tid < n && stage < 3) st[tid] = y + (stage == 2 ? 1.0 : 0.5) * hs * k;
            __syncthreads();
        }
        if (tid < n) y += hs / 6.0 * acc;
    }
    if (tid < n) x_out[tid] = (T)y;
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
        return empc_fail_internal(EMPC_EUNSUPPORTED, "more links than the library supports (16)");
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
