// Parameterized small-matrix convex MPC on the GPU (gfx950): the paper's
// other method (Sec. IV-B small-matrix formulation, parameterized as in
// Sec. IV-E), for linear problems.  With z the knot vector, the states
// x_1..x_T = S z + v and the cost of eq. 3 is J(z) = z^T P z + 2 q^T z + c;
// the knot bounds make the MPC a box-constrained QP.
//  - qp_traj_kernel: S and v.  One workgroup per column: the response of
//    unit knot j from rest (column j of S, built step by step as the paper
//    describes, each row the previous one times A_d plus B_d in the knot's
//    proportions), and one workgroup for the free response v from x0 with
//    w_d; one thread per state row, the state exchanged through LDS each
//    step (the paper's own thread-per-state layout: the work is tiny).
//  - qp_gram_kernel: P = S^T Qb S + Phi^T Rb Phi, 16 x 16 output tiles with
//    the shared dimension T n staged through LDS; the input part in closed
//    form from the knot weights.  qp_lin_kernel: q and c.
//  - qp_box_kernel: the box QP by the projected Newton method (Bertsekas
//    1982): Newton steps of the quadratic restricted to the variables off
//    their bounds (Cholesky solves), an Armijo search along the projection
//    arc; one workgroup.
// Every step computes in FP64; inputs and outputs are in the problem dtype.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace empc {

namespace {

constexpr int TRAJ_THREADS = 128;  // >= the largest linear state count (80)
constexpr int QP_THREADS = 1024;
constexpr int QP_MAX_PM = 1024;    // one knot parameter per QP thread

// weight of knot a at step k (u_k = (1-c) U_idx1 + c U_idx2)
__device__ inline double knot_weight(int T, int p, int k, int a) {
    const Knot s = knot_at(T, p, k);
    const double c = (double)s.rem / (double)s.den;
    return (a == s.a ? 1.0 - c : 0.0) + (a == s.b ? c : 0.0);
}

template <typename T>
__global__ __launch_bounds__(TRAJ_THREADS) void qp_traj_kernel(ProbView<T> P,
                                                               const T *__restrict__ x0,
                                                               double *__restrict__ S,
                                                               double *__restrict__ v) {
    __shared__ double x[2][TRAJ_THREADS];
    const int n = P.n, m = P.m, pm = P.p * P.m, r = threadIdx.x;
    const int j = blockIdx.x;  // column; j == pm: the free response
    const bool free_resp = j == pm;
    const int aj = free_resp ? 0 : j / m, ij = free_resp ? 0 : j % m;
    if (r < n) x[0][r] = free_resp ? (double)x0[r] : 0.0;
    __syncthreads();
    for (int k = 0; k < P.Tn; ++k) {
        const double *xc = x[k & 1];
        if (r < n) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += (double)P.Ad[r * n + c] * xc[c];
            if (free_resp) {
                if (P.wd) s += (double)P.wd[r];
            } else {
                s += (double)P.Bd[r * m + ij] * knot_weight(P.Tn, P.p, k, aj);
            }
            x[(k + 1) & 1][r] = s;
            if (free_resp)
                v[(int64_t)k * n + r] = s;
            else
                S[((int64_t)k * n + r) * pm + j] = s;
        }
        __syncthreads();
    }
}

// weight of state row K = k n + r of the stacked cost: q_r (+ qf_r at x_T)
template <typename T>
__device__ inline double row_weight(const ProbView<T> &P, int K) {
    const int k = K / P.n, r = K % P.n;
    double w = (double)P.q[r];
    if (k == P.Tn - 1 && P.qf) w += (double)P.qf[r];
    return w;
}

template <typename T>
__global__ __launch_bounds__(256) void qp_gram_kernel(ProbView<T> P, const double *__restrict__ S,
                                                      T *__restrict__ Pout) {
    __shared__ double As[16][17], Bs[16][17];
    const int pm = P.p * P.m, K = P.Tn * P.n;
    const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
    const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
    double acc = 0.0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        // thread (ti, tj) stages row k0 + ti, columns i0 + tj / j0 + tj
        const int kr = k0 + ti;
        double a = 0.0, b = 0.0;
        if (kr < K) {
            const double w = row_weight(P, kr);
            if (i0 + tj < pm) a = w * S[(int64_t)kr * pm + i0 + tj];
            if (j0 + tj < pm) b = S[(int64_t)kr * pm + j0 + tj];
        }
        As[ti][tj] = a;
        Bs[ti][tj] = b;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc += As[kk][ti] * Bs[kk][tj];
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i < pm && j < pm) {
        const int m = P.m;
        if (i % m == j % m) {
            // input part: sum_k w_k(knot of i) w_k(knot of j) r_input
            double s = 0.0;
            for (int k = 0; k < P.Tn; ++k)
                s += knot_weight(P.Tn, P.p, k, i / m) * knot_weight(P.Tn, P.p, k, j / m);
            acc += s * (double)P.r[i % m];
        }
        Pout[(int64_t)i * pm + j] = (T)acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void qp_lin_kernel(ProbView<T> P, const double *__restrict__ S,
                                                     const double *__restrict__ v,
                                                     T *__restrict__ qout, T *__restrict__ cout) {
    __shared__ double part[256];
    const int pm = P.p * P.m, K = P.Tn * P.n, m = P.m;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < pm) {
        double s = 0.0;
        for (int kr = 0; kr < K; ++kr) {
            const double g = P.xg ? (double)P.xg[kr % P.n] : 0.0;
            s += S[(int64_t)kr * pm + i] * row_weight(P, kr) * (v[kr] - g);
        }
        if (P.ug) {
            double wsum = 0.0;
            for (int k = 0; k < P.Tn; ++k) wsum += knot_weight(P.Tn, P.p, k, i / m);
            s -= wsum * (double)P.r[i % m] * (double)P.ug[i % m];
        }
        qout[i] = (T)s;
    }
    if (blockIdx.x == 0) {
        double s = 0.0;
        for (int kr = threadIdx.x; kr < K; kr += blockDim.x) {
            const double e = v[kr] - (P.xg ? (double)P.xg[kr % P.n] : 0.0);
            s += row_weight(P, kr) * e * e;
        }
        if (P.ug)
            for (int ii = threadIdx.x; ii < m; ii += blockDim.x)
                s += (double)P.Tn * (double)P.r[ii] * (double)P.ug[ii] * (double)P.ug[ii];
        part[threadIdx.x] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) *cout = (T)part[0];
    }
}

// sum over the workgroup (every thread gets it)
__device__ inline double block_sum(double x, double *red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = QP_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// max over the workgroup (every thread gets it)
__device__ inline double block_max(double x, double *red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = QP_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Box QP min f(z) = z^T P z + 2 q^T z, lo <= z <= hi, by Bertsekas' projected
// Newton method (SIAM J. Control Optim. 20, 1982): with g = 2 (P z + q) and
// w = |z - clip(z - g)|_inf, the variables within min(eps, w) of a bound
// whose gradient points out of the box are held on a scaled gradient step,
// the rest take the Newton step of the reduced quadratic (a Cholesky solve
// of P on the free variables), and the step is cut back along the
// projection arc until the Armijo condition f(z) - f(z') >= sigma g^T (z -
// z') holds.  Globally convergent for a positive definite P; once the active
// set is the optimal one the full Newton step lands on the minimizer.
template <typename T>
__global__ __launch_bounds__(QP_THREADS) void qp_box_kernel(
    int pm, int m, const T *__restrict__ umin, const T *__restrict__ umax,
    const T *__restrict__ Pm, const T *__restrict__ qv, const T *__restrict__ cp, int max_iter,
    double *__restrict__ H, T *__restrict__ zout, T *__restrict__ cost, int *__restrict__ info) {
    __shared__ double z[QP_MAX_PM], d[QP_MAX_PM], y[QP_MAX_PM], red[QP_THREADS];
    __shared__ int act[QP_MAX_PM], idx[QP_MAX_PM], s_nfree;
    const int i = threadIdx.x;
    const bool mine = i < pm;
    const double lo = mine ? (double)umin[i % m] : 0.0, hi = mine ? (double)umax[i % m] : 0.0;
    const double qi = mine ? (double)qv[i] : 0.0;
    const double pii = mine ? (double)Pm[(int64_t)i * pm + i] : 1.0;
    auto clip = [&](double v) { return v < lo ? lo : (v > hi ? hi : v); };
    // (P v)_i for v in LDS
    auto pdot = [&](const double *v) {
        double s = 0.0;
        if (mine)
            for (int j = 0; j < pm; ++j) s += (double)Pm[(int64_t)i * pm + j] * v[j];
        return s;
    };
    if (mine) z[i] = clip(0.0);
    __syncthreads();
    double pz = pdot(z);
    double f = block_sum(mine ? z[i] * (pz + 2.0 * qi) : 0.0, red);
    int it = 0, converged = 0;
    const double eps0 = 1e-3;
    for (; it < max_iter; ++it) {
        const double g = mine ? 2.0 * (pz + qi) : 0.0;
        const double w = block_max(mine ? fabs(z[i] - clip(z[i] - g)) : 0.0, red);
        const double gs = block_max(mine ? fabs(g) : 0.0, red);
        if (w <= 1e-14 * (1.0 + gs)) {
            converged = 1;
            break;
        }
        const double eps = w < eps0 ? w : eps0;
        int a = 0;
        if (mine) a = (z[i] <= lo + eps && g > 0.0) || (z[i] >= hi - eps && g < 0.0);
        if (mine) act[i] = a;
        __syncthreads();
        if (i == 0) {
            int c = 0;
            for (int t = 0; t < pm; ++t)
                if (!act[t]) idx[c++] = t;
            s_nfree = c;
        }
        __syncthreads();
        const int nf = s_nfree;
        // Newton step on the free variables: P_FF d_F = -(P z + q)_F
        for (int e = i; e < nf * nf; e += QP_THREADS) {
            const int r = e / nf, c = e % nf;
            H[e] = (double)Pm[(int64_t)idx[r] * pm + idx[c]];
        }
        if (mine && !a) d[i] = -(pz + qi);  // gathered below
        if (mine && a) d[i] = -g / (2.0 * pii);
        __syncthreads();
        if (i < nf) y[i] = d[idx[i]];
        __syncthreads();
        for (int k = 0; k < nf; ++k) {
            if (i == 0) H[k * nf + k] = sqrt(H[k * nf + k]);
            __syncthreads();
            const double dk = H[k * nf + k];
            for (int r = k + 1 + i; r < nf; r += QP_THREADS) H[r * nf + k] /= dk;
            __syncthreads();
            const int wdt = nf - k - 1;
            for (int e = i; e < wdt * wdt; e += QP_THREADS) {
                const int r = k + 1 + e / wdt, c = k + 1 + e % wdt;
                if (c <= r) H[r * nf + c] -= H[r * nf + k] * H[c * nf + k];
            }
            __syncthreads();
        }
        for (int k = 0; k < nf; ++k) {
            if (i == 0) y[k] /= H[k * nf + k];
            __syncthreads();
            for (int r = k + 1 + i; r < nf; r += QP_THREADS) y[r] -= H[r * nf + k] * y[k];
            __syncthreads();
        }
        for (int k = nf - 1; k >= 0; --k) {
            if (i == 0) y[k] /= H[k * nf + k];
            __syncthreads();
            for (int r = i; r < k; r += QP_THREADS) y[r] -= H[k * nf + r] * y[k];
            __syncthreads();
        }
        if (i < nf) d[idx[i]] = y[i];
        __syncthreads();
        // Armijo search along the projection arc
        const double z_old = mine ? z[i] : 0.0;
        double alpha = 1.0, pz_new = pz, f_new = f;
        bool moved = false;
        for (int ls = 0; ls < 60; ++ls) {
            const double zt = mine ? clip(z_old + alpha * d[i]) : 0.0;
            __syncthreads();
            if (mine) y[i] = zt;
            __syncthreads();
            pz_new = pdot(y);
            f_new = block_sum(mine ? zt * (pz_new + 2.0 * qi) : 0.0, red);
            const double dec = block_sum(mine ? g * (z_old - zt) : 0.0, red);
            if (f - f_new >= 1e-4 * dec) {
                moved = true;
                break;
            }
            alpha *= 0.5;
        }
        if (!moved) {  // no decrease left at rounding level
            converged = 1;
            break;
        }
        // a step below rounding of z: nothing left to gain
        const double step = block_max(mine ? fabs(y[i] - z_old) : 0.0, red);
        const double zmax = block_max(mine ? fabs(z_old) : 0.0, red);
        if (mine) z[i] = y[i];
        pz = pz_new;
        f = f_new;
        __syncthreads();
        if (step <= 1e-15 * (1.0 + zmax)) {
            converged = 1;
            ++it;
            break;
        }
    }
    if (mine) zout[i] = (T)z[i];
    if (i == 0) {
        *cost = (T)(f + (double)*cp);
        info[0] = it;
        info[1] = converged;
    }
}

}  // namespace

size_t qp_workspace_bytes(int n, int T, int pm) {
    const size_t S = (size_t)T * n * pm, v = (size_t)T * n, H = (size_t)pm * pm;
    return ((S + 31) / 32 * 32 + (v + 31) / 32 * 32 + H) * sizeof(double);
}

template <typename T>
hipError_t launch_qp_form(const ProbView<T> &P, const T *x0, void *ws, T *Pout, T *qout, T *cout,
                          hipStream_t s) {
    const int pm = P.p * P.m, n = P.n;
    double *S = (double *)ws;
    double *v = S + ((size_t)P.Tn * n * pm + 31) / 32 * 32;
    hipLaunchKernelGGL(qp_traj_kernel<T>, dim3(pm + 1), dim3(TRAJ_THREADS), 0, s, P, x0, S, v);
    const unsigned tiles = (unsigned)((pm + 15) / 16);
    hipLaunchKernelGGL(qp_gram_kernel<T>, dim3(tiles, tiles), dim3(256), 0, s, P, S, Pout);
    hipLaunchKernelGGL(qp_lin_kernel<T>, dim3((pm + 255) / 256), dim3(256), 0, s, P, S, v, qout,
                       cout);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_qp_solve(const ProbView<T> &P, const T *Pm, const T *q, const T *c, void *ws,
                           int max_iter, T *z, T *cost, int *info, hipStream_t s) {
    const int pm = P.p * P.m, n = P.n;
    double *H = (double *)ws + ((size_t)P.Tn * n * pm + 31) / 32 * 32 + ((size_t)P.Tn * n + 31) / 32 * 32;
    hipLaunchKernelGGL(qp_box_kernel<T>, dim3(1), dim3(QP_THREADS), 0, s, pm, P.m, P.umin, P.umax,
                       Pm, q, c, max_iter, H, z, cost, info);
    return hipGetLastError();
}

template hipError_t launch_qp_form<float>(const ProbView<float> &, const float *, void *, float *,
                                          float *, float *, hipStream_t);
template hipError_t launch_qp_form<double>(const ProbView<double> &, const double *, void *,
                                           double *, double *, double *, hipStream_t);
template hipError_t launch_qp_solve<float>(const ProbView<float> &, const float *, const float *,
                                           const float *, void *, int, float *, float *, int *,
                                           hipStream_t);
template hipError_t launch_qp_solve<double>(const ProbView<double> &, const double *,
                                            const double *, const double *, void *, int, double *,
                                            double *, int *, hipStream_t);

}  // namespace empc

using namespace empc;

empc_status empc_validate_problem_internal(const empc_problem *P);
empc_status empc_fail_internal(empc_status s, const char *msg);

namespace {

empc_status check_qp_problem(const empc_problem *P) {
    empc_status st = empc_validate_problem_internal(P);
    if (st) return st;
    if (P->model != EMPC_LINEAR)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "the convex form needs a linear model");
    if (P->qb) return empc_fail_internal(EMPC_EUNSUPPORTED, "the state box penalty is not quadratic");
    if (P->Q || P->R || P->Qf)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "the convex form takes diagonal weights");
    if (P->p * P->m > QP_MAX_PM)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "more than 1024 knot parameters");
    return EMPC_OK;
}

empc_status qp_launched(hipError_t e) {
    if (e == hipSuccess) return EMPC_OK;
    return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t empc_qp_workspace_bytes(const empc_problem *prob) {
    if (check_qp_problem(prob)) return 0;
    return qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m);
}

empc_status empc_qp_form(const empc_problem *prob, const void *x0, void *workspace,
                         size_t ws_bytes, void *P, void *q, void *c, void *stream) {
    empc_status st = check_qp_problem(prob);
    if (st) return st;
    if (!x0 || !P || !q || !c) return empc_fail_internal(EMPC_EINVAL, "x0, P, q and c are required");
    if (!workspace || ws_bytes < qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m))
        return empc_fail_internal(EMPC_EWORKSPACE, "convex workspace too small");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qp_launched(e);
    hipStream_t s = (hipStream_t)stream;
    if (prob->dtype == EMPC_F32)
        e = launch_qp_form<float>(view_of<float>(*prob), (const float *)x0, workspace, (float *)P,
                                  (float *)q, (float *)c, s);
    else
        e = launch_qp_form<double>(view_of<double>(*prob), (const double *)x0, workspace,
                                   (double *)P, (double *)q, (double *)c, s);
    return qp_launched(e);
}

empc_status empc_qp_solve(const empc_problem *prob, const void *P, const void *q, const void *c,
                          void *workspace, size_t ws_bytes, int32_t max_iter, void *z, void *cost,
                          int32_t *info, void *stream) {
    empc_status st = check_qp_problem(prob);
    if (st) return st;
    if (!P || !q || !c || !z || !cost || !info)
        return empc_fail_internal(EMPC_EINVAL, "P, q, c, z, cost and info are required");
    if (max_iter < 1) return empc_fail_internal(EMPC_EINVAL, "max_iter must be >= 1");
    if (!workspace || ws_bytes < qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m))
        return empc_fail_internal(EMPC_EWORKSPACE, "convex workspace too small");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qp_launched(e);
    hipStream_t s = (hipStream_t)stream;
    if (prob->dtype == EMPC_F32)
        e = launch_qp_solve<float>(view_of<float>(*prob), (const float *)P, (const float *)q,
                                   (const float *)c, workspace, max_iter, (float *)z,
                                   (float *)cost, (int *)info, s);
    else
        e = launch_qp_solve<double>(view_of<double>(*prob), (const double *)P, (const double *)q,
                                    (const double *)c, workspace, max_iter, (double *)z,
                                    (double *)cost, (int *)info, s);
    return qp_launched(e);
}

}  // extern "C"
