// Adjoint gradient of the rollout cost with respect to the knots, and Adam
// refinement built on it (gfx950).
//
// One wavefront (one workgroup of 64 lanes) per candidate.  Linear model:
// lane i owns state i (n <= 64) and, for i < m, input i; the state vector is
// exchanged through LDS each step and A_d, B_d sit in LDS.  Pendulum chain:
// lane j owns joint j (d <= 64); the cumulative angles, gravity torques and
// the adjoint's prefix / suffix sums are wavefront scans.
//
// With lambda_k = dJ/dx_k:
//   lambda_T = 2 (Q + Q_f)(x_T - g),
//   lambda_k = 2 Q (x_k - g) + f_x(x_k, u_k)^T lambda_{k+1},
//   dJ/du_k  = 2 R (u_k - u_g) + f_u(x_k, u_k)^T lambda_{k+1},
// and dJ/du_k goes to knots idx1 and idx2 with weights 1-c and c.  States
// are stored every S = ceil(sqrt(T)) steps on the forward pass; the backward
// pass recomputes each segment of S states from its checkpoint.
#include <math.h>

#include "internal.hpp"

namespace empc {

template <typename T>
__device__ inline T wsum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// inclusive prefix sum over lanes 0..63
template <typename T>
__device__ inline T scan_up(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}
// inclusive suffix sum over lanes 63..0
template <typename T>
__device__ inline T scan_down(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_down(v, o, 64);
        if (lane + o < 64) v += y;
    }
    return v;
}

template <typename T>
__device__ inline T sin_f(T x);
template <>
__device__ inline float sin_f<float>(float x) { return sinf(x); }
template <>
__device__ inline double sin_f<double>(double x) { return sin(x); }
template <typename T>
__device__ inline T cos_f(T x);
template <>
__device__ inline float cos_f<float>(float x) { return cosf(x); }
template <>
__device__ inline double cos_f<double>(double x) { return cos(x); }

// LDS plan (element counts), shared with the host-side size check.
struct GradPlan {
    int S, nchk;
    size_t oA, oB, oU, oG, oM1, oM2, oX, oUin, oChk, oSeg, total;
};
inline GradPlan grad_plan(int model, int n, int m, int T, int p) {
    GradPlan g;
    g.S = 1;
    while (g.S * g.S < T) ++g.S;
    g.nchk = (T + g.S - 1) / g.S;
    const size_t pm = (size_t)p * m;
    size_t o = 0;
    g.oA = o; o += model == EMPC_LINEAR ? (size_t)n * n : 0;
    g.oB = o; o += model == EMPC_LINEAR ? (size_t)n * m : 0;
    g.oU = o; o += pm;
    g.oG = o; o += pm;
    g.oM1 = o; o += pm;
    g.oM2 = o; o += pm;
    g.oX = o; o += 64;
    g.oUin = o; o += 64;
    g.oChk = o; o += (size_t)g.nchk * n;
    g.oSeg = o; o += (size_t)g.S * n;
    g.total = o;
    return g;
}

template <typename T>
struct Lane {
    // per-lane constants (linear: state/input role; chain: joint role)
    T q, qf, xg, r, ug, w;                // linear state i / input i
    T cg, invI, kst, dmp, wq, wv, wqf, wvf, gq, gv, wr, gu;  // chain joint j
};

template <typename T>
__global__ __launch_bounds__(64) void adjoint_kernel(ProbView<T> P, int model, GradPlan G,
                                                     const T *__restrict__ x0,
                                                     const T *__restrict__ knots, int64_t ld,
                                                     T *__restrict__ dJ, T *__restrict__ cost,
                                                     int steps, T lr, T *__restrict__ knots_io,
                                                     T *__restrict__ cost_io) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    T *sA = sm + G.oA, *sB = sm + G.oB, *sU = sm + G.oU, *sG = sm + G.oG;
    T *sM1 = sm + G.oM1, *sM2 = sm + G.oM2, *sX = sm + G.oX, *sUin = sm + G.oUin;
    T *sChk = sm + G.oChk, *sSeg = sm + G.oSeg;
    const int lane = threadIdx.x;
    const int64_t cand = blockIdx.x;
    const int n = P.n, m = P.m, pm = P.p * P.m, Tn = P.Tn, S = G.S;
    const bool lin = model == EMPC_LINEAR;
    const bool refine = steps > 0;

    // ---- load
    if (lin) {
        for (int t = lane; t < n * n; t += 64) sA[t] = P.Ad[t];
        for (int t = lane; t < n * m; t += 64) sB[t] = P.Bd[t];
    }
    const T *src = refine ? knots_io : knots;
    for (int j = lane; j < pm; j += 64) {
        sU[j] = src[(int64_t)j * ld + cand];
        sM1[j] = 0;
        sM2[j] = 0;
    }
    Lane<T> L;
    if (lin) {
        const bool si = lane < n, ui = lane < m;
        L.q = si ? P.q[lane] : (T)0;
        L.qf = (si && P.qf) ? P.qf[lane] : (T)0;
        L.xg = (si && P.xg) ? P.xg[lane] : (T)0;
        L.w = (si && P.wd) ? P.wd[lane] : (T)0;
        L.r = ui ? P.r[lane] : (T)0;
        L.ug = (ui && P.ug) ? P.ug[lane] : (T)0;
    } else {
        const int d = m;
        const bool in = lane < d;
        T tail = 0, inert = 0, dist = 0;
        if (in) {
            for (int i = lane; i < d; ++i) {
                tail += P.mass[i];
                dist += P.len[i];
                inert += P.mass[i] * dist * dist;
            }
        }
        L.cg = in ? P.gravity * P.len[lane] * tail : (T)0;
        L.invI = in ? (T)1 / inert : (T)0;
        L.kst = in ? P.stiff[lane] : (T)0;
        L.dmp = in ? P.damp[lane] : (T)0;
        L.wq = in ? P.q[lane] : (T)0;
        L.wv = in ? P.q[d + lane] : (T)0;
        L.wqf = (in && P.qf) ? P.qf[lane] : (T)0;
        L.wvf = (in && P.qf) ? P.qf[d + lane] : (T)0;
        L.gq = (in && P.xg) ? P.xg[lane] : (T)0;
        L.gv = (in && P.xg) ? P.xg[d + lane] : (T)0;
        L.wr = in ? P.r[lane] : (T)0;
        L.gu = (in && P.ug) ? P.ug[lane] : (T)0;
    }
    __syncthreads();

    const int d = m;  // chain joints
    // lane-owned state: linear xi (state lane); chain (q, v) of joint lane
    auto input_at = [&](int k) -> T {  // lane's own input at step k (lane < m)
        const Knot kn = knot_at(Tn, P.p, k);
        const T c = (T)kn.rem / (T)kn.den;
        if (lane >= m) return (T)0;
        return ((T)1 - c) * sU[kn.a * m + lane] + c * sU[kn.b * m + lane];
    };
    // one linear step: xi <- A x + B u + w (u of this step in sUin)
    auto lin_step = [&](T xi) -> T {
        if (lane < n) sX[lane] = xi;
        __syncthreads();
        T s = L.w;
        if (lane < n) {
            for (int j = 0; j < n; ++j) s += sA[lane * n + j] * sX[j];
            for (int j = 0; j < m; ++j) s += sB[lane * m + j] * sUin[j];
        }
        __syncthreads();
        return lane < n ? s : (T)0;
    };
    auto chain_step = [&](T &q, T &v, T u) {
        const T phi = scan_up(q);
        const T sg = L.cg * sin_f<T>(phi);
        const T Gj = scan_down(sg);
        const T acc = (u - L.kst * q - L.dmp * v - Gj) * L.invI;
        v = v + P.dt * acc;
        q = q + P.dt * v;
    };

    // forward pass: returns J; stores checkpoints when chk != 0
    auto forward = [&](bool chk, T &xi, T &qj, T &vj) -> T {
        T J = 0;
        xi = (lin && lane < n) ? x0[lane] : (T)0;
        qj = (!lin && lane < d) ? x0[lane] : (T)0;
        vj = (!lin && lane < d) ? x0[d + lane] : (T)0;
        for (int k = 0; k < Tn; ++k) {
            if (chk && k % S == 0) {
                if (lin) {
                    if (lane < n) sChk[(k / S) * n + lane] = xi;
                } else if (lane < d) {
                    sChk[(k / S) * n + lane] = qj;
                    sChk[(k / S) * n + d + lane] = vj;
                }
            }
            const T u = input_at(k);
            if (lin) {
                if (lane < m) sUin[lane] = u;
                xi = lin_step(xi);
                const T e = L.xg - xi, eu = L.ug - u;
                J += L.q * e * e + L.r * eu * eu;
            } else {
                chain_step(qj, vj, u);
                const T eq = L.gq - qj, ev = L.gv - vj, eu = L.gu - u;
                J += L.wq * eq * eq + L.wv * ev * ev + L.wr * eu * eu;
            }
        }
        if (lin) {
            const T e = L.xg - xi;
            J += L.qf * e * e;
        } else {
            const T eq = L.gq - qj, ev = L.gv - vj;
            J += L.wqf * eq * eq + L.wvf * ev * ev;
        }
        return wsum(J);
    };

    // backward pass from the final state: fills sG with dJ/dknots
    auto backward = [&](T xT, T qT, T vT) {
        for (int j = lane; j < pm; j += 64) sG[j] = 0;
        T lam = 0, lq = 0, lv = 0;
        if (lin) {
            lam = (T)2 * (L.q + L.qf) * (xT - L.xg);
        } else {
            lq = (T)2 * (L.wq + L.wqf) * (qT - L.gq);
            lv = (T)2 * (L.wv + L.wvf) * (vT - L.gv);
        }
        __syncthreads();
        for (int sg = G.nchk - 1; sg >= 0; --sg) {
            const int k0 = sg * S, k1 = min(k0 + S, Tn);
            // recompute x_k0 .. x_{k1-1} into sSeg
            T xi = 0, qj = 0, vj = 0;
            if (lin) {
                if (lane < n) xi = sChk[sg * n + lane];
            } else if (lane < d) {
                qj = sChk[sg * n + lane];
                vj = sChk[sg * n + d + lane];
            }
            for (int k = k0; k < k1; ++k) {
                if (lin) {
                    if (lane < n) sSeg[(k - k0) * n + lane] = xi;
                } else if (lane < d) {
                    sSeg[(k - k0) * n + lane] = qj;
                    sSeg[(k - k0) * n + d + lane] = vj;
                }
                if (k + 1 < k1) {
                    const T u = input_at(k);
                    if (lin) {
                        if (lane < m) sUin[lane] = u;
                        xi = lin_step(xi);
                    } else {
                        chain_step(qj, vj, u);
                    }
                }
            }
            __syncthreads();
            for (int k = k1 - 1; k >= k0; --k) {
                const Knot kn = knot_at(Tn, P.p, k);
                const T c = (T)kn.rem / (T)kn.den;
                const T u = input_at(k);
                T gu;
                if (lin) {
                    if (lane < n) sX[lane] = lam;
                    __syncthreads();
                    T bu = 0, ax = 0;
                    if (lane < m)
                        for (int i = 0; i < n; ++i) bu += sB[i * m + lane] * sX[i];
                    if (lane < n)
                        for (int i = 0; i < n; ++i) ax += sA[i * n + lane] * sX[i];
                    __syncthreads();
                    gu = (T)2 * L.r * (u - L.ug) + bu;
                    if (k >= 1 && lane < n) {
                        const T xk = sSeg[(k - k0) * n + lane];
                        lam = (T)2 * L.q * (xk - L.xg) + ax;
                    }
                } else {
                    const T qk = lane < d ? sSeg[(k - k0) * n + lane] : (T)0;
                    const T vk = lane < d ? sSeg[(k - k0) * n + d + lane] : (T)0;
                    const T phi = scan_up(qk);
                    const T Sv = scan_down(L.cg * cos_f<T>(phi));
                    const T mu = lv + P.dt * lq;
                    const T nu = mu * L.invI;
                    const T pf = scan_up(nu);
                    const T sn = Sv * nu;
                    const T R = scan_down(sn) - sn;
                    const T dadq = -L.kst * nu - (Sv * pf + R);
                    const T lq_n = lq + P.dt * dadq;
                    const T lv_n = mu - P.dt * L.dmp * nu;
                    gu = (T)2 * L.wr * (u - L.gu) + P.dt * nu;
                    if (k >= 1) {
                        lq = lq_n + (T)2 * L.wq * (qk - L.gq);
                        lv = lv_n + (T)2 * L.wv * (vk - L.gv);
                    }
                }
                if (lane < m) {
                    sG[kn.a * m + lane] += ((T)1 - c) * gu;
                    sG[kn.b * m + lane] += c * gu;
                }
            }
            __syncthreads();
        }
        __syncthreads();
    };

    T xi, qj, vj;
    if (!refine) {
        const T J = forward(true, xi, qj, vj);
        backward(xi, qj, vj);
        for (int j = lane; j < pm; j += 64) dJ[(int64_t)j * ld + cand] = sG[j];
        if (cost && lane == 0) cost[cand] = J;
        return;
    }
    // Adam (Kingma & Ba 2015), bias-corrected, clamp after each update
    const T b1 = (T)0.9, b2 = (T)0.999, eps = (T)1e-8;
    T b1t = 1, b2t = 1;
    for (int t = 1; t <= steps; ++t) {
        forward(true, xi, qj, vj);
        backward(xi, qj, vj);
        b1t *= b1;
        b2t *= b2;
        for (int j = lane; j < pm; j += 64) {
            const T g = sG[j];
            const T m1 = b1 * sM1[j] + ((T)1 - b1) * g;
            const T m2 = b2 * sM2[j] + ((T)1 - b2) * g * g;
            sM1[j] = m1;
            sM2[j] = m2;
            const T mh = m1 / ((T)1 - b1t), vh = m2 / ((T)1 - b2t);
            T U = sU[j] - lr * mh / (sqrt(vh) + eps);
            const int i = j % m;
            U = U < P.umin[i] ? P.umin[i] : U;
            U = U > P.umax[i] ? P.umax[i] : U;
            sU[j] = U;
        }
        __syncthreads();
    }
    const T Jn = forward(false, xi, qj, vj);
    if (Jn < cost_io[cand]) {  // uniform: Jn is a wave sum
        for (int j = lane; j < pm; j += 64) knots_io[(int64_t)j * ld + cand] = sU[j];
        if (lane == 0) cost_io[cand] = Jn;
    }
}

size_t grad_smem_bytes(int model, int n, int m, int T, int p, size_t esize) {
    return grad_plan(model, n, m, T, p).total * esize;
}

template <typename T>
hipError_t launch_grad(const ProbView<T> &P, int model, const T *x0, const T *knots, int64_t ncand,
                       int64_t ld, T *dJ, T *cost, int refine_steps, T lr, T *knots_io,
                       T *cost_io, hipStream_t s) {
    const GradPlan G = grad_plan(model, P.n, P.m, P.Tn, P.p);
    const size_t bytes = G.total * sizeof(T);
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)adjoint_kernel<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(adjoint_kernel<T>, dim3((unsigned)ncand), dim3(64), bytes, s, P, model, G,
                       x0, knots, ld, dJ, cost, refine_steps, lr, knots_io, cost_io);
    return hipGetLastError();
}
template hipError_t launch_grad<float>(const ProbView<float> &, int, const float *, const float *,
                                       int64_t, int64_t, float *, float *, int, float, float *,
                                       float *, hipStream_t);
template hipError_t launch_grad<double>(const ProbView<double> &, int, const double *,
                                        const double *, int64_t, int64_t, double *, double *, int,
                                        double, double *, double *, hipStream_t);

}  // namespace empc
