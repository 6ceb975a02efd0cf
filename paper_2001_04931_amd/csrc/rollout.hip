// Rollout + cost kernels (gfx950).
//
// Linear model (eq. 2): the population-batched step X <- A_d X + B_d U + w_d
// is a dense contraction with M = n states, K = n + m, N = candidates, so it
// runs on the matrix cores: v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64,
// one wavefront per tile of 16 candidates.
//
// The accumulator of a 16x16x4 MFMA leaves lane l holding, in register v
// (v = 0..3), row R(l/16, v) of column l%16, with R(g, v) = 4g + v for the
// f32 instruction and R(g, v) = g + 4v for the f64 one.  The B operand of the
// same instruction takes row l/16 of column l%16 from lane l.  So accumulator
// register v of M-tile t, used as a B operand as it stands, supplies the K
// slice made of state rows {16t + R(g, v) : g = 0..3}; permuting the columns
// of A_d to match that K order (the contraction order is free) chains the
// steps with no cross-lane data movement.  A_d, B_d live in registers as A
// operands (one value per lane per MFMA), the state lives in accumulators,
// and knot interpolation, the dynamics step and the cost are fused in one
// loop over the horizon.
//
// Pendulum chain: one candidate per lane, joint state in registers, the
// per-joint constants (gravity coefficients, inverse inertia, weights) in LDS
// where every lane reads the same address (broadcast).
#include <math.h>

#include "internal.hpp"

namespace empc {

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator row of lane group g, register v
    __device__ static constexpr int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int g, int v) { return g + 4 * v; }
};

// NT = ceil(n / 16) M-tiles, NU = ceil(m / 4) input K-slices.
template <typename T, int NT, int NU, int WPB>
__global__ __launch_bounds__(64 * WPB) void roll_linear_mfma(ProbView<T> P,
                                                             const T *__restrict__ x0,
                                                             const T *__restrict__ knots,
                                                             int64_t ld, int64_t ncand,
                                                             T *__restrict__ cost) {
    typedef typename Mfma<T>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    const int64_t cand0 = tile * 16;
    if (cand0 >= ncand) return;  // wave-uniform
    const int col = lane & 15, grp = lane >> 4;
    const int64_t cand = cand0 + col;
    const bool valid = cand < ncand;
    const int n = P.n, m = P.m;

    // A operands.  aX[mt][4t+v]: A_d[16mt + col][16t + R(grp, v)].
    T aX[NT][4 * NT];
    T aU[NT][NU];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
        const int row = 16 * mt + col;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk = 16 * t + Mfma<T>::row(grp, v);
                aX[mt][4 * t + v] = (row < n && kk < n) ? P.Ad[row * n + kk] : (T)0;
            }
#pragma unroll
        for (int s = 0; s < NU; ++s) {
            const int j = 4 * s + grp;
            aU[mt][s] = (row < n && j < m) ? P.Bd[row * m + j] : (T)0;
        }
    }
    // State and per-row constants in accumulator layout: row 16mt + R(grp, v).
    v4 X[NT], Wd[NT], Qw[NT], Xg[NT], Qf[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + Mfma<T>::row(grp, v);
            const bool in = row < n;
            X[mt][v] = in ? x0[row] : (T)0;
            Wd[mt][v] = (in && P.wd) ? P.wd[row] : (T)0;
            Qw[mt][v] = in ? P.q[row] : (T)0;
            Xg[mt][v] = (in && P.xg) ? P.xg[row] : (T)0;
            Qf[mt][v] = (in && P.qf) ? P.qf[row] : (T)0;
        }
    T Rw[NU], Ug[NU];
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        const int j = 4 * s + grp;
        Rw[s] = j < m ? P.r[j] : (T)0;
        Ug[s] = (j < m && P.ug) ? P.ug[j] : (T)0;
    }

    T J = 0;
    int cur_a = -1;
    T ua[NU], ub[NU];
    for (int k = 0; k < P.Tn; ++k) {
        const Knot kn = knot_at(P.Tn, P.p, k);
        if (kn.a != cur_a) {  // wave-uniform: knots change p-1 times
            cur_a = kn.a;
#pragma unroll
            for (int s = 0; s < NU; ++s) {
                const int j = 4 * s + grp;
                const bool ok = valid && j < m;
                ua[s] = ok ? knots[(int64_t)(kn.a * m + j) * ld + cand] : (T)0;
                ub[s] = ok ? knots[(int64_t)(kn.b * m + j) * ld + cand] : (T)0;
            }
        }
        const T c = (T)kn.rem / (T)kn.den;
        T u[NU];
#pragma unroll
        for (int s = 0; s < NU; ++s) u[s] = ((T)1 - c) * ua[s] + c * ub[s];

        v4 acc[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) acc[mt] = Wd[mt];
        // input part first: it does not depend on the previous step
#pragma unroll
        for (int s = 0; s < NU; ++s)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) acc[mt] = Mfma<T>::op(aU[mt][s], u[s], acc[mt]);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int mt = 0; mt < NT; ++mt)
                    acc[mt] = Mfma<T>::op(aX[mt][4 * t + v], X[t][v], acc[mt]);
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) X[mt] = acc[mt];

        T js = 0;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T e = Xg[mt][v] - X[mt][v];
                js += Qw[mt][v] * e * e;
            }
#pragma unroll
        for (int s = 0; s < NU; ++s) {
            const T e = Ug[s] - u[s];
            js += Rw[s] * e * e;
        }
        J += js;
    }
    T jt = 0;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const T e = Xg[mt][v] - X[mt][v];
            jt += Qf[mt][v] * e * e;
        }
    J += jt;
    J += __shfl_xor(J, 16, 64);
    J += __shfl_xor(J, 32, 64);
    if (grp == 0 && valid) cost[cand] = J;
}

// ---------------------------------------------------------------------------
// Pendulum chain.  Per-joint constants in LDS.
template <typename T>
struct JointConst {
    T cg;    // g l_r M_r (gravity coefficient of absolute angle r)
    T invI;  // 1 / I_j
    T kst, dmp;
    T wq, wv, wqf, wvf;  // stage and terminal weights of q_j and qd_j
    T gq, gv;            // goals of q_j and qd_j
    T wr, gu;            // input weight and goal
};

template <typename T>
__device__ void chain_constants_lds(const ProbView<T> &P, JointConst<T> *jc) {
    const int d = P.m;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        T tail = 0;
        for (int i = j; i < d; ++i) tail += P.mass[i];
        T inert = 0, dist = 0;
        for (int i = j; i < d; ++i) {
            dist += P.len[i];
            inert += P.mass[i] * dist * dist;
        }
        JointConst<T> c;
        c.cg = P.gravity * P.len[j] * tail;
        c.invI = (T)1 / inert;
        c.kst = P.stiff[j];
        c.dmp = P.damp[j];
        c.wq = P.q[j];
        c.wv = P.q[d + j];
        c.wqf = P.qf ? P.qf[j] : (T)0;
        c.wvf = P.qf ? P.qf[d + j] : (T)0;
        c.gq = P.xg ? P.xg[j] : (T)0;
        c.gv = P.xg ? P.xg[d + j] : (T)0;
        c.wr = P.r[j];
        c.gu = P.ug ? P.ug[j] : (T)0;
        jc[j] = c;
    }
}

template <typename T>
__device__ inline T sin_of(T x);
template <>
__device__ inline float sin_of<float>(float x) { return sinf(x); }
template <>
__device__ inline double sin_of<double>(double x) { return sin(x); }

template <typename T, int DMAX>
__global__ __launch_bounds__(256) void roll_chain(ProbView<T> P, const T *__restrict__ x0,
                                                  const T *__restrict__ knots, int64_t ld,
                                                  int64_t ncand, T *__restrict__ cost) {
    __shared__ JointConst<T> jc[DMAX];
    chain_constants_lds(P, jc);
    __syncthreads();
    const int64_t cand = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cand >= ncand) return;
    const int d = P.m;
    const T dt = P.dt;
    T q[DMAX], v[DMAX], ua[DMAX], ub[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        q[j] = j < d ? x0[j] : (T)0;
        v[j] = j < d ? x0[d + j] : (T)0;
    }
    T J = 0;
    int cur_a = -1;
    for (int k = 0; k < P.Tn; ++k) {
        // re-read the per-joint constants from LDS every step instead of
        // letting them be hoisted into (and overflow) registers
        asm volatile("" ::: "memory");
        const Knot kn = knot_at(P.Tn, P.p, k);
        if (kn.a != cur_a) {
            cur_a = kn.a;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                ua[j] = j < d ? knots[(int64_t)(kn.a * d + j) * ld + cand] : (T)0;
                ub[j] = j < d ? knots[(int64_t)(kn.b * d + j) * ld + cand] : (T)0;
            }
        }
        const T c = (T)kn.rem / (T)kn.den;
        // gravity torque: G_j = sum_{r>=j} cg_r sin(phi_r), phi_r = q_0 + .. + q_r
        T sg[DMAX];
        T phi = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (j < d) {
                phi += q[j];
                sg[j] = jc[j].cg * sin_of<T>(phi);
            }
        }
        T G = 0, js = 0;
#pragma unroll
        for (int j = DMAX - 1; j >= 0; --j) {
            if (j < d) {
                const JointConst<T> cj = jc[j];
                G += sg[j];
                const T u = ((T)1 - c) * ua[j] + c * ub[j];
                const T acc = (u - cj.kst * q[j] - cj.dmp * v[j] - G) * cj.invI;
                v[j] = v[j] + dt * acc;
                q[j] = q[j] + dt * v[j];
                const T eq = cj.gq - q[j], ev = cj.gv - v[j], eu = cj.gu - u;
                js += cj.wq * eq * eq + cj.wv * ev * ev + cj.wr * eu * eu;
            }
        }
        J += js;
    }
    T jt = 0;
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        if (j < d) {
            const T eq = jc[j].gq - q[j], ev = jc[j].gv - v[j];
            jt += jc[j].wqf * eq * eq + jc[j].wvf * ev * ev;
        }
    }
    cost[cand] = J + jt;
}

// ---------------------------------------------------------------------------
// Dispatch.
template <typename T, int NT, int NU>
static hipError_t go_linear(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                            int64_t ld, T *cost, hipStream_t s) {
    constexpr int WPB = 4;
    const int64_t tiles = (ncand + 15) / 16;
    const int64_t blocks = (tiles + WPB - 1) / WPB;
    hipLaunchKernelGGL((roll_linear_mfma<T, NT, NU, WPB>), dim3((unsigned)blocks), dim3(64 * WPB),
                       0, s, P, x0, knots, ld, ncand, cost);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t go_linear_nu(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                               int64_t ld, T *cost, hipStream_t s) {
    const int nu = (P.m + 3) / 4;
    if (nu <= 1) return go_linear<T, NT, 1>(P, x0, knots, ncand, ld, cost, s);
    if (nu <= 2) return go_linear<T, NT, 2>(P, x0, knots, ncand, ld, cost, s);
    if (nu <= 4) return go_linear<T, NT, 4>(P, x0, knots, ncand, ld, cost, s);
    if (nu <= 6) return go_linear<T, NT, 6>(P, x0, knots, ncand, ld, cost, s);
    if (nu <= 8) return go_linear<T, NT, 8>(P, x0, knots, ncand, ld, cost, s);
    return go_linear<T, NT, 10>(P, x0, knots, ncand, ld, cost, s);
}

template <typename T, int DMAX>
static hipError_t go_chain(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                           int64_t ld, T *cost, hipStream_t s) {
    const int64_t blocks = (ncand + 255) / 256;
    hipLaunchKernelGGL((roll_chain<T, DMAX>), dim3((unsigned)blocks), dim3(256), 0, s, P, x0,
                       knots, ld, ncand, cost);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rollout(const ProbView<T> &P, int model, const T *x0, const T *knots,
                          int64_t ncand, int64_t ld, T *cost, hipStream_t s) {
    if (ncand <= 0) return hipSuccess;
    if (model == EMPC_LINEAR) {
        const int nt = (P.n + 15) / 16;
        switch (nt) {
            case 1: return go_linear_nu<T, 1>(P, x0, knots, ncand, ld, cost, s);
            case 2: return go_linear_nu<T, 2>(P, x0, knots, ncand, ld, cost, s);
            case 3: return go_linear_nu<T, 3>(P, x0, knots, ncand, ld, cost, s);
            case 4: return go_linear_nu<T, 4>(P, x0, knots, ncand, ld, cost, s);
            default: return go_linear_nu<T, 5>(P, x0, knots, ncand, ld, cost, s);
        }
    }
    const int d = P.m;
    if (d <= 4) return go_chain<T, 4>(P, x0, knots, ncand, ld, cost, s);
    if (d <= 8) return go_chain<T, 8>(P, x0, knots, ncand, ld, cost, s);
    if (d <= 16) return go_chain<T, 16>(P, x0, knots, ncand, ld, cost, s);
    if (d <= 24) return go_chain<T, 24>(P, x0, knots, ncand, ld, cost, s);
    return go_chain<T, 40>(P, x0, knots, ncand, ld, cost, s);
}

template hipError_t launch_rollout<float>(const ProbView<float> &, int, const float *,
                                          const float *, int64_t, int64_t, float *, hipStream_t);
template hipError_t launch_rollout<double>(const ProbView<double> &, int, const double *,
                                           const double *, int64_t, int64_t, double *,
                                           hipStream_t);

// ---------------------------------------------------------------------------
// Plant: one model step of a single state vector (closed-loop simulation).
template <typename T>
__global__ void plant_kernel(ProbView<T> P, int model, const T *__restrict__ x,
                             const T *__restrict__ u, const T *__restrict__ noise,
                             T *__restrict__ x_next) {
    // one block of 64 threads; thread i computes row / joint i serially
    __shared__ T xs[2 * Limits::MAX_N_LINEAR];
    const int n = P.n, m = P.m;
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = x[i];
    __syncthreads();
    if (model == EMPC_LINEAR) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            T s = P.wd ? P.wd[i] : (T)0;
            for (int j = 0; j < n; ++j) s += P.Ad[i * n + j] * xs[j];
            for (int j = 0; j < m; ++j) s += P.Bd[i * m + j] * u[j];
            x_next[i] = s + (noise ? noise[i] : (T)0);
        }
        return;
    }
    const int d = m;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        T G = 0;
        for (int r = j; r < d; ++r) {
            T phi = 0, tail = 0;
            for (int s = 0; s <= r; ++s) phi += xs[s];
            for (int i = r; i < d; ++i) tail += P.mass[i];
            G += P.gravity * P.len[r] * tail * sin_of<T>(phi);
        }
        T inert = 0, dist = 0;
        for (int i = j; i < d; ++i) {
            dist += P.len[i];
            inert += P.mass[i] * dist * dist;
        }
        const T acc = (u[j] - P.stiff[j] * xs[j] - P.damp[j] * xs[d + j] - G) / inert;
        const T vn = xs[d + j] + P.dt * acc;
        x_next[d + j] = vn + (noise ? noise[d + j] : (T)0);
        x_next[j] = xs[j] + P.dt * vn + (noise ? noise[j] : (T)0);
    }
}

template <typename T>
hipError_t launch_plant(const ProbView<T> &P, int model, const T *x, const T *u, const T *noise,
                        T *x_next, hipStream_t s) {
    hipLaunchKernelGGL(plant_kernel<T>, dim3(1), dim3(64), 0, s, P, model, x, u, noise, x_next);
    return hipGetLastError();
}
template hipError_t launch_plant<float>(const ProbView<float> &, int, const float *,
                                        const float *, const float *, float *, hipStream_t);
template hipError_t launch_plant<double>(const ProbView<double> &, int, const double *,
                                         const double *, const double *, double *, hipStream_t);

}  // namespace empc
