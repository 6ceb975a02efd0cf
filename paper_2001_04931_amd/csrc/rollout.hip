// Pendulum-chain rollout + cost and the plant step (gfx950).  The linear
// model's rollout lives in rollout_linear.hpp.
//
// Pendulum chain: one candidate per lane, joint state in registers, the
// per-joint constants (gravity coefficients, inverse inertia, weights) in LDS
// where every lane reads the same address (broadcast).
#include <hip/hip_ext.h>
#include <math.h>

#include "rollout_chain.hpp"

namespace empc {

// Launch through hipExtLaunchKernelGGL when timing events are given: the
// events are stamped by the kernel's own dispatch, with no extra stream
// packets around it.
template <typename K, typename... Args>
static hipError_t launch_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                               const Events &ev, Args... args) {
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return hipGetLastError();
}

template <typename T, int DMAX, int FEAT>
static hipError_t go_chain(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                           int64_t ld, T *cost, hipStream_t s, const Events &ev, int threads) {
    const int64_t blocks = (ncand + threads - 1) / threads;
    return launch_timed(roll_chain<T, DMAX, FEAT>, dim3((unsigned)blocks), dim3(threads), 0, s, ev,
                        P, x0, knots, ld, ncand, cost);
}

// workgroup size of a chain form (RF_RULE: 256)
static int chain_threads(int form) {
    return form == RF_CH64 ? 64 : (form == RF_CH128 ? 128 : 256);
}

template <typename T, int FEAT>
static hipError_t go_chain_forms(const ProbView<T> &P, const T *x0, const T *knots,
                                 int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                 const Events &ev, int form) {
    const int d = P.m, threads = chain_threads(form);
    if (d <= 4) return go_chain<T, 4, FEAT>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    if (d <= 8) return go_chain<T, 8, FEAT>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    // one candidate per 16-lane row for larger chains (threads / 16 per
    // workgroup)
    const dim3 rows((unsigned)((ncand + threads / 16 - 1) / (threads / 16))), blk(threads);
    if (d <= 16)
        return launch_timed(roll_chain_rows<T, 1, FEAT>, rows, blk, 0, s, ev, P, x0, knots, ld,
                            ncand, cost);
    if (d <= 32)
        return launch_timed(roll_chain_rows<T, 2, FEAT>, rows, blk, 0, s, ev, P, x0, knots, ld,
                            ncand, cost);
    return launch_timed(roll_chain_rows<T, 3, FEAT>, rows, blk, 0, s, ev, P, x0, knots, ld, ncand,
                        cost);  // d <= 48
}

template <typename T>
hipError_t launch_rollout(const ProbView<T> &P, int model, const T *x0, const T *knots,
                          int64_t ncand, int64_t ld, T *cost, hipStream_t s, const Events &ev,
                          int form) {
    if (ncand <= 0) return hipSuccess;
    if (model == EMPC_LINEAR)
        return launch_linear<T>(P, x0, knots, ncand, ld, cost, s, ev, form >= RF_CH64 ? RF_RULE : form);
    const int cf = form >= RF_CH64 ? form : RF_RULE;
    const int feat = (P.qb ? CF_BOX : 0) | (P.qhi ? CF_LIMIT : 0) | (P.fc ? CF_FRIC : 0);
    switch (feat) {
        case 1: return go_chain_forms<T, 1>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 2: return go_chain_forms<T, 2>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 3: return go_chain_forms<T, 3>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 4: return go_chain_forms<T, 4>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 5: return go_chain_forms<T, 5>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 6: return go_chain_forms<T, 6>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        case 7: return go_chain_forms<T, 7>(P, x0, knots, ncand, ld, cost, s, ev, cf);
        default: return go_chain_forms<T, 0>(P, x0, knots, ncand, ld, cost, s, ev, cf);
    }
}

template hipError_t launch_rollout<float>(const ProbView<float> &, int, const float *,
                                          const float *, int64_t, int64_t, float *, hipStream_t,
                                          const Events &, int);
template hipError_t launch_rollout<double>(const ProbView<double> &, int, const double *,
                                           const double *, int64_t, int64_t, double *,
                                           hipStream_t, const Events &, int);

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
    // gravity term of each absolute angle, g l_r (sum_{i>=r} m_i) sin(phi_r),
    // phi_r = q_0 + .. + q_r; one thread walks the chain once
    __shared__ T sg[Limits::MAX_D_CHAIN];
    if (threadIdx.x == 0) {
        T phi = 0;
        for (int r = 0; r < d; ++r) {
            phi += xs[r];
            sg[r] = phi;
        }
        T tail = 0;
        for (int r = d - 1; r >= 0; --r) {
            tail += P.mass[r];
            sg[r] = P.gravity * P.len[r] * tail * sin_of<T>(sg[r]);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        T G = 0;  // gravity torque on joint j: sum over r >= j
        for (int r = d - 1; r >= j; --r) G += sg[r];
        T inert = 0, dist = 0;
        for (int i = j; i < d; ++i) {
            dist += P.len[i];
            inert += P.mass[i] * dist * dist;
        }
        const T f = u[j] - P.stiff[j] * xs[j] - P.damp[j] * xs[d + j] - G;
        T vn = xs[d + j] + P.dt * (f / inert);
        if (P.fc) vn = dry_friction(xs[d + j], vn, f, P.dt / inert, P.fc[j], P.fs[j]);
        T qn = xs[j] + P.dt * vn;
        if (P.qhi) joint_limit(qn, vn, P.qlo[j], P.qhi[j], P.rest);
        x_next[d + j] = vn + (noise ? noise[d + j] : (T)0);
        x_next[j] = qn + (noise ? noise[j] : (T)0);
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
