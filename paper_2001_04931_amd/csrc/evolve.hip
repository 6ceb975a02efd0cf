// Single-problem evolutionary step launchers: next population and parent
// selection (bodies in evolve_body.hpp).
#include "evolve_body.hpp"

namespace empc {

template <typename T>
hipError_t launch_population(const ProbView<T> &P, const empc_ga &ga, const T *knots_in,
                             int64_t ld_in, const int64_t *elite_idx, const T *elite_rows,
                             const int *has_elites, int cold_mode, T *knots_out, int64_t ld_out,
                             uint32_t tick, uint32_t gen, hipStream_t s,
                             const PopVariant<T> &var, int R_override) {
    const int pm = P.p * P.m;
    const GaStreams gs = ga_streams(ga.seed, P.m, pm);
    // parameter groups per thread: a workgroup's draws shared by its
    // children (parents, mutation flags, crossover bits) are taken once per
    // workgroup, so large populations take 32 or 64 parameters per
    // workgroup instead of 16, as long as thousands of workgroups remain
    const int64_t wgs1 = pop_tiles_s(ga.pop) * pop_tiles_g(pm);
    const int R = (R_override == 1 || R_override == 2 || R_override == 4)
                      ? R_override
                      : (wgs1 >= 4096 ? 4 : wgs1 >= 2048 ? 2 : 1);
    const int64_t blocks = pop_tiles_s(ga.pop) * pop_tiles_g(pm, R);
    hipLaunchKernelGGL(population_kernel<T>, dim3((unsigned)blocks), dim3(POP_THREADS), 0, s, P, gs,
                       (int64_t)ga.pop, ga.n_elite, ga.elitism, (T)ga.sigma, knots_in, ld_in,
                       elite_idx, elite_rows, has_elites, cold_mode, knots_out, ld_out, tick, gen,
                       var, R);
    return hipGetLastError();
}
template hipError_t launch_population<float>(const ProbView<float> &, const empc_ga &,
                                             const float *, int64_t, const int64_t *,
                                             const float *, const int *, int, float *, int64_t,
                                             uint32_t, uint32_t, hipStream_t,
                                             const PopVariant<float> &, int);
template hipError_t launch_population<double>(const ProbView<double> &, const empc_ga &,
                                              const double *, int64_t, const int64_t *,
                                              const double *, const int *, int, double *,
                                              int64_t, uint32_t, uint32_t, hipStream_t,
                                              const PopVariant<double> &, int);

template <typename T>
hipError_t launch_select(const ProbView<T> &P, const T *cost, const T *knots, int64_t ld,
                         int64_t pop, int k, int64_t *elite_idx, int64_t *best_idx, T *elite_rows,
                         T *elite_cost, int *has_elites, int *best_slot, T *u_star, T *best_cost,
                         hipStream_t s) {
    typedef typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type K;
    auto go = [&](auto kernel, int nthr) {
        hipLaunchKernelGGL(kernel, dim3(1), dim3(nthr), 0, s, cost, pop, k, knots, ld, P.p * P.m,
                           P.m, elite_idx, best_idx, elite_rows, elite_cost, has_elites, best_slot,
                           u_star, best_cost);
    };
    // one wavefront's bitonic sort up to 256 candidates; 256 threads up to
    // 1024 candidates, else 1024 threads (measured at 4096: 7.1 against
    // 9.2 us; at 16384: 11.6 against 21.4 us)
    if (pop <= 256) {
        go(select_small_kernel<T, K>, 64);
    } else if (pop <= 1024) {
        go(select_kernel<T, K, 4, 256>, 256);
    } else {
        const int64_t per = (pop + 1023) / 1024;
        if (per <= 4)
            go(select_kernel<T, K, 4, 1024>, 1024);
        else if (per <= 16)
            go(select_kernel<T, K, 16, 1024>, 1024);
        else if (per <= 64)
            go(select_kernel<T, K, 64, 1024>, 1024);
        else
            go(select_kernel<T, K, 0, 1024>, 1024);
    }
    return hipGetLastError();
}
template hipError_t launch_select<float>(const ProbView<float> &, const float *, const float *,
                                         int64_t, int64_t, int, int64_t *, int64_t *, float *,
                                         float *, int *, int *, float *, float *, hipStream_t);
template hipError_t launch_select<double>(const ProbView<double> &, const double *,
                                          const double *, int64_t, int64_t, int, int64_t *,
                                          int64_t *, double *, double *, int *, int *, double *,
                                          double *, hipStream_t);

// ---------------------------------------------------------------------------
// Gradient-refined solves: the parents of a generation, gathered into a
// structure-of-arrays block [pm][k], are refined by Adam (adjoint.hip), then
// copied to the parent buffer (the same [pm][k] layout) for the next
// population, and the best refined parent gives u* and the best cost.
template <typename T>
__global__ __launch_bounds__(256) void gather_parents_kernel(const T *__restrict__ knots,
                                                             int64_t ld,
                                                             const int64_t *__restrict__ elite_idx,
                                                             int k, int pm, T *__restrict__ E) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)k * pm) return;
    const int j = (int)(t / k), s = (int)(t % k);
    E[t] = knots[(int64_t)j * ld + elite_idx[s]];
}

template <typename T>
__global__ __launch_bounds__(256) void finish_refine_kernel(const T *__restrict__ E, int k, int pm,
                                                            int m, const T *__restrict__ ecost,
                                                            T *__restrict__ elite_rows,
                                                            int *__restrict__ best_slot_out,
                                                            T *__restrict__ u_star,
                                                            T *__restrict__ best_cost) {
    typedef typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type K;
    __shared__ int s_best;
    const int tid = threadIdx.x;
    for (int t = tid; t < k * pm; t += blockDim.x) elite_rows[t] = E[t];  // same layout
    if (tid < 64) {
        K bk = ~(K)0;
        int bs = k;
        for (int s = tid; s < k; s += 64) {
            const K key = sort_key(ecost[s]);
            if (key < bk || (key == bk && s < bs)) {
                bk = key;
                bs = s;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const K ok = __shfl_xor(bk, o, 64);
            const int os = __shfl_xor(bs, o, 64);
            if (ok < bk || (ok == bk && os < bs)) {
                bk = ok;
                bs = os;
            }
        }
        if (tid == 0) s_best = bs < k ? bs : 0;
    }
    __syncthreads();
    const int b = s_best;
    if (tid == 0) {
        if (best_slot_out) *best_slot_out = b;
        if (best_cost) *best_cost = ecost[b];
    }
    if (u_star)
        for (int i = tid; i < m; i += blockDim.x) u_star[i] = E[(int64_t)i * k + b];
}

template <typename T>
hipError_t launch_gather_parents(const T *knots, int64_t ld, const int64_t *elite_idx, int k,
                                 int pm, T *E, hipStream_t s) {
    const int64_t total = (int64_t)k * pm;
    hipLaunchKernelGGL(gather_parents_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       s, knots, ld, elite_idx, k, pm, E);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_finish_refine(const T *E, int k, int pm, int m, const T *ecost, T *elite_rows,
                                int *best_slot, T *u_star, T *best_cost, hipStream_t s) {
    hipLaunchKernelGGL(finish_refine_kernel<T>, dim3(1), dim3(256), 0, s, E, k, pm, m, ecost,
                       elite_rows, best_slot, u_star, best_cost);
    return hipGetLastError();
}
template hipError_t launch_gather_parents<float>(const float *, int64_t, const int64_t *, int, int,
                                                 float *, hipStream_t);
template hipError_t launch_gather_parents<double>(const double *, int64_t, const int64_t *, int,
                                                  int, double *, hipStream_t);
template hipError_t launch_finish_refine<float>(const float *, int, int, int, const float *,
                                                float *, int *, float *, float *, hipStream_t);
template hipError_t launch_finish_refine<double>(const double *, int, int, int, const double *,
                                                 double *, int *, double *, double *, hipStream_t);

}  // namespace empc
