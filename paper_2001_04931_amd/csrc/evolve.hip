// Evolutionary step kernels (gfx950): next population and parent selection
// (Sec. V, Alg. 1 warm/cold start; parent selection of the numParents lowest
// costs).
#include <math.h>

#include "internal.hpp"

namespace empc {

template <typename T>
__device__ inline void sincos_of(T x, T *s, T *c);
template <>
__device__ inline void sincos_of<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <>
__device__ inline void sincos_of<double>(double x, double *s, double *c) { sincos(x, s, c); }
template <typename T>
__device__ inline T log_of(T x);
template <>
__device__ inline float log_of<float>(float x) { return logf(x); }
template <>
__device__ inline double log_of<double>(double x) { return log(x); }

// One thread per (parameter j, slot s), slot fastest so that writes of
// knots_out[j * ld + s] coalesce.
// Parent knots come from elite_rows ([k][pm], when non-NULL) or from
// knots_in at elite_idx[.].
// cold_mode: 0 warm, 1 cold, 2 cold iff *has_elites == 0.
template <typename T>
__global__ __launch_bounds__(256) void population_kernel(
    ProbView<T> P, GaStreams gs, int64_t pop, int k, int elitism, T sigma,
    const T *__restrict__ knots_in, int64_t ld_in, const int64_t *__restrict__ elite_idx,
    const T *__restrict__ elite_rows, const int *__restrict__ has_elites, int cold_mode,
    T *__restrict__ knots_out, int64_t ld_out, uint32_t tick, uint32_t gen) {
    const int m = P.m, pm = P.p * P.m;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pop * pm) return;
    const int64_t s = t % pop;
    const int j = (int)(t / pop);
    const int i = j % m;
    const bool cold = cold_mode == 1 || (cold_mode == 2 && *has_elites == 0);
    const uint32_t slot = (uint32_t)s;
    T val;
    if (cold) {
        const U4 w = ga_draw(gs, slot, gen, tick, 1, (uint32_t)(j / 4));
        val = P.umin[i] + (P.umax[i] - P.umin[i]) * uni23<T>(word_of(w, j % 4));
    } else if (elitism && s < k) {
        val = elite_rows ? elite_rows[s * pm + j] : knots_in[(int64_t)j * ld_in + elite_idx[s]];
    } else {
        const U4 w0 = ga_draw(gs, slot, gen, tick, 0, 0);
        const int p1 = (int)__umulhi(w0.x, (uint32_t)k);
        const int p2 = (int)__umulhi(w0.y, (uint32_t)k);
        const U4 wx = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.XB + j / 128));
        const int jb = j % 128;
        const bool from2 = (word_of(wx, jb / 32) >> (jb % 32)) & 1u;
        const int par = from2 ? p2 : p1;
        val = elite_rows ? elite_rows[(int64_t)par * pm + j]
                         : knots_in[(int64_t)j * ld_in + elite_idx[par]];
        const U4 wf = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(1 + i / 128));
        const int ib = i % 128;
        if ((word_of(wf, ib / 32) >> (ib % 32)) & 1u) {
            const U4 wn = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.NB + j / 4));
            const int pair = (j % 4) / 2;
            const T u1 = uni23<T>(word_of(wn, 2 * pair));
            const T u2 = uni23<T>(word_of(wn, 2 * pair + 1));
            const T rad = sqrt((T)-2 * log_of<T>(u1));
            T sn, cs;
            sincos_of<T>((T)6.283185307179586 * u2, &sn, &cs);
            val += sigma * rad * ((j & 1) ? sn : cs);
        }
        val = val < P.umin[i] ? P.umin[i] : val;
        val = val > P.umax[i] ? P.umax[i] : val;
    }
    knots_out[(int64_t)j * ld_out + s] = val;
}

template <typename T>
hipError_t launch_population(const ProbView<T> &P, const empc_ga &ga, const T *knots_in,
                             int64_t ld_in, const int64_t *elite_idx, const T *elite_rows,
                             const int *has_elites, int cold_mode, T *knots_out, int64_t ld_out,
                             uint32_t tick, uint32_t gen, hipStream_t s) {
    const int pm = P.p * P.m;
    const GaStreams gs = ga_streams(ga.seed, P.m, pm);
    const int64_t total = (int64_t)ga.pop * pm;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(population_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, P, gs,
                       (int64_t)ga.pop, ga.n_elite, ga.elitism, (T)ga.sigma, knots_in, ld_in,
                       elite_idx, elite_rows, has_elites, cold_mode, knots_out, ld_out, tick, gen);
    return hipGetLastError();
}
template hipError_t launch_population<float>(const ProbView<float> &, const empc_ga &,
                                             const float *, int64_t, const int64_t *,
                                             const float *, const int *, int, float *, int64_t,
                                             uint32_t, uint32_t, hipStream_t);
template hipError_t launch_population<double>(const ProbView<double> &, const empc_ga &,
                                              const double *, int64_t, const int64_t *,
                                              const double *, const int *, int, double *,
                                              int64_t, uint32_t, uint32_t, hipStream_t);

// ---------------------------------------------------------------------------
// Selection: one workgroup of 1024 threads (16 wavefronts).
//  1. radix select of the k-th smallest sortable cost key, 8 bits per pass;
//  2. one ordered pass in chunks of 1024 indices: keys below the threshold
//     are taken, keys equal to it are taken by ascending index until k are
//     taken; block prefix sums give each taken index its position, so the
//     elite list comes out in ascending index order;
//  3. best = lowest (key, index) among the elites; copy the elite knot rows,
//     costs, u* = knot 0 of the best, the best cost and the warm-start flag.
constexpr int SEL_THREADS = 1024;
constexpr int SEL_WAVES = SEL_THREADS / 64;

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Exclusive block prefix sum of v over the 1024 threads; *total gets the sum.
__device__ inline int block_excl_scan(int v, int *wsum, int *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int incl = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SEL_WAVES; ++w) {
        const int x = wsum[w];
        base += w < wave ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

template <typename T, typename K>
__global__ __launch_bounds__(SEL_THREADS) void select_kernel(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    __shared__ int hist[256];
    __shared__ int wsum[SEL_WAVES];
    __shared__ int s_digit, s_rem;
    __shared__ int64_t s_elite[Limits::MAX_ELITE];
    __shared__ int s_best_slot;
    const int tid = threadIdx.x;
    for (int s = tid; s < k; s += SEL_THREADS) s_elite[s] = 0;

    K prefix = 0, mask = 0;
    int remaining = k;
    for (int shift = (int)sizeof(K) * 8 - 8; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += SEL_THREADS) hist[b] = 0;
        __syncthreads();
        for (int64_t i = tid; i < pop; i += SEL_THREADS) {
            const K key = sort_key(cost[i]);
            if ((key & mask) == prefix) atomicAdd(&hist[(int)((key >> shift) & 255)], 1);
        }
        __syncthreads();
        if (tid < 64) {
            // lane owns bins 4*lane .. 4*lane+3
            const int h0 = hist[4 * tid], h1 = hist[4 * tid + 1], h2 = hist[4 * tid + 2],
                      h3 = hist[4 * tid + 3];
            const int own = h0 + h1 + h2 + h3;
            const int incl = wave_incl_scan(own);
            const int excl = incl - own;
            const unsigned long long hit = __ballot(incl >= remaining);
            const int first = __ffsll((long long)hit) - 1;
            if (tid == first) {
                int cum = excl, dsel = 4 * tid;
                const int hs[4] = {h0, h1, h2, h3};
                for (int q = 0; q < 4; ++q) {
                    if (cum + hs[q] >= remaining) {
                        dsel = 4 * tid + q;
                        break;
                    }
                    cum += hs[q];
                }
                s_digit = dsel;
                s_rem = remaining - cum;
            }
        }
        __syncthreads();
        prefix |= (K)s_digit << shift;
        mask |= (K)255 << shift;
        remaining = s_rem;
        __syncthreads();
    }
    const K thr = prefix;
    // ordered pass
    int eq_base = 0, sel_base = 0;
    for (int64_t c0 = 0; c0 < pop; c0 += SEL_THREADS) {
        const int64_t i = c0 + tid;
        K key = ~(K)0;
        bool in = i < pop;
        if (in) key = sort_key(cost[i]);
        const int is_eq = (in && key == thr) ? 1 : 0;
        int eq_tot;
        const int eq_rank = block_excl_scan(is_eq, wsum, &eq_tot) + eq_base;
        const int sel = (in && (key < thr || (is_eq && eq_rank < remaining))) ? 1 : 0;
        int sel_tot;
        const int pos = block_excl_scan(sel, wsum, &sel_tot) + sel_base;
        if (sel && pos < k) s_elite[pos] = i;
        eq_base += eq_tot;
        sel_base += sel_tot;
    }
    __syncthreads();
    // best among the elites (wave 0)
    if (tid < 64) {
        K bk = ~(K)0;
        int bs = k;
        for (int s = tid; s < k; s += 64) {
            const K key = sort_key(cost[s_elite[s]]);
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
        if (tid == 0) s_best_slot = bs;
    }
    __syncthreads();
    const int bslot = s_best_slot;
    for (int s = tid; s < k; s += SEL_THREADS) {
        if (elite_idx_out) elite_idx_out[s] = s_elite[s];
        if (elite_cost) elite_cost[s] = cost[s_elite[s]];
    }
    if (elite_rows)
        for (int t = tid; t < k * pm; t += SEL_THREADS) {
            const int s = t / pm, j = t - s * pm;
            elite_rows[t] = knots[(int64_t)j * ld + s_elite[s]];
        }
    if (tid == 0) {
        if (best_idx_out) *best_idx_out = s_elite[bslot];
        if (has_elites) *has_elites = 1;
        if (best_slot_out) *best_slot_out = bslot;
        if (best_cost) *best_cost = cost[s_elite[bslot]];
    }
    // u*(i) = get_u_from_U(U_best(i), t = 0): knot 0 (idx1 = 0, c = 0)
    if (u_star)
        for (int i = tid; i < m; i += SEL_THREADS) u_star[i] = knots[(int64_t)i * ld + s_elite[bslot]];
}

template <typename T>
hipError_t launch_select(const ProbView<T> &P, const T *cost, const T *knots, int64_t ld,
                         int64_t pop, int k, int64_t *elite_idx, int64_t *best_idx, T *elite_rows,
                         T *elite_cost, int *has_elites, int *best_slot, T *u_star, T *best_cost,
                         hipStream_t s) {
    typedef typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type K;
    hipLaunchKernelGGL((select_kernel<T, K>), dim3(1), dim3(SEL_THREADS), 0, s, cost, pop, k,
                       knots, ld, P.p * P.m, P.m, elite_idx, best_idx, elite_rows, elite_cost,
                       has_elites, best_slot, u_star, best_cost);
    return hipGetLastError();
}
template hipError_t launch_select<float>(const ProbView<float> &, const float *, const float *,
                                         int64_t, int64_t, int, int64_t *, int64_t *, float *,
                                         float *, int *, int *, float *, float *, hipStream_t);
template hipError_t launch_select<double>(const ProbView<double> &, const double *,
                                          const double *, int64_t, int64_t, int, int64_t *,
                                          int64_t *, double *, double *, int *, int *, double *,
                                          double *, hipStream_t);

}  // namespace empc
