// Device bodies of the evolutionary step (gfx950): next population and
// parent selection (Sec. V, Alg. 1 warm / cold start; parent selection of the
// numParents lowest costs).  Shared by the single-problem kernels
// (evolve.hip) and the problem-batched ones (batched.hip).
#pragma once
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

// One thread per (slot s, group g of four parameters j = 4g..4g+3), slot
// fastest so that each of the four stores knots_out[j * ld + s] coalesces.
// The four parameters share their Philox blocks: block 0 (parents), one
// mutation-flag block, one crossover block and one normal block (four
// normals from two Box-Muller pairs).
// Parent knots come from elite_rows ([k][pm], when non-NULL) or from
// knots_in at elite_idx[.].
// cold_mode: 0 warm, 1 cold, 2 cold iff *has_elites == 0.
template <typename T>
__device__ __forceinline__ void population_body(
    const ProbView<T> &P, const GaStreams &gs, int64_t pop, int k, int elitism, T sigma,
    const T *__restrict__ knots_in, int64_t ld_in, const int64_t *__restrict__ elite_idx,
    const T *__restrict__ elite_rows, bool cold, T *__restrict__ knots_out, int64_t ld_out,
    uint32_t tick, uint32_t gen, int64_t t) {
    const int m = P.m, pm = P.p * P.m, ng = (pm + 3) / 4;
    if (t >= pop * ng) return;
    const int64_t s = t % pop;
    const int g = (int)(t / pop);
    const int j0 = 4 * g;
    const uint32_t slot = (uint32_t)s;
    auto parent = [&](int par, int j) -> T {
        return elite_rows ? elite_rows[(int64_t)par * pm + j]
                          : knots_in[(int64_t)j * ld_in + elite_idx[par]];
    };
    T val[4];
    if (cold) {
        const U4 w = ga_draw(gs, slot, gen, tick, 1, (uint32_t)g);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = (j0 + r) % m;
            val[r] = P.umin[i] + (P.umax[i] - P.umin[i]) * uni23<T>(word_of(w, r));
        }
    } else if (elitism && s < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) val[r] = j0 + r < pm ? parent((int)s, j0 + r) : (T)0;
    } else {
        const U4 w0 = ga_draw(gs, slot, gen, tick, 0, 0);
        const int p1 = (int)__umulhi(w0.x, (uint32_t)k);
        const int p2 = (int)__umulhi(w0.y, (uint32_t)k);
        // j0..j0+3 lie in one 128-parameter crossover block
        const U4 wx = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.XB + j0 / 128));
        int fblk = -1;
        U4 wf = {0, 0, 0, 0};
        bool flag[4];
        bool any = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = (j0 + r) % m;
            if (1 + i / 128 != fblk) {
                fblk = 1 + i / 128;
                wf = ga_draw(gs, slot, gen, tick, 0, (uint32_t)fblk);
            }
            const int ib = i % 128;
            flag[r] = j0 + r < pm && ((word_of(wf, ib / 32) >> (ib % 32)) & 1u);
            any |= flag[r];
        }
        T z[4] = {0, 0, 0, 0};
        if (any) {
            const U4 wn = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.NB + g));
#pragma unroll
            for (int pair = 0; pair < 2; ++pair) {
                if (flag[2 * pair] || flag[2 * pair + 1]) {
                    const T u1 = uni23<T>(word_of(wn, 2 * pair));
                    const T u2 = uni23<T>(word_of(wn, 2 * pair + 1));
                    const T rad = sqrt((T)-2 * log_of<T>(u1));
                    T sn, cs;
                    sincos_of<T>((T)6.283185307179586 * u2, &sn, &cs);
                    z[2 * pair] = rad * cs;
                    z[2 * pair + 1] = rad * sn;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + r;
            if (j >= pm) {
                val[r] = 0;
                continue;
            }
            const int i = j % m, jb = j % 128;
            const bool from2 = (word_of(wx, jb / 32) >> (jb % 32)) & 1u;
            T v = parent(from2 ? p2 : p1, j);
            if (flag[r]) v += sigma * z[r];
            v = v < P.umin[i] ? P.umin[i] : v;
            v = v > P.umax[i] ? P.umax[i] : v;
            val[r] = v;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (j0 + r < pm) knots_out[(int64_t)(j0 + r) * ld_out + s] = val[r];
}

template <typename T>
__global__ __launch_bounds__(256) void population_kernel(
    ProbView<T> P, GaStreams gs, int64_t pop, int k, int elitism, T sigma,
    const T *__restrict__ knots_in, int64_t ld_in, const int64_t *__restrict__ elite_idx,
    const T *__restrict__ elite_rows, const int *__restrict__ has_elites, int cold_mode,
    T *__restrict__ knots_out, int64_t ld_out, uint32_t tick, uint32_t gen) {
    const bool cold = cold_mode == 1 || (cold_mode == 2 && *has_elites == 0);
    population_body<T>(P, gs, pop, k, elitism, sigma, knots_in, ld_in, elite_idx, elite_rows, cold,
                       knots_out, ld_out, tick, gen, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Selection: one workgroup of 256 threads (4 wavefronts; a small group keeps
// its barriers cheap, and 4096..16384 keys need no more).  Thread t owns the
// contiguous index range [t*per, (t+1)*per), per = ceil(pop / 256), with the
// sortable keys cached in registers when per <= CACHE.
//  1. radix select of the k-th smallest key, 8 bits per pass.  Costs of a
//     population cluster, so most keys of a pass hit the same few bins: the
//     histogram is replicated 16 times (lane % 16 picks the replica, replicas
//     257 words apart so that one bin of different replicas falls in
//     different LDS banks), which bounds same-address atomics to 4 lanes;
//     two histogram buffers alternate so that clearing the next pass's
//     buffer needs no barrier of its own;
//  2. keys below the threshold are taken, keys equal to it by ascending index
//     until k are taken; two block prefix sums place every taken index, so
//     the elite list comes out in ascending index order;
//  3. best = lowest (key, index) among the elites; elite indices, costs,
//     optionally the elite knot rows, u* = knot 0 of the best, the best cost
//     and the warm-start flag.
constexpr int SEL_THREADS = 256;
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int HREP = 16, HSTRIDE = 257;

__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// Exclusive block prefix sum of v; *total gets the sum.
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

// Inverse of sort_key (NaN keys decode to a NaN, -0 to +0).
__device__ inline float key_value(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
__device__ inline double key_value(uint64_t k) {
    return __longlong_as_double(
        (long long)((k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
}

template <typename T, typename K, int CACHE>
__device__ __forceinline__ void select_body(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    __shared__ int hist[2][HREP * HSTRIDE];
    __shared__ int tot[256];
    __shared__ int wsum[SEL_WAVES];
    __shared__ int s_digit, s_rem;
    __shared__ int64_t s_elite[Limits::MAX_ELITE];
    __shared__ K s_ekey[Limits::MAX_ELITE];
    __shared__ int s_best_slot;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int s = tid; s < k; s += SEL_THREADS) {
        s_elite[s] = 0;
        s_ekey[s] = ~(K)0;
    }
    for (int b = tid; b < HREP * HSTRIDE; b += SEL_THREADS) hist[0][b] = 0;

    const int64_t per = (pop + SEL_THREADS - 1) / SEL_THREADS;
    const int64_t i0 = (int64_t)tid * per;
    const int64_t nmine = per < pop - i0 ? per : (pop - i0 > 0 ? pop - i0 : 0);
    K cache[CACHE > 0 ? CACHE : 1];
    if (CACHE > 0) {
#pragma unroll
        for (int r = 0; r < (CACHE > 0 ? CACHE : 1); ++r)
            cache[r] = r < nmine ? sort_key(cost[i0 + r]) : ~(K)0;
    }
    auto key_at = [&](int64_t r) -> K {
        if (CACHE > 0) {
            K v = cache[0];
#pragma unroll
            for (int q = 1; q < (CACHE > 0 ? CACHE : 1); ++q) v = r == q ? cache[q] : v;
            return v;
        }
        return sort_key(cost[i0 + r]);
    };
    __syncthreads();

    K prefix = 0, mask = 0;
    int remaining = k;
    int buf = 0;
    for (int shift = (int)sizeof(K) * 8 - 8; shift >= 0; shift -= 8) {
        int *myh = hist[buf] + (lane & (HREP - 1)) * HSTRIDE;
        if (CACHE > 0) {
#pragma unroll
            for (int r = 0; r < (CACHE > 0 ? CACHE : 1); ++r) {
                const K key = cache[r];
                if (r < nmine && (key & mask) == prefix)
                    atomicAdd(&myh[(int)((key >> shift) & 255)], 1);
            }
        } else {
            for (int64_t r = 0; r < nmine; ++r) {
                const K key = key_at(r);
                if ((key & mask) == prefix) atomicAdd(&myh[(int)((key >> shift) & 255)], 1);
            }
        }
        // clear the other buffer for the next pass
        for (int b = tid; b < HREP * HSTRIDE; b += SEL_THREADS) hist[buf ^ 1][b] = 0;
        __syncthreads();
        {
            int sum = 0;
#pragma unroll
            for (int rep = 0; rep < HREP; ++rep) sum += hist[buf][rep * HSTRIDE + tid];
            tot[tid] = sum;
        }
        __syncthreads();
        if (tid < 64) {
            // lane owns bins 4*lane .. 4*lane+3
            const int h0 = tot[4 * tid], h1 = tot[4 * tid + 1], h2 = tot[4 * tid + 2],
                      h3 = tot[4 * tid + 3];
            const int own = h0 + h1 + h2 + h3;
            const int incl = wave_incl_scan(own);
            const int excl = incl - own;
            const unsigned long long hit = __ballot(incl >= remaining);
            const int first = __ffsll((long long)hit) - 1;
            if (tid == first) {
                int cum = excl, dsel = 4 * tid + 3;
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
        buf ^= 1;
    }
    const K thr = prefix;
    // ordered pass over this thread's contiguous range
    int my_eq = 0;
    for (int64_t r = 0; r < nmine; ++r) my_eq += key_at(r) == thr ? 1 : 0;
    int eq_tot;
    const int eq_base = block_excl_scan(my_eq, wsum, &eq_tot);
    int my_sel = 0;
    {
        int e = eq_base;
        for (int64_t r = 0; r < nmine; ++r) {
            const K key = key_at(r);
            const bool eq = key == thr;
            my_sel += (key < thr || (eq && e < remaining)) ? 1 : 0;
            e += eq ? 1 : 0;
        }
    }
    int sel_tot;
    int pos = block_excl_scan(my_sel, wsum, &sel_tot);
    {
        int e = eq_base;
        for (int64_t r = 0; r < nmine; ++r) {
            const K key = key_at(r);
            const bool eq = key == thr;
            if (key < thr || (eq && e < remaining)) {
                if (pos < k) {
                    s_elite[pos] = i0 + r;
                    s_ekey[pos] = key;
                }
                ++pos;
            }
            e += eq ? 1 : 0;
        }
    }
    __syncthreads();
    // best among the elites (wave 0)
    if (tid < 64) {
        K bk = ~(K)0;
        int bs = k;
        for (int s = tid; s < k; s += 64) {
            const K key = s_ekey[s];
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
        if (tid == 0) s_best_slot = bs < k ? bs : 0;
    }
    __syncthreads();
    const int bslot = s_best_slot;
    for (int s = tid; s < k; s += SEL_THREADS) {
        if (elite_idx_out) elite_idx_out[s] = s_elite[s];
        if (elite_cost) elite_cost[s] = key_value(s_ekey[s]);
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
        if (best_cost) *best_cost = key_value(s_ekey[bslot]);
    }
    // u*(i) = get_u_from_U(U_best(i), t = 0): knot 0 (idx1 = 0, c = 0)
    if (u_star)
        for (int i = tid; i < m; i += SEL_THREADS) u_star[i] = knots[(int64_t)i * ld + s_elite[bslot]];
}

template <typename T, typename K, int CACHE>
__global__ __launch_bounds__(SEL_THREADS) void select_kernel(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    select_body<T, K, CACHE>(cost, pop, k, knots, ld, pm, m, elite_idx_out, best_idx_out,
                             elite_rows, elite_cost, has_elites, best_slot_out, u_star, best_cost);
}


}  // namespace empc
