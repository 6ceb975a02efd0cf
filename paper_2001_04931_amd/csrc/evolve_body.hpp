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

// One Box-Muller pair from two Philox words.
template <typename T>
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, T &z0, T &z1) {
    const T u1 = uni23<T>(wa);
    const T u2 = uni23<T>(wb);
    const T rad = sqrt((T)-2 * log_of<T>(u1));
    T sn, cs;
    sincos_of<T>((T)6.283185307179586 * u2, &sn, &cs);
    z0 = rad * cs;
    z1 = rad * sn;
}
// FP32: the hardware's log2, square root, sine and cosine (the last two take
// the angle in revolutions, so 2 pi u2 needs no multiply and no range
// reduction: u2 is in (0, 1]).  Absolute error of z below 3e-6 for |z| < 6,
// i.e. below 3e-7 after the sigma = 0.1 scaling, against about 1e-7 for the
// library functions; their range-reduced polynomials cost several times the
// instructions.
template <>
__device__ __forceinline__ void box_muller<float>(uint32_t wa, uint32_t wb, float &z0, float &z1) {
    const float u1 = uni23<float>(wa);
    const float u2 = uni23<float>(wb);
    const float rad =
        __builtin_amdgcn_sqrtf(-2.0f * 0.6931471805599453f * __builtin_amdgcn_logf(u1));
    z0 = rad * __builtin_amdgcn_cosf(u2);
    z1 = rad * __builtin_amdgcn_sinf(u2);
}

// Mutation of one inherited parameter and the bounds (Sec. V warm start).
template <typename T>
__device__ __forceinline__ T mutate_clamp(T v, bool flag, T sigma, T z, T lo, T hi) {
    if (flag) v += sigma * z;
    v = v < lo ? lo : v;
    v = v > hi ? hi : v;
    return v;
}

// Next population (Sec. V, Alg. 1 warm / cold start).  One workgroup of 256
// threads per tile of 64 slots x 4 groups of 4 consecutive parameters: lane l
// of wavefront w builds parameters 4 g .. 4 g + 3 (g = 4 tile_g + w) of slot
// 64 tile_s + l, so that each store of a wavefront covers 64 consecutive
// slots.  The draws that belong to a slot rather than to a parameter (block
// 0: the two parents; the mutation-flag block; the crossover block of the
// tile's 16 parameters, which never straddle a 128-parameter block) are
// taken once per slot by wavefronts 0, 1 and 2 and shared through LDS; each
// thread then draws only its own normal block (two Box-Muller pairs), and
// only if one of its four inputs is flagged.  Parent knots come from
// elite_rows ([p m][k], parameter-major, when non-NULL: the k parents of one
// parameter share two cache lines) or from knots_in at elite_idx[.].
// Inputs per problem: at most 128 (one mutation-flag block).
constexpr int POP_SLOTS = 64;   // slots per workgroup, one per lane
constexpr int POP_GROUPS = 4;   // groups of four parameters, one per wavefront
constexpr int POP_THREADS = 64 * POP_GROUPS;

template <typename T>
__device__ __forceinline__ void population_tile(
    const ProbView<T> &P, const GaStreams &gs, int64_t pop, int k, int elitism, T sigma,
    const T *__restrict__ knots_in, int64_t ld_in, const int64_t *__restrict__ elite_idx,
    const T *__restrict__ elite_rows, bool cold, T *__restrict__ knots_out, int64_t ld_out,
    uint32_t tick, uint32_t gen, int64_t tile_s, int tile_g, const PopVariant<T> &var,
    int R = 1) {
    __shared__ int s_par[POP_SLOTS][2];
    __shared__ int64_t s_eidx[Limits::MAX_ELITE];
    __shared__ __align__(16) uint32_t s_flag[POP_SLOTS][4];
    __shared__ __align__(16) uint32_t s_xw[POP_SLOTS][4];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = P.m, pm = P.p * P.m;
    // the workgroup's parameters: 16 R from jt (R in {1, 2, 4, 8}, so that
    // they lie in one 128-parameter crossover block); wavefront w takes the
    // groups of four at jt + 16 r + 4 w, r < R
    const int jt = tile_g * POP_GROUPS * 4 * R;
    if (jt >= pm) return;  // whole workgroup: no parameter here
    const int64_t s = tile_s * POP_SLOTS + lane;
    const uint32_t slot = (uint32_t)s;
    // the parents' indices are staged in LDS by the fourth wavefront while
    // the others draw, so no global load waits on a draw
    if (!cold && w == 3 && !elite_rows)
        for (int i = lane; i < k; i += 64) s_eidx[i] = elite_idx[i];
    if (!cold && s < pop) {
        if (w == 0) {
            const U4 w0 = ga_draw(gs, slot, gen, tick, 0, 0);
            s_par[lane][0] = (int)__umulhi(w0.x, (uint32_t)k);
            s_par[lane][1] = (int)__umulhi(w0.y, (uint32_t)k);
        } else if (w == 1) {
            const U4 wf = ga_draw(gs, slot, gen, tick, 0, 1);
            s_flag[lane][0] = wf.x;
            s_flag[lane][1] = wf.y;
            s_flag[lane][2] = wf.z;
            s_flag[lane][3] = wf.w;
        } else if (w == 2) {
            const int xb = jt / 128;
            const U4 wx = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.XB + xb));
            s_xw[lane][0] = wx.x;
            s_xw[lane][1] = wx.y;
            s_xw[lane][2] = wx.z;
            s_xw[lane][3] = wx.w;
        }
    }
    __syncthreads();
    if (s >= pop) return;
    // distance-dependent mutation noise (Sec. VII): sigma_min at the goal,
    // growing linearly to sigma at distance sigma_dist (uniform per wavefront)
    if (var.sigma_dist > (T)0) {
        T d2 = 0;
        for (int i = 0; i < P.n; ++i) {
            const T e = var.x0[i] - (P.xg ? P.xg[i] : (T)0);
            d2 += e * e;
        }
        const T r = sqrt(d2) / var.sigma_dist;
        sigma = var.sigma_min + (sigma - var.sigma_min) * (r < (T)1 ? r : (T)1);
    }
    for (int rg = 0; rg < R; ++rg) {
        const int j0 = jt + 16 * rg + 4 * w;
        if (j0 >= pm) break;
        // inputs of parameters j0 .. j0+3: one division, then wrap at m
        int ii[4];
        ii[0] = j0 % m;
#pragma unroll
        for (int r = 1; r < 4; ++r) ii[r] = ii[r - 1] + 1 == m ? 0 : ii[r - 1] + 1;
        T val[4];
        if (cold) {
            const U4 wc = ga_draw(gs, slot, gen, tick, 1, (uint32_t)(j0 / 4));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ii[r];
                val[r] = P.umin[i] + (P.umax[i] - P.umin[i]) * uni23<T>(word_of(wc, r));
            }
        } else {
            const T *base = elite_rows ? elite_rows : knots_in;
            const int64_t step = elite_rows ? k : ld_in;
            // the parent's values of all four parameters are loaded first, so
            // that the loads are in flight together and behind the draws;
            // parameter j of the parent stored at src, and with the shift the
            // carried input one control step later, (1-d) U_a + d U_{a+1} for
            // knot a < p-1 (d = (p-1)/(T-1), the knot spacing in steps
            // inverted).  Indices past the last parameter load parameter
            // pm-1 and are never stored.
            const T d = P.p > 1 ? (T)(P.p - 1) / (T)(P.Tn - 1) : (T)0;
            const bool elite_slot = elitism && s < k;
            int64_t src[4];
            bool flag[4] = {false, false, false, false};
            if (elite_slot) {
                const int64_t e = elite_rows ? s : s_eidx[s];
#pragma unroll
                for (int r = 0; r < 4; ++r) src[r] = e;
            } else {
                const int p1 = s_par[lane][0], p2 = s_par[lane][1];
                const int64_t src1 = elite_rows ? (int64_t)p1 : s_eidx[p1];
                const int64_t src2 = elite_rows ? (int64_t)p2 : s_eidx[p2];
                typedef uint32_t w4 __attribute__((ext_vector_type(4)));
                const w4 fw = *reinterpret_cast<const w4 *>(&s_flag[lane][0]);
                const w4 xw = *reinterpret_cast<const w4 *>(&s_xw[lane][0]);
                auto word = [](const w4 &v, int q) {
                    return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
                };
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = j0 + r, jb = j % 128;
                    flag[r] = j < pm && ((word(fw, ii[r] / 32) >> (ii[r] % 32)) & 1u);
                    const bool from2 = (word(xw, jb / 32) >> (jb % 32)) & 1u;
                    src[r] = from2 ? src2 : src1;
                }
            }
            T pv[4], pn[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + r < pm ? j0 + r : pm - 1;
                pv[r] = base[src[r] + (int64_t)j * step];
            }
            if (var.shift) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = j0 + r < pm ? j0 + r : pm - 1;
                    pn[r] = j / m < P.p - 1 ? base[src[r] + (int64_t)(j + m) * step] : pv[r];
                }
            }
            T z[4] = {0, 0, 0, 0};
            if (flag[0] || flag[1] || flag[2] || flag[3]) {
                const U4 wn = ga_draw(gs, slot, gen, tick, 0, (uint32_t)(gs.NB + j0 / 4));
                if (flag[0] || flag[1]) box_muller<T>(wn.x, wn.y, z[0], z[1]);
                if (flag[2] || flag[3]) box_muller<T>(wn.z, wn.w, z[2], z[3]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + r;
                if (j >= pm) {
                    val[r] = 0;
                    continue;
                }
                T v = pv[r];
                if (var.shift && j / m < P.p - 1) v = ((T)1 - d) * v + d * pn[r];
                val[r] = elite_slot ? v
                                    : mutate_clamp<T>(v, flag[r], sigma, z[r], P.umin[ii[r]],
                                                      P.umax[ii[r]]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (j0 + r < pm) knots_out[(int64_t)(j0 + r) * ld_out + s] = val[r];
    }
}

// tiles of a population of `pop` slots and p m parameters
__host__ __device__ inline int64_t pop_tiles_s(int64_t pop) { return (pop + POP_SLOTS - 1) / POP_SLOTS; }
__host__ __device__ inline int pop_tiles_g(int pm, int R = 1) {
    return ((pm + 3) / 4 + POP_GROUPS * R - 1) / (POP_GROUPS * R);
}

template <typename T>
__global__ __launch_bounds__(POP_THREADS) void population_kernel(
    ProbView<T> P, GaStreams gs, int64_t pop, int k, int elitism, T sigma,
    const T *__restrict__ knots_in, int64_t ld_in, const int64_t *__restrict__ elite_idx,
    const T *__restrict__ elite_rows, const int *__restrict__ has_elites, int cold_mode,
    T *__restrict__ knots_out, int64_t ld_out, uint32_t tick, uint32_t gen, PopVariant<T> var,
    int R) {
    const bool cold = cold_mode == 1 || (cold_mode == 2 && *has_elites == 0);
    const int64_t nts = pop_tiles_s(pop);
    population_tile<T>(P, gs, pop, k, elitism, sigma, knots_in, ld_in, elite_idx, elite_rows, cold,
                       knots_out, ld_out, tick, gen, blockIdx.x % nts, (int)(blockIdx.x / nts),
                       var, R);
}

// ---------------------------------------------------------------------------
// Selection (parent selection: the numParents lowest costs).  One workgroup
// of 256 threads (4 wavefronts; a small group keeps its barriers cheap, and
// 4096..16384 keys need no more).  Thread t owns the contiguous index range
// [t per, (t+1) per), per = ceil(pop / 256), with the sortable keys cached
// in registers when per <= CACHE (loaded 16 bytes at a time).
//     Populations above 1024 use a workgroup of 1024 threads instead.
//  1. radix select of the k-th smallest key, 8 bits per pass, starting below
//     the bytes that every key shares (from the block's min and max key).
//     Costs of a population cluster, so most keys of a pass hit the same few
//     bins: the histogram is replicated 16 times (lane % 16 picks the
//     replica, replicas 257 words apart so that one bin of different
//     replicas falls in different LDS banks), which bounds same-address
//     atomics to 4 lanes; two histogram buffers alternate so that clearing
//     the next pass's buffer needs no barrier of its own, and every
//     wavefront scans the bin totals itself, so a pass has two barriers;
//  2. keys below the threshold are taken, keys equal to it by ascending index
//     until k are taken; one block prefix sum of the packed (below, equal)
//     counts places every taken index, so the elite list comes out in
//     ascending index order;
//  3. best = lowest (key, index) among the elites; elite indices, costs,
//     optionally the elite knot rows, u* = knot 0 of the best, the best cost
//     and the warm-start flag.
constexpr int SEL_THREADS = 256;
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int HREP = 16, HSTRIDE = 257;

// Inclusive scan over a full wavefront: within each 16-lane row by DPP row
// shifts (zero shifted in), then the totals of the rows below, read from
// lanes 15, 31 and 47.  Every lane of the wavefront must be active.
__device__ inline int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(v, 15);
    const int r1 = __builtin_amdgcn_readlane(v, 31);
    const int r2 = __builtin_amdgcn_readlane(v, 47);
    const int row = (threadIdx.x & 63) >> 4;
    return v + (row > 0 ? r0 : 0) + (row > 1 ? r1 : 0) + (row > 2 ? r2 : 0);
}

// Exclusive block prefix sum of v over NW wavefronts; *total gets the sum.
template <int NW>
__device__ inline int block_excl_scan(int v, int *wsum, int *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int incl = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int x = wsum[w];
        base += w < wave ? x : 0;
        tot += x;
    }
    *total = tot;
    return base + incl - v;
}

template <typename K>
__device__ inline K wave_min(K v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const K u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}
template <typename K>
__device__ inline K wave_max(K v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const K u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

// Inverse of sort_key (NaN keys decode to a NaN, -0 to +0).
__device__ inline float key_value(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
__device__ inline double key_value(uint64_t k) {
    return __longlong_as_double(
        (long long)((k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
}

// NREP: histogram replicas (a power of two <= 16); a one-wavefront selection
// inside the persistent batched kernel takes 1 to keep its LDS small.
template <typename T, typename K, int CACHE, int NTHR = SEL_THREADS, int NREP = HREP>
__device__ __forceinline__ void select_body(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    __shared__ int hist[2][NREP * HSTRIDE];
    __shared__ int tot[256];
    __shared__ int wsum[(NTHR / 64)];
    __shared__ K s_lo[(NTHR / 64)], s_hi[(NTHR / 64)];
    __shared__ int64_t s_elite[Limits::MAX_ELITE];
    __shared__ K s_ekey[Limits::MAX_ELITE];
    __shared__ int s_best_slot;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int b = tid; b < NREP * HSTRIDE; b += NTHR) hist[0][b] = 0;

    const int64_t per = (pop + NTHR - 1) / NTHR;
    const int64_t i0 = (int64_t)tid * per;
    const int64_t nmine = per < pop - i0 ? per : (pop - i0 > 0 ? pop - i0 : 0);
    K cache[CACHE > 0 ? CACHE : 1];
    if constexpr (CACHE > 0) {
        typedef T v4 __attribute__((ext_vector_type(4)));
        const bool vec = CACHE % 4 == 0 && nmine == CACHE &&
                         (reinterpret_cast<uintptr_t>(cost + i0) & (sizeof(v4) - 1)) == 0;
        if (vec) {
#pragma unroll
            for (int q = 0; q < CACHE / 4; ++q) {
                const v4 c = reinterpret_cast<const v4 *>(cost + i0)[q];
                cache[4 * q + 0] = sort_key(c.x);
                cache[4 * q + 1] = sort_key(c.y);
                cache[4 * q + 2] = sort_key(c.z);
                cache[4 * q + 3] = sort_key(c.w);
            }
        } else {
#pragma unroll
            for (int r = 0; r < CACHE; ++r) cache[r] = r < nmine ? sort_key(cost[i0 + r]) : ~(K)0;
        }
    }
    // visit this thread's keys in index order; with the cache every index
    // is a compile-time constant, so the keys stay in registers
    auto for_each_key = [&](auto &&f) {
        if (CACHE > 0) {
#pragma unroll
            for (int r = 0; r < (CACHE > 0 ? CACHE : 1); ++r)
                if (r < nmine) f((int64_t)r, cache[r]);
        } else {
            for (int64_t r = 0; r < nmine; ++r) f(r, sort_key(cost[i0 + r]));
        }
    };
    {  // the block's smallest and largest key
        K lo = ~(K)0, hi = 0;
        for_each_key([&](int64_t, K key) {
            lo = key < lo ? key : lo;
            hi = key > hi ? key : hi;
        });
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane == 0) {
            s_lo[wave] = lo;
            s_hi[wave] = hi;
        }
    }
    __syncthreads();
    K lo = s_lo[0], hi = s_hi[0];
#pragma unroll
    for (int w = 1; w < (NTHR / 64); ++w) {
        lo = s_lo[w] < lo ? s_lo[w] : lo;
        hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    // bytes every key shares need no pass: start at the highest byte where
    // the smallest and the largest key differ (byte 0 if they are equal)
    constexpr int BITS = (int)sizeof(K) * 8;
    int top = BITS - 8;
    while (top > 0 && (((lo ^ hi) >> top) & 255) == 0) top -= 8;
    K mask = (~(K)0 << top) << 8;  // the bytes above `top` (two shifts: no shift by BITS)
    K prefix = lo & mask;
    int remaining = k;
    int buf = 0;
    for (int shift = top; shift >= 0; shift -= 8) {
        int *myh = hist[buf] + (lane & (NREP - 1)) * HSTRIDE;
        for_each_key([&](int64_t, K key) {
            if ((key & mask) == prefix) atomicAdd(&myh[(int)((key >> shift) & 255)], 1);
        });
        // clear the other buffer for the next pass
        for (int b = tid; b < NREP * HSTRIDE; b += NTHR) hist[buf ^ 1][b] = 0;
        __syncthreads();
        for (int bin = tid; bin < 256; bin += NTHR) {  // one bin per thread
            int sum = 0;
#pragma unroll
            for (int rep = 0; rep < NREP; ++rep) sum += hist[buf][rep * HSTRIDE + bin];
            tot[bin] = sum;
        }
        __syncthreads();
        // every wavefront finds the digit itself: lane owns bins 4 lane .. +3
        const int h0 = tot[4 * lane], h1 = tot[4 * lane + 1], h2 = tot[4 * lane + 2],
                  h3 = tot[4 * lane + 3];
        const int own = h0 + h1 + h2 + h3;
        const int incl = wave_incl_scan(own);
        const unsigned long long hit = __ballot(incl >= remaining);
        const int first = __ffsll((long long)hit) - 1;
        int cum = incl - own, q = 3;
        if (cum + h0 >= remaining) {
            q = 0;
        } else if (cum + h0 + h1 >= remaining) {
            q = 1;
            cum += h0;
        } else if (cum + h0 + h1 + h2 >= remaining) {
            q = 2;
            cum += h0 + h1;
        } else {
            cum += h0 + h1 + h2;
        }
        const int digit = __builtin_amdgcn_readlane(4 * lane + q, first);
        remaining -= __builtin_amdgcn_readlane(cum, first);
        prefix |= (K)digit << shift;
        mask |= (K)255 << shift;
        buf ^= 1;
    }
    const K thr = prefix;
    // ordered pass over this thread's contiguous range: one scan of the
    // packed counts (below the threshold in the low half, equal in the high)
    int my_lt = 0, my_eq = 0;
    for_each_key([&](int64_t, K key) {
        my_lt += key < thr ? 1 : 0;
        my_eq += key == thr ? 1 : 0;
    });
    int packed_tot, lt_base, eq_base;
    if (CACHE > 0 && pop < (1 << 15)) {  // below < k <= 256, equal < 2^15: packed in 31 bits
        const int base = block_excl_scan<NTHR / 64>(my_lt | (my_eq << 16), wsum, &packed_tot);
        lt_base = base & 0xFFFF;
        eq_base = base >> 16;
    } else {
        int t1;
        lt_base = block_excl_scan<NTHR / 64>(my_lt, wsum, &t1);
        __syncthreads();
        eq_base = block_excl_scan<NTHR / 64>(my_eq, wsum, &t1);
    }
    {
        int e = eq_base;
        int pos = lt_base + min(eq_base, remaining);
        for_each_key([&](int64_t r, K key) {
            const bool eq = key == thr;
            if (key < thr || (eq && e < remaining)) {
                if (pos < k) {
                    s_elite[pos] = i0 + r;
                    s_ekey[pos] = key;
                }
                ++pos;
            }
            e += eq ? 1 : 0;
        });
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
    for (int s = tid; s < k; s += NTHR) {
        if (elite_idx_out) elite_idx_out[s] = s_elite[s];
        if (elite_cost) elite_cost[s] = key_value(s_ekey[s]);
    }
    if (elite_rows)  // parameter-major: elite_rows[j k + s]
        for (int t = tid; t < k * pm; t += NTHR) {
            const int j = t / k, s = t - j * k;
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
        for (int i = tid; i < m; i += NTHR) u_star[i] = knots[(int64_t)i * ld + s_elite[bslot]];
}

// Selection for populations of at most 256 by one wavefront (no
// histogram passes): lane l holds candidates l, l + 64, l + 128, l + 192 as (key,
// index) pairs (past the population: the largest key and an index past the
// population), a bitonic network sorts the 256 pairs ascending (partners
// closer than 64 positions through lane shuffles, farther ones within the
// lane's registers), so position p holds the p-th lowest (key, index) and
// the parents are positions 0..k-1, the best one position 0.  Each parent's
// slot in the ascending-index parent list is its rank by index among them.
// The outputs are those of select_body, bit for bit (the same total order
// decides).
template <typename T, typename K>
__global__ __launch_bounds__(64) void select_small_kernel(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    __shared__ int s_sidx[256];      // sorted indices (positions 0..k-1)
    __shared__ int64_t s_elite[256];  // parents in ascending index order
    __shared__ K s_ekey[256];
    __shared__ int s_best_slot;
    const int lane = threadIdx.x;
    K key[4];
    int idx[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = lane + 64 * r;
        idx[r] = e;
        key[r] = e < pop ? sort_key(cost[e]) : ~(K)0;
    }
    auto less = [](K ka, int ia, K kb, int ib) { return ka < kb || (ka == kb && ia < ib); };
#pragma unroll
    for (int size = 2; size <= 256; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride > 0; stride >>= 1) {
            if (stride >= 64) {  // partner in this lane: register r ^ (stride / 64)
                const int rb = stride / 64;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r & rb) continue;
                    const int e = lane + 64 * r, h = r | rb;
                    const bool asc = (e & size) == 0;
                    const bool swap = asc ? less(key[h], idx[h], key[r], idx[r])
                                          : less(key[r], idx[r], key[h], idx[h]);
                    if (swap) {
                        const K tk = key[r];
                        const int ti = idx[r];
                        key[r] = key[h];
                        idx[r] = idx[h];
                        key[h] = tk;
                        idx[h] = ti;
                    }
                }
            } else {  // partner lane ^ stride, same register
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = lane + 64 * r;
                    const K ok = __shfl_xor(key[r], stride, 64);
                    const int oi = __shfl_xor(idx[r], stride, 64);
                    const bool asc = (e & size) == 0, lower = (e & stride) == 0;
                    // the lower position keeps the smaller pair when ascending
                    const bool other_less = less(ok, oi, key[r], idx[r]);
                    const bool take = (lower == asc) ? other_less : !other_less;
                    if (take) {
                        key[r] = ok;
                        idx[r] = oi;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) s_sidx[lane + 64 * r] = idx[r];
    __syncthreads();
    // parent at sorted position p < k goes to slot rank(p) = number of
    // parents with a smaller index
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = lane + 64 * r;
        if (p < k) {
            int rank = 0;
            for (int q = 0; q < k; ++q) rank += s_sidx[q] < idx[r] ? 1 : 0;
            s_elite[rank] = idx[r];
            s_ekey[rank] = key[r];
            if (p == 0) s_best_slot = rank;
        }
    }
    __syncthreads();
    const int bslot = s_best_slot;
    for (int s2 = lane; s2 < k; s2 += 64) {
        if (elite_idx_out) elite_idx_out[s2] = s_elite[s2];
        if (elite_cost) elite_cost[s2] = key_value(s_ekey[s2]);
    }
    if (elite_rows)  // parameter-major: elite_rows[j k + s]
        for (int t = lane; t < k * pm; t += 64) {
            const int j = t / k, s2 = t - j * k;
            elite_rows[t] = knots[(int64_t)j * ld + s_elite[s2]];
        }
    if (lane == 0) {
        if (best_idx_out) *best_idx_out = s_elite[bslot];
        if (has_elites) *has_elites = 1;
        if (best_slot_out) *best_slot_out = bslot;
        if (best_cost) *best_cost = key_value(s_ekey[bslot]);
    }
    if (u_star)
        for (int i = lane; i < m; i += 64) u_star[i] = knots[(int64_t)i * ld + s_elite[bslot]];
}

template <typename T, typename K, int CACHE, int NTHR>
__global__ __launch_bounds__(NTHR) void select_kernel(
    const T *__restrict__ cost, int64_t pop, int k, const T *__restrict__ knots, int64_t ld,
    int pm, int m, int64_t *__restrict__ elite_idx_out, int64_t *__restrict__ best_idx_out,
    T *__restrict__ elite_rows, T *__restrict__ elite_cost, int *__restrict__ has_elites,
    int *__restrict__ best_slot_out, T *__restrict__ u_star, T *__restrict__ best_cost) {
    select_body<T, K, CACHE, NTHR>(cost, pop, k, knots, ld, pm, m, elite_idx_out, best_idx_out,
                                   elite_rows, elite_cost, has_elites, best_slot_out, u_star,
                                   best_cost);
}


}  // namespace empc
