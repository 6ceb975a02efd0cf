// Internal declarations of the EMPC HIP library (gfx950).  Not installed;
// the public interface is include/empc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/empc.h"

namespace empc {

// ---------------------------------------------------------------------------
// Problem view handed to kernels by value.  Pointers are device pointers of
// element type T (the problem dtype).
template <typename T>
struct ProbView {
    int n, m, Tn, p;
    const T *Ad, *Bd, *wd;
    const T *stiff, *damp, *mass, *len;
    T gravity, dt;
    const T *q, *r, *qf, *xg, *ug, *umin, *umax;
    const T *xlo, *xhi, *qb;  // state box penalty (qb NULL: none)
    const T *sb;              // charge per step outside the box (NULL: none)
    const T *qlo, *qhi;       // chain joint limits with impacts (NULL: none)
    T rest;                   // impact restitution
    const T *Qm, *Rm, *Qfm;   // full weights (NULL: the diagonals)
    const T *fc, *fs;         // chain dry friction: sliding, breakaway (NULL: none)
};

template <typename T>
inline ProbView<T> view_of(const empc_problem &P) {
    ProbView<T> v;
    v.n = P.n; v.m = P.m; v.Tn = P.T; v.p = P.p;
    v.Ad = (const T *)P.Ad; v.Bd = (const T *)P.Bd; v.wd = (const T *)P.wd;
    v.stiff = (const T *)P.stiffness; v.damp = (const T *)P.damping;
    v.mass = (const T *)P.mass; v.len = (const T *)P.length;
    v.gravity = (T)P.gravity; v.dt = (T)P.dt;
    v.q = (const T *)P.q; v.r = (const T *)P.r; v.qf = (const T *)P.qf;
    v.xg = (const T *)P.x_goal; v.ug = (const T *)P.u_goal;
    v.umin = (const T *)P.u_min; v.umax = (const T *)P.u_max;
    v.xlo = (const T *)P.x_min; v.xhi = (const T *)P.x_max; v.qb = (const T *)P.qb;
    v.sb = (const T *)P.sb;
    v.qlo = (const T *)P.q_min; v.qhi = (const T *)P.q_max; v.rest = (T)P.restitution;
    v.Qm = (const T *)P.Q; v.Rm = (const T *)P.R; v.Qfm = (const T *)P.Qf;
    v.fc = (const T *)P.fric_c; v.fs = (const T *)P.fric_s;
    return v;
}

// the problem has full weights (the vector-ALU rollout handles them)
template <typename T>
__host__ __device__ inline bool full_weights(const ProbView<T> &P) {
    return P.Qm || P.Rm || P.Qfm;
}

// State box penalty of one state: squared distance to [lo, hi] (unweighted),
// and the derivative of w times it.
template <typename T>
__host__ __device__ inline T box_pen(T x, T lo, T hi) {
    const T o = x - hi, u = lo - x;
    return (o > (T)0 ? o * o : (T)0) + (u > (T)0 ? u * u : (T)0);
}
// 1 if x lies outside [lo, hi], else 0 (the step charge's indicator)
template <typename T>
__host__ __device__ inline T box_out(T x, T lo, T hi) {
    return (x > hi || x < lo) ? (T)1 : (T)0;
}
// Joint limit with an impact: a joint past a limit is put back on it and its
// rate, if it still points outward, reversed and scaled by e.
template <typename T>
__host__ __device__ inline void joint_limit(T &q, T &v, T lo, T hi, T e) {
    if (q > hi) {
        q = hi;
        if (v > (T)0) v = -e * v;
    } else if (q < lo) {
        q = lo;
        if (v < (T)0) v = -e * v;
    }
}
// Dry friction with stiction on one joint's rate update: v the rate before
// the step, vf = v + dti f the rate without friction (f the other torques,
// dti = dt / I), tc the sliding and ts the breakaway torque.  At rest: stays
// at rest while |f| <= ts, else breaks away against tc; moving: slowed by
// tc, and held at zero where that (or f within ts) turns it round.
template <typename T>
__host__ __device__ inline T dry_friction(T v, T vf, T f, T dti, T tc, T ts) {
    const T af = f < (T)0 ? -f : f;
    if (v == (T)0) return af <= ts ? (T)0 : vf - dti * tc * (f > (T)0 ? (T)1 : (T)-1);
    const T vn = vf - dti * tc * (v > (T)0 ? (T)1 : (T)-1);
    return (vn * v <= (T)0 && af <= ts) ? (T)0 : vn;
}
template <typename T>
__host__ __device__ inline T box_pen_grad(T x, T lo, T hi, T w) {
    const T o = x - hi, u = lo - x;
    return o > (T)0 ? (T)2 * w * o : (u > (T)0 ? (T)-2 * w * u : (T)0);
}

// Knot interpolation of Sec. IV-C in exact integers: with num = k (p-1) and
// den = T-1, idx1 = num / den, c = (num mod den) / den, idx2 = min(idx1+1, p-1).
struct Knot {
    int a, b;
    int rem, den;
};
__host__ __device__ inline Knot knot_at(int T, int p, int k) {
    Knot s;
    if (p == 1 || T == 1) {
        s.a = 0; s.b = 0; s.rem = 0; s.den = 1;
        return s;
    }
    int num = k * (p - 1);
    s.den = T - 1;
    s.a = num / s.den;
    s.rem = num - s.a * s.den;
    s.b = s.a + 1 < p ? s.a + 1 : p - 1;
    return s;
}

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11).
struct U4 {
    uint32_t x, y, z, w;
};
__device__ inline U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // one 32 x 32 -> 64-bit product per multiplier (a single
        // v_mad_u64_u32 instead of separate low and high multiplies)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}
__device__ inline uint32_t word_of(const U4 &v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Stream layout of the evolutionary draws (counter = (slot, gen, tick,
// stream << 24 | block), key = seed): warm start (stream 0) uses block 0 for
// the two parent draws, blocks 1.. for mutation flags (input i: block
// 1 + i/128, bit i%128), blocks XB.. for crossover bits (parameter j: block
// XB + j/128, bit j%128), blocks NB.. for normals (parameter j: block NB + j/4,
// Box-Muller pair (0,1) or (2,3)); cold start (stream 1): parameter j uses
// block j/4, word j%4.
struct GaStreams {
    uint32_t k0, k1;
    int XB, NB;
};
inline GaStreams ga_streams(uint64_t seed, int m, int pm) {
    GaStreams s;
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    s.XB = 1 + (m + 127) / 128;
    s.NB = s.XB + (pm + 127) / 128;
    return s;
}
__device__ inline U4 ga_draw(const GaStreams &g, uint32_t slot, uint32_t gen, uint32_t tick,
                             uint32_t stream, uint32_t block) {
    return philox10(U4{slot, gen, tick, (stream << 24) | block}, g.k0, g.k1);
}
// Open-interval uniform (2 (w >> 9) + 1) 2^-24, exact in float and double.
template <typename T>
__device__ inline T uni23(uint32_t w) {
    return ((T)(w >> 9) + (T)0.5) * (T)(1.0 / 8388608.0);
}

// ---------------------------------------------------------------------------
// Totally ordered unsigned keys of costs: NaN maps above +inf and -0 to the
// key of +0, so that key order is the numeric order of the costs.
__device__ inline uint32_t sort_key(float v) {
    if (v != v) return 0xFFFFFFFFu;
    const uint32_t b = v == 0.0f ? 0u : __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline uint64_t sort_key(double v) {
    if (v != v) return ~0ull;
    const uint64_t b = v == 0.0 ? 0ull : (uint64_t)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// ---------------------------------------------------------------------------
// One problem of a batch: its view and its slice of the batch workspace.
template <typename T>
struct BatchSlot {
    ProbView<T> P;
    int model;
    uint32_t key_hi;   // Philox key high word of this problem: seed_hi ^ index
    const T *x0;       // n
    T *knots[2];       // [pm][pop] each
    T *cost;           // pop
    T *elite_rows;     // [pm][k], parameter-major
    T *elite_cost;     // k
    int64_t *elite_idx, *best_idx;
    int *has_elites;
    T *u_star;         // m (inside the caller's packed u* array)
    T *best_cost;      // 1
};

// Pointers that a kernel reads from memory (a batch slot's fields) are of
// unknown address space to the compiler, so accesses through them compile
// to flat instructions, which also count against the LDS wait counter (an
// LDS wait then drains every global load in flight).  All of a slot's
// memory is device global memory: re-made from its integer value as a
// global pointer (a cast the optimizer keeps), each becomes global loads
// and stores.
template <typename T>
__device__ __forceinline__ T *global_ptr(T *p) {
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ ProbView<T> global_view(ProbView<T> v) {
    v.Ad = global_ptr(v.Ad); v.Bd = global_ptr(v.Bd); v.wd = global_ptr(v.wd);
    v.stiff = global_ptr(v.stiff); v.damp = global_ptr(v.damp);
    v.mass = global_ptr(v.mass); v.len = global_ptr(v.len);
    v.q = global_ptr(v.q); v.r = global_ptr(v.r); v.qf = global_ptr(v.qf);
    v.xg = global_ptr(v.xg); v.ug = global_ptr(v.ug);
    v.umin = global_ptr(v.umin); v.umax = global_ptr(v.umax);
    v.xlo = global_ptr(v.xlo); v.xhi = global_ptr(v.xhi); v.qb = global_ptr(v.qb);
    v.sb = global_ptr(v.sb); v.qlo = global_ptr(v.qlo); v.qhi = global_ptr(v.qhi);
    v.Qm = global_ptr(v.Qm); v.Rm = global_ptr(v.Rm); v.Qfm = global_ptr(v.Qfm);
    v.fc = global_ptr(v.fc); v.fs = global_ptr(v.fs);
    return v;
}

// ---------------------------------------------------------------------------
// Launchers (one per kernel family), defined in the .hip files.
// All return a hipError_t from the launch.
struct Limits {
    static constexpr int MAX_N_LINEAR = 80;
    static constexpr int MAX_M_LINEAR = 40;
    static constexpr int MAX_D_CHAIN = 40;
    static constexpr int MAX_ELITE = 256;
};
constexpr int VALU_FULL_NMAX = 64;  // largest n with full weights (16-lane row form)
constexpr int VALU_FULL_MMAX = 32;  // largest m with full weights

// Optional start / stop events stamped by a kernel's dispatch.
// Workgroups are dispatched to the chip's 8 XCDs round-robin (linear
// workgroup b on XCD b mod 8), and each XCD has its own L2.  The rollout
// kernels map workgroup b to work item xcd_swizzle(b, nb) instead of b, so
// that each XCD gets one contiguous range of tiles: neighbouring tiles share
// cache lines of the candidate-innermost knot layout, which are then fetched
// by one L2 instead of two.  A bijection of [0, nb).
__device__ inline int64_t xcd_swizzle(int64_t b, int64_t nb) {
    constexpr int64_t NX = 8;
    const int64_t q = nb / NX, r = nb % NX, x = b % NX;
    return x * q + (x < r ? x : r) + b / NX;
}
// The same for a 2-D grid (x fastest): returns the swizzled linear index.
__device__ inline int64_t xcd_swizzle_2d() {
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    return xcd_swizzle((int64_t)blockIdx.y * gridDim.x + blockIdx.x, nb);
}

// ---------------------------------------------------------------------------
// Cross-lane helpers on DPP row shifts (a row = 16 lanes; shifted-in lanes
// read 0) and lane reads.  Every lane of the wavefront must be active.
template <typename T>
__device__ inline T row_shift_up(T v, int n);  // lane r gets lane r-n of its row, 0 below
template <>
__device__ inline float row_shift_up<float>(float v, int n) {
    int x = __float_as_int(v), y = 0;
    switch (n) {
        case 1: y = __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false); break;
        case 2: y = __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false); break;
        case 4: y = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false); break;
        default: y = __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false); break;
    }
    return __int_as_float(y);
}
template <typename T>
__device__ inline T row_shift_down(T v, int n);  // lane r gets lane r+n of its row, 0 above
template <>
__device__ inline float row_shift_down<float>(float v, int n) {
    int x = __float_as_int(v), y = 0;
    switch (n) {
        case 1: y = __builtin_amdgcn_update_dpp(0, x, 0x101, 0xf, 0xf, false); break;
        case 2: y = __builtin_amdgcn_update_dpp(0, x, 0x102, 0xf, 0xf, false); break;
        case 4: y = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xf, 0xf, false); break;
        default: y = __builtin_amdgcn_update_dpp(0, x, 0x108, 0xf, 0xf, false); break;
    }
    return __int_as_float(y);
}
// 64-bit values: two 32-bit DPP moves
template <>
__device__ inline double row_shift_up<double>(double v, int n) {
    const int lo = (int)(__double_as_longlong(v) & 0xffffffffll);
    const int hi = (int)(__double_as_longlong(v) >> 32);
    const float flo = row_shift_up<float>(__int_as_float(lo), n);
    const float fhi = row_shift_up<float>(__int_as_float(hi), n);
    return __longlong_as_double(((long long)(unsigned)__float_as_int(fhi) << 32) |
                                (unsigned)__float_as_int(flo));
}
template <>
__device__ inline double row_shift_down<double>(double v, int n) {
    const int lo = (int)(__double_as_longlong(v) & 0xffffffffll);
    const int hi = (int)(__double_as_longlong(v) >> 32);
    const float flo = row_shift_down<float>(__int_as_float(lo), n);
    const float fhi = row_shift_down<float>(__int_as_float(hi), n);
    return __longlong_as_double(((long long)(unsigned)__float_as_int(fhi) << 32) |
                                (unsigned)__float_as_int(flo));
}
// inclusive scans over the 16 lanes of a row
template <typename T>
__device__ inline T row_scan_up(T v) {
    v += row_shift_up<T>(v, 1);
    v += row_shift_up<T>(v, 2);
    v += row_shift_up<T>(v, 4);
    v += row_shift_up<T>(v, 8);
    return v;
}
template <typename T>
__device__ inline T row_scan_down(T v) {
    v += row_shift_down<T>(v, 1);
    v += row_shift_down<T>(v, 2);
    v += row_shift_down<T>(v, 4);
    v += row_shift_down<T>(v, 8);
    return v;
}

// lane j's value in every lane
template <typename T>
__device__ inline T lane_bcast(T v, int j);
template <>
__device__ inline float lane_bcast<float>(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
template <>
__device__ inline double lane_bcast<double>(double v, int j) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// inclusive prefix sum over the 64 lanes of a wavefront
template <typename T>
__device__ inline T wave_scan_up(T v) {
    v = row_scan_up<T>(v);
    const T r0 = lane_bcast<T>(v, 15), r1 = lane_bcast<T>(v, 31), r2 = lane_bcast<T>(v, 47);
    const int row = (threadIdx.x & 63) >> 4;
    return v + (row > 0 ? r0 : (T)0) + (row > 1 ? r1 : (T)0) + (row > 2 ? r2 : (T)0);
}
// inclusive suffix sum over the 64 lanes of a wavefront
template <typename T>
__device__ inline T wave_scan_down(T v) {
    v = row_scan_down<T>(v);
    const T r1 = lane_bcast<T>(v, 16), r2 = lane_bcast<T>(v, 32), r3 = lane_bcast<T>(v, 48);
    const int row = (threadIdx.x & 63) >> 4;
    return v + (row < 1 ? r1 : (T)0) + (row < 2 ? r2 : (T)0) + (row < 3 ? r3 : (T)0);
}
// sum over the 64 lanes, in every lane
template <typename T>
__device__ inline T wave_total(T v) {
    return lane_bcast<T>(wave_scan_up<T>(v), 63);
}

struct Events {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Rollout launch shapes.  RF_RULE: the fixed rule (linear: the M-split form
// below 1024 tiles of 16 candidates, else one wavefront per tile and four
// per workgroup; chains: 256-thread workgroups).  Linear: RF_ONE1/2/4 one
// wavefront per tile, 1 / 2 / 4 per workgroup; RF_SPLIT the M-split form
// (more than 16 states); RF_VALU256 / RF_VALU64 one lane per candidate on the
// vector ALUs (n, m <= 16) in workgroups of 256 / 64.  Chains: RF_CH64 /
// RF_CH128 / RF_CH256 workgroup sizes.  All matrix-core forms give the same
// bits, and all chain forms; the VALU forms sum in another order.
enum RolloutForm {
    RF_RULE = 0, RF_ONE1 = 1, RF_ONE2 = 2, RF_ONE4 = 3, RF_SPLIT = 4, RF_VALU256 = 5,
    RF_VALU64 = 6, RF_FROWS = 7, RF_CH64 = 11, RF_CH128 = 12, RF_CH256 = 13
};

template <typename T>
hipError_t launch_rollout(const ProbView<T> &P, int model, const T *x0, const T *knots,
                          int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                          const Events &ev = Events(), int form = RF_RULE);

// Linear model only (defined per dtype in rollout_linear_f32.hip / _f64.hip).
template <typename T>
hipError_t launch_linear(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                         int64_t ld, T *cost, hipStream_t s, const Events &ev, int form);

// Warm-start and exploration variants of a population launch (empc_ga):
// shift the carried parents one control step later (parents read from
// elite_rows only), and the distance-dependent mutation noise (needs x0).
template <typename T>
struct PopVariant {
    const T *x0 = nullptr;  // state of the solve (for sigma_dist > 0)
    T sigma_min = 0, sigma_dist = 0;
    int shift = 0;
};
template <typename T>
inline PopVariant<T> pop_variant(const empc_ga &ga, const void *x0, bool shift_now) {
    PopVariant<T> v;
    v.x0 = (const T *)x0;
    v.sigma_min = (T)ga.sigma_min;
    v.sigma_dist = x0 ? (T)ga.sigma_dist : (T)0;
    v.shift = (ga.shift && shift_now) ? 1 : 0;
    return v;
}

// R_override: parameter groups of 16 per population workgroup (1, 2 or 4;
// 0 = the rule: 2 or 4 when the launch would have 2048 / 4096 or more
// workgroups).  Every choice gives the same bits.
template <typename T>
hipError_t launch_population(const ProbView<T> &P, const empc_ga &ga, const T *knots_in,
                             int64_t ld_in, const int64_t *elite_idx, const T *elite_rows,
                             const int *has_elites, int cold_mode, T *knots_out, int64_t ld_out,
                             uint32_t tick, uint32_t gen, hipStream_t s,
                             const PopVariant<T> &var = PopVariant<T>(), int R_override = 0);

// Selection writes elite indices (ascending), best index, and optionally the
// elite knots [pm][k] (parameter-major), elite costs [k], the warm-start flag, u* and the
// best cost.
template <typename T>
hipError_t launch_select(const ProbView<T> &P, const T *cost, const T *knots, int64_t ld,
                         int64_t pop, int k, int64_t *elite_idx, int64_t *best_idx, T *elite_rows,
                         T *elite_cost, int *has_elites, int *best_slot, T *u_star, T *best_cost,
                         hipStream_t s);

template <typename T>
hipError_t launch_gather_parents(const T *knots, int64_t ld, const int64_t *elite_idx, int k,
                                 int pm, T *E, hipStream_t s);
template <typename T>
hipError_t launch_finish_refine(const T *E, int k, int pm, int m, const T *ecost, T *elite_rows,
                                int *best_slot, T *u_star, T *best_cost, hipStream_t s);

template <typename T>
hipError_t launch_grad(const ProbView<T> &P, int model, const T *x0, const T *knots, int64_t ncand,
                       int64_t ld, T *dJ, T *cost, int refine_steps, T lr, T *knots_io,
                       T *cost_io, hipStream_t s);

// LDS bytes of the adjoint kernel; the kernel needs n <= 64 (linear) or
// d <= 64 (chain) and at most MAX_GRAD_LDS bytes.
size_t grad_smem_bytes(int model, int n, int m, int T, int p, size_t esize);
constexpr size_t MAX_GRAD_LDS = 160 * 1024;

template <typename T>
hipError_t launch_plant(const ProbView<T> &P, int model, const T *x, const T *u, const T *noise,
                        T *x_next, hipStream_t s);

// Parameterized small-matrix convex MPC (convex.hip)
size_t qp_workspace_bytes(int n, int T, int pm);
template <typename T>
hipError_t launch_qp_form(const ProbView<T> &P, const T *x0, void *ws, T *Pout, T *qout, T *cout,
                          hipStream_t s);
// the S, v part of the form's workspace (what launch_qp_form needs)
size_t qp_form_bytes(int n, int T, int pm);
constexpr int QP_REFINE_MAX_PM = 1024;  // parameters of the quadratic refinement
template <typename T>
hipError_t launch_qp_refine(const ProbView<T> &P, const T *Pm, const T *q, const T *c,
                            const T *knots, int64_t ld, const int64_t *idx, T *Z, int k,
                            int steps, T lr, T *cost_io, hipStream_t s);
template <typename T>
hipError_t launch_qp_solve(const ProbView<T> &P, const T *Pm, const T *q, const T *c, void *ws,
                           int max_iter, T *z, T *cost, int *info, hipStream_t s);

// N-link planar robot (nlink.hip): links per robot the library supports
constexpr int NLINK_MAX = 16;
template <typename T>
hipError_t launch_nlink_linearize(int N, const T *mass, const T *len, double b, double dt,
                                  const T *x, const T *u, T *Ad, T *Bd, T *wd, hipStream_t s);
template <typename T>
hipError_t launch_nlink_step(int N, const T *mass, const T *len, double b, double dt, int sub,
                             const T *x, const T *u, T *x_next, hipStream_t s);

}  // namespace empc
