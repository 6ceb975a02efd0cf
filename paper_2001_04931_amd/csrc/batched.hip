// Problem-batched EMPC tick (gfx950): many independent problems of different
// sizes advance one control tick together.  Per generation: one population
// launch over all problems, one rollout launch per kernel shape class (the
// problems whose state and input counts select the same register tiling),
// on up to four side streams, one selection launch over all problems; then
// one tiny launch advances the device tick counter, so the same launch
// sequence, captured once as a HIP graph, replays tick after tick.  A
// persistent work-queue form is below as well.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <vector>

#include "evolve_body.hpp"
#include "rollout_chain.hpp"
#include "rollout_linear.hpp"

namespace empc {

// One workgroup per (problem, population tile) that holds parameters: the
// map lists them problem after problem, so problems with fewer parameters
// take fewer workgroups (no workgroups that would only exit).
template <typename T>
__global__ __launch_bounds__(POP_THREADS) void batch_population(const BatchSlot<T> *__restrict__ slots,
                                                        const int2 *__restrict__ popmap,
                                                        int64_t pop, int k, int elitism, T sigma,
                                                        uint32_t seed_lo, int g,
                                                        const uint32_t *__restrict__ tick,
                                                        int shift, T sigma_min, T sigma_dist,
                                                        int R, unsigned *__restrict__ counters,
                                                        int ncounters) {
    // the persistent form's work-queue heads and completion counters start
    // every generation at zero (its kernels run after this one)
    if (counters && blockIdx.x == 0)
        for (int c = threadIdx.x; c < ncounters; c += blockDim.x) counters[c] = 0;
    const int2 e = popmap[blockIdx.x];  // (problem, tile within the problem)
    const BatchSlot<T> &S = slots[e.x];
    const ProbView<T> P = global_view(S.P);
    GaStreams gs;
    gs.k0 = seed_lo;
    gs.k1 = S.key_hi;
    gs.XB = 1 + (P.m + 127) / 128;
    gs.NB = gs.XB + (P.p * P.m + 127) / 128;
    const bool first = g == 0;
    const bool cold = first && *S.has_elites == 0;
    const int64_t nts = pop_tiles_s(pop);
    PopVariant<T> var;
    var.x0 = global_ptr(S.x0);
    var.sigma_min = sigma_min;
    var.sigma_dist = sigma_dist;
    var.shift = first ? shift : 0;
    population_tile<T>(P, gs, pop, k, elitism, sigma,
                       first ? nullptr : global_ptr(S.knots[(g + 1) & 1]), pop,
                       first ? nullptr : global_ptr(S.elite_idx),
                       first ? global_ptr(S.elite_rows) : nullptr, cold,
                       global_ptr(S.knots[g & 1]), pop, *tick, (uint32_t)g, e.y % nts,
                       (int)(e.y / nts), var, R);
}

template <typename T, int NT, int NU, int WPB, bool BOX>
__global__ __launch_bounds__(64 * WPB) void batch_roll_linear(const BatchSlot<T> *__restrict__ slots,
                                                              const int *__restrict__ items,
                                                              int64_t pop, int g) {
    const int64_t w = xcd_swizzle_2d();
    const BatchSlot<T> &S = slots[items[w / gridDim.x]];
    linear_tile<T, NT, NU, true, BOX>(global_view(S.P), global_ptr(S.x0),
                                      global_ptr(S.knots[g & 1]), pop, pop, global_ptr(S.cost),
                                      (w % gridDim.x) * WPB + (threadIdx.x >> 6));
}

// linear problems of at most 16 states and 16 inputs, the vector-ALU form:
// one lane per candidate, 64 per workgroup, through the single-problem VALU
// kernel's device body (so a problem rounds as its single solve in that form
// does)
template <int NM, int MM, bool BOX>
__global__ __launch_bounds__(64) void batch_roll_linear_valu(const BatchSlot<float> *__restrict__ slots,
                                                             const int *__restrict__ items,
                                                             int64_t pop, int g) {
    const BatchSlot<float> &S = slots[items[blockIdx.y]];
    valu_block<float, NM, MM, BOX, false>(global_view(S.P), global_ptr(S.x0),
                                          global_ptr(S.knots[g & 1]), pop, pop,
                                          global_ptr(S.cost), (int64_t)blockIdx.x * 64 + threadIdx.x);
}

// linear problems of more than 16 states: the M-split form, one workgroup
// of NT wavefronts per tile, as in the single-problem rollout
template <typename T, int NT, int NU, bool BOX>
__global__ __launch_bounds__(64 * NT) void batch_roll_linear_split(
    const BatchSlot<T> *__restrict__ slots, const int *__restrict__ items, int64_t pop, int g) {
    const int64_t w = xcd_swizzle_2d();
    const BatchSlot<T> &S = slots[items[w / gridDim.x]];
    linear_tile_split<T, NT, NU, true, BOX>(global_view(S.P), global_ptr(S.x0),
                                            global_ptr(S.knots[g & 1]), pop, pop,
                                            global_ptr(S.cost), w % gridDim.x);
}

template <typename T, int DMAX, bool BOX>
__global__ __launch_bounds__(256) void batch_roll_chain(const BatchSlot<T> *__restrict__ slots,
                                                        const int *__restrict__ items, int64_t pop,
                                                        int g) {
    __shared__ JointConst<T> jc[DMAX];
    const BatchSlot<T> &S = slots[items[blockIdx.y]];
    const ProbView<T> P = global_view(S.P);
    chain_constants_lds(P, jc);
    __syncthreads();
    const int64_t cand = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cand >= pop) return;
    chain_candidate<T, DMAX, BOX>(P, jc, global_ptr(S.x0), global_ptr(S.knots[g & 1]), pop,
                                  global_ptr(S.cost), cand);
}

// chains of more than 8 joints: one candidate per 16-lane row, as in the
// single-problem rollout (same arithmetic, same rounding); WPB wavefronts
// (4 WPB candidates) per workgroup
template <typename T, int J, int WPB, bool BOX>
__global__ __launch_bounds__(64 * WPB) void batch_roll_chain_rows(const BatchSlot<T> *__restrict__ slots,
                                                                  const int *__restrict__ items,
                                                                  int64_t pop, int g) {
    const int64_t w = xcd_swizzle_2d();
    const BatchSlot<T> &S = slots[items[w / gridDim.x]];
    const int64_t cand0 = (w % gridDim.x) * (4 * WPB);
    if (cand0 + (threadIdx.x >> 6) * 4 >= pop) return;  // whole wavefront past the end
    chain_row_candidate<T, J, BOX>(global_view(S.P), global_ptr(S.x0),
                                   global_ptr(S.knots[g & 1]), pop, pop, global_ptr(S.cost),
                                   cand0 + (threadIdx.x >> 4), threadIdx.x & 15);
}

// one workgroup per problem: problem items[blockIdx.x] (items NULL: blockIdx.x)
template <typename T, typename K, int CACHE>
__global__ __launch_bounds__(SEL_THREADS) void batch_select(const BatchSlot<T> *__restrict__ slots,
                                                            const int *__restrict__ items,
                                                            int64_t pop, int k, int g, int last) {
    const BatchSlot<T> &S = slots[items ? items[blockIdx.x] : (int)blockIdx.x];
    select_body<T, K, CACHE, SEL_THREADS>(
        global_ptr(S.cost), pop, k, global_ptr(S.knots[g & 1]), pop, S.P.p * S.P.m, S.P.m,
        global_ptr(S.elite_idx), global_ptr(S.best_idx), last ? global_ptr(S.elite_rows) : nullptr,
        global_ptr(S.elite_cost), global_ptr(S.has_elites), nullptr,
        last ? global_ptr(S.u_star) : nullptr, last ? global_ptr(S.best_cost) : nullptr);
}

__global__ void batch_tick_advance(uint32_t *tick) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *tick += 1;
}

// ---------------------------------------------------------------------------
// Persistent form: per register tier one kernel of one-wavefront workgroups
// that pull (problem, unit) items from a work queue (an atomic head); a unit
// is a 16-candidate tile (linear, MFMA), 16 candidates in four passes of four
// 16-lane rows (chains of more than 8 joints) or 64 candidates (chains of at
// most 8 joints, one per lane).  The wave that completes the last unit of a
// problem (an atomic count per problem) runs that problem's selection; the
// wave that completes the last selection of a tick's last generation
// advances the tick.  Nothing waits on anything: a wave only ever takes the
// next item or finds the queue empty and exits, so the grid always drains.
// The kernels of different tiers run concurrently on side streams; within a
// tier every problem uses the same compiled code paths, so the register
// allocation of a tier is that of its largest class, not of the whole batch.
// Tiers: 0 linear of more than 32 states, 1 linear of 17..32, 2 linear of at
// most 16, 3 pendulum chains.
// Counters (reset by the population kernel): head[4], probs_done, done[nprob].
constexpr int PTIERS = 4;
enum { PC_LIN = 0, PC_LANE = 1, PC_ROW = 2 };

struct PersistArgs {
    const BatchSlot<float> *slots;
    const int2 *items;       // (problem, unit), this tier's, heaviest first
    const int *units;        // per problem: its number of units
    const int *code;         // per problem: kind * 256 + shape (see pcode)
    unsigned *head;          // this tier's queue head
    unsigned *done;          // per problem: units completed
    unsigned *probs_done;    // selections completed (all tiers)
    uint32_t *tick;
    int nitems, nprob, k, g, last;
    int64_t pop;
};

__host__ __device__ inline int pcode(int kind, int a, int b) { return kind * 256 + a * 16 + b; }

template <int NT, int NU>
__device__ __forceinline__ void p_linear(const BatchSlot<float> &S, int64_t pop, int g, int unit) {
    linear_tile<float, NT, NU, true, false>(global_view(S.P), global_ptr(S.x0),
                                            global_ptr(S.knots[g & 1]), pop, pop,
                                            global_ptr(S.cost), unit);
}
template <int NT>
__device__ __forceinline__ bool p_linear_nu(int nu, const BatchSlot<float> &S, int64_t pop, int g,
                                            int unit) {
    switch (nu) {
        case 1: p_linear<NT, 1>(S, pop, g, unit); return true;
        case 2: p_linear<NT, 2>(S, pop, g, unit); return true;
        case 4: p_linear<NT, 4>(S, pop, g, unit); return true;
        case 6: p_linear<NT, 6>(S, pop, g, unit); return true;
        case 8: p_linear<NT, 8>(S, pop, g, unit); return true;
        case 10: p_linear<NT, 10>(S, pop, g, unit); return true;
    }
    return false;
}
template <int J>
__device__ __forceinline__ void p_rows(const BatchSlot<float> &S, int64_t pop, int g, int unit) {
    const int lane = threadIdx.x & 63;
    for (int pass = 0; pass < 4; ++pass) {
        const int64_t c0 = (int64_t)unit * 16 + pass * 4;
        if (c0 >= pop) break;  // wave-uniform
        chain_row_candidate<float, J, false>(global_view(S.P), global_ptr(S.x0),
                                             global_ptr(S.knots[g & 1]), pop, pop,
                                             global_ptr(S.cost), c0 + (lane >> 4), lane & 15);
    }
}
template <int DMAX>
__device__ __forceinline__ void p_lane(const BatchSlot<float> &S, JointConst<float> *jc,
                                       int64_t pop, int g, int unit) {
    __syncthreads();  // the previous item's readers of jc are done
    const ProbView<float> P = global_view(S.P);
    chain_constants_lds(P, jc);
    __syncthreads();
    const int64_t cand = (int64_t)unit * 64 + (threadIdx.x & 63);
    if (cand < pop)
        chain_candidate<float, DMAX, false>(P, jc, global_ptr(S.x0), global_ptr(S.knots[g & 1]),
                                            pop, global_ptr(S.cost), cand);
}

template <int TIER>
__device__ __forceinline__ void p_item(int code, const BatchSlot<float> &S, JointConst<float> *jc,
                                       int64_t pop, int g, int unit) {
    const int kind = code >> 8, a = (code >> 4) & 15, b = code & 15;
    if constexpr (TIER == 0) {
        if (a == 3) p_linear_nu<3>(b, S, pop, g, unit);
        else if (a == 4) p_linear_nu<4>(b, S, pop, g, unit);
        else p_linear_nu<5>(b, S, pop, g, unit);
    } else if constexpr (TIER == 1) {
        p_linear_nu<2>(b, S, pop, g, unit);
    } else if constexpr (TIER == 2) {
        p_linear_nu<1>(b, S, pop, g, unit);
    } else {
        if (kind == PC_LANE) {
            if (a == 4) p_lane<4>(S, jc, pop, g, unit);
            else p_lane<8>(S, jc, pop, g, unit);
        } else {
            if (a == 1) p_rows<1>(S, pop, g, unit);
            else if (a == 2) p_rows<2>(S, pop, g, unit);
            else p_rows<3>(S, pop, g, unit);
        }
    }
}

// waves per SIMD each tier's kernel is compiled for (bounds its registers):
// the register need of the tier's largest class decides
template <int TIER>
constexpr int persist_waves() { return TIER == 0 ? 1 : (TIER == 3 ? 3 : 2); }

template <int TIER>
__global__ __launch_bounds__(64, persist_waves<TIER>()) void batch_persist(PersistArgs A) {
    constexpr int CACHE = 16;  // keys per lane: populations of at most 1024
    __shared__ JointConst<float> jc[8];
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned it = 0;
        if (lane == 0) it = atomicAdd(A.head, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= (unsigned)A.nitems) break;
        const int2 e = A.items[it];
        const BatchSlot<float> &S = A.slots[e.x];
        p_item<TIER>(A.code[e.x], S, jc, A.pop, A.g, e.y);
        // publish this unit's costs, then count it; the wave that completes
        // a problem sees every other unit's costs after its acquire fence
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned prev = 0;
        if (lane == 0) prev = atomicAdd(&A.done[e.x], 1u);
        prev = __builtin_amdgcn_readfirstlane(__shfl(prev, 0, 64));
        if (prev + 1 != (unsigned)A.units[e.x]) continue;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        select_body<float, uint32_t, CACHE, 64, 1>(
            global_ptr(S.cost), A.pop, A.k, global_ptr(S.knots[A.g & 1]), A.pop, S.P.p * S.P.m,
            S.P.m, global_ptr(S.elite_idx), global_ptr(S.best_idx),
            A.last ? global_ptr(S.elite_rows) : nullptr, global_ptr(S.elite_cost),
            global_ptr(S.has_elites), nullptr, A.last ? global_ptr(S.u_star) : nullptr,
            A.last ? global_ptr(S.best_cost) : nullptr);
        if (A.last) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            unsigned pd = 0;
            if (lane == 0) pd = atomicAdd(A.probs_done, 1u);
            pd = __builtin_amdgcn_readfirstlane(__shfl(pd, 0, 64));
            if (pd + 1 == (unsigned)A.nprob && lane == 0) *A.tick += 1;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side.

struct BatchClass {
    int model;   // EMPC_LINEAR / EMPC_PENDULUM_CHAIN
    int a, b;    // linear: (NT, NU bucket); chain: (DMAX, 0)
    int box;     // the problems have a state box penalty
    int first;   // offset in the device item list
    int count;
    double work;  // cost estimate (rule-based, or measured by the autotuner)
    int stream;   // side stream its rollout runs on
    int variant;  // launch shape, one of class_variants()
    float tuned_us[4] = {-1, -1, -1, -1};  // autotuner: mean launch time per shape
    int vnm = 0;         // linear, NT = 1: the VALU form's padded state count
                         // shared by every problem of the class (0: none)
    int allow_valu = 0;  // the plan offers the VALU form (empc_batch_allow_valu)
};

// Launch shapes a class can use.  The matrix-core shapes of a class run the
// same per-candidate device code in the same order, so the choice among them
// changes the time, never a result; the VALU form sums the cost in another
// order, so it is offered only when the plan allows it.
//   linear:   0..2  one wavefront per tile, 4 / 2 / 1 wavefronts per
//                   workgroup; 3  the M-split form (NT > 1), or the VALU form
//                   with 64 threads (NT = 1, allowed and vnm > 0)
//   chain, lane per candidate (DMAX <= 8): 0..2  256 / 128 / 64 threads
//   chain, row per candidate:              0..2  4 / 2 / 1 wavefronts
int class_variants(const BatchClass &c) {
    if (c.model == EMPC_LINEAR) return (c.a > 1 || (c.allow_valu && c.vnm > 0)) ? 4 : 3;
    return 3;
}

// The rollouts of the kernel-shape classes are independent, so they run on
// side streams forked from and joined back into the caller's stream (in a
// captured graph: parallel branches); the GPU fills the tail of one class's
// launch with another's.  At most this many side streams (the box's hardware
// queues bound the useful number).
constexpr int BATCH_STREAMS = 4;

int nu_bucket(int m) {
    const int nu = (m + 3) / 4;
    if (nu <= 1) return 1;
    if (nu <= 2) return 2;
    if (nu <= 4) return 4;
    if (nu <= 6) return 6;
    if (nu <= 8) return 8;
    return 10;
}
// chain kernel classes: lane per candidate up to 8 joints, then a 16-lane
// row per candidate with 1, 2 or 3 joints per lane
int dmax_bucket(int d) {
    if (d <= 4) return 4;
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    return 48;
}

template <int NT, int NU, int WPB, bool BOX>
static void go_batch_linear_wpb(const BatchSlot<float> *slots, const int *items, int count,
                                int64_t pop, int g, hipStream_t s) {
    const int64_t tiles = (pop + 15) / 16;
    hipLaunchKernelGGL((batch_roll_linear<float, NT, NU, WPB, BOX>),
                       dim3((unsigned)((tiles + WPB - 1) / WPB), (unsigned)count), dim3(64 * WPB), 0,
                       s, slots, items, pop, g);
}
template <int NT, int NU, bool BOX>
static void go_batch_linear_box(int variant, const BatchSlot<float> *slots, const int *items,
                                int count, int64_t pop, int g, hipStream_t s) {
    if (NT > 1 && variant == 3) {
        hipLaunchKernelGGL((batch_roll_linear_split<float, NT, NU, BOX>),
                           dim3((unsigned)((pop + 15) / 16), (unsigned)count), dim3(64 * NT), 0, s,
                           slots, items, pop, g);
        return;
    }
    if (variant == 1) return go_batch_linear_wpb<NT, NU, 2, BOX>(slots, items, count, pop, g, s);
    if (variant == 2) return go_batch_linear_wpb<NT, NU, 1, BOX>(slots, items, count, pop, g, s);
    go_batch_linear_wpb<NT, NU, 4, BOX>(slots, items, count, pop, g, s);
}
template <int NT, int NU>
static void go_batch_linear(int box, int variant, const BatchSlot<float> *slots, const int *items,
                            int count, int64_t pop, int g, hipStream_t s) {
    if (box) return go_batch_linear_box<NT, NU, true>(variant, slots, items, count, pop, g, s);
    go_batch_linear_box<NT, NU, false>(variant, slots, items, count, pop, g, s);
}
template <int NM, int MM>
static void go_batch_valu_mm(int box, const BatchSlot<float> *slots, const int *items, int count,
                             int64_t pop, int g, hipStream_t s) {
    const dim3 grid((unsigned)((pop + 63) / 64), (unsigned)count);
    if (box)
        hipLaunchKernelGGL((batch_roll_linear_valu<NM, MM, true>), grid, dim3(64), 0, s, slots,
                           items, pop, g);
    else
        hipLaunchKernelGGL((batch_roll_linear_valu<NM, MM, false>), grid, dim3(64), 0, s, slots,
                           items, pop, g);
}
template <int NM>
static void go_batch_valu_nm(int nu, int box, const BatchSlot<float> *slots, const int *items,
                             int count, int64_t pop, int g, hipStream_t s) {
    // the input bucket of the class fixes the padded input count as the
    // single-problem launch picks it from m (at most 4, 8, 16)
    if (nu == 1) return go_batch_valu_mm<NM, 4>(box, slots, items, count, pop, g, s);
    if (nu == 2) return go_batch_valu_mm<NM, 8>(box, slots, items, count, pop, g, s);
    go_batch_valu_mm<NM, 16>(box, slots, items, count, pop, g, s);
}
static void go_batch_valu(const BatchClass &c, const BatchSlot<float> *slots, const int *items,
                          int64_t pop, int g, hipStream_t s) {
    if (c.vnm == 4) return go_batch_valu_nm<4>(c.b, c.box, slots, items, c.count, pop, g, s);
    if (c.vnm == 8) return go_batch_valu_nm<8>(c.b, c.box, slots, items, c.count, pop, g, s);
    go_batch_valu_nm<16>(c.b, c.box, slots, items, c.count, pop, g, s);
}
template <int NT>
static void go_batch_linear_nu(int nu, int box, int variant, const BatchSlot<float> *slots,
                               const int *items, int count, int64_t pop, int g, hipStream_t s) {
    switch (nu) {
        case 1: go_batch_linear<NT, 1>(box, variant, slots, items, count, pop, g, s); break;
        case 2: go_batch_linear<NT, 2>(box, variant, slots, items, count, pop, g, s); break;
        case 4: go_batch_linear<NT, 4>(box, variant, slots, items, count, pop, g, s); break;
        case 6: go_batch_linear<NT, 6>(box, variant, slots, items, count, pop, g, s); break;
        case 8: go_batch_linear<NT, 8>(box, variant, slots, items, count, pop, g, s); break;
        default: go_batch_linear<NT, 10>(box, variant, slots, items, count, pop, g, s); break;
    }
}
template <int J, int WPB, bool BOX>
static void go_batch_chain_rows_wpb(const BatchSlot<float> *slots, const int *items, int count,
                                    int64_t pop, int g, hipStream_t s) {
    hipLaunchKernelGGL((batch_roll_chain_rows<float, J, WPB, BOX>),
                       dim3((unsigned)((pop + 4 * WPB - 1) / (4 * WPB)), (unsigned)count),
                       dim3(64 * WPB), 0, s, slots, items, pop, g);
}
template <int J, bool BOX>
static void go_batch_chain_rows_box(int variant, const BatchSlot<float> *slots, const int *items,
                                    int count, int64_t pop, int g, hipStream_t s) {
    if (variant == 1) return go_batch_chain_rows_wpb<J, 2, BOX>(slots, items, count, pop, g, s);
    if (variant == 2) return go_batch_chain_rows_wpb<J, 1, BOX>(slots, items, count, pop, g, s);
    go_batch_chain_rows_wpb<J, 4, BOX>(slots, items, count, pop, g, s);
}
template <int J>
static void go_batch_chain_rows(int box, int variant, const BatchSlot<float> *slots,
                                const int *items, int count, int64_t pop, int g, hipStream_t s) {
    if (box) return go_batch_chain_rows_box<J, true>(variant, slots, items, count, pop, g, s);
    go_batch_chain_rows_box<J, false>(variant, slots, items, count, pop, g, s);
}
template <int DMAX, bool BOX>
static void go_batch_chain_box(int variant, const BatchSlot<float> *slots, const int *items,
                               int count, int64_t pop, int g, hipStream_t s) {
    const int threads = variant == 1 ? 128 : variant == 2 ? 64 : 256;
    hipLaunchKernelGGL((batch_roll_chain<float, DMAX, BOX>),
                       dim3((unsigned)((pop + threads - 1) / threads), (unsigned)count),
                       dim3(threads), 0, s, slots, items, pop, g);
}
template <int DMAX>
static void go_batch_chain(int box, int variant, const BatchSlot<float> *slots, const int *items,
                           int count, int64_t pop, int g, hipStream_t s) {
    if (box) return go_batch_chain_box<DMAX, true>(variant, slots, items, count, pop, g, s);
    go_batch_chain_box<DMAX, false>(variant, slots, items, count, pop, g, s);
}
// one class's rollout launch, in its chosen shape
static void launch_class(const BatchClass &c, int variant, const BatchSlot<float> *slots,
                         const int *d_items, int64_t pop, int g, hipStream_t s) {
    const int *items = d_items + c.first;
    if (c.model == EMPC_LINEAR) {
        if (c.a == 1 && variant == 3) return go_batch_valu(c, slots, items, pop, g, s);
        switch (c.a) {
            case 1: go_batch_linear_nu<1>(c.b, c.box, variant, slots, items, c.count, pop, g, s); break;
            case 2: go_batch_linear_nu<2>(c.b, c.box, variant, slots, items, c.count, pop, g, s); break;
            case 3: go_batch_linear_nu<3>(c.b, c.box, variant, slots, items, c.count, pop, g, s); break;
            case 4: go_batch_linear_nu<4>(c.b, c.box, variant, slots, items, c.count, pop, g, s); break;
            default: go_batch_linear_nu<5>(c.b, c.box, variant, slots, items, c.count, pop, g, s); break;
        }
        return;
    }
    switch (c.a) {
        case 4: go_batch_chain<4>(c.box, variant, slots, items, c.count, pop, g, s); break;
        case 8: go_batch_chain<8>(c.box, variant, slots, items, c.count, pop, g, s); break;
        case 16: go_batch_chain_rows<1>(c.box, variant, slots, items, c.count, pop, g, s); break;
        case 32: go_batch_chain_rows<2>(c.box, variant, slots, items, c.count, pop, g, s); break;
        default: go_batch_chain_rows<3>(c.box, variant, slots, items, c.count, pop, g, s); break;
    }
}

}  // namespace empc

using namespace empc;

struct empc_batch {
    int nprob = 0;
    empc_ga ga{};
    int64_t pop = 0;
    std::vector<BatchClass> classes;
    BatchSlot<float> *d_slots = nullptr;
    int2 *d_popmap = nullptr;  // population workgroups: (problem, tile)
    int64_t pop_wgs = 0;
    int pop_r = 1;  // parameter groups per population thread
    int *d_items = nullptr;
    uint32_t *d_tick = nullptr;
    int nstreams = 0;  // side streams in use (all BATCH_STREAMS are created)
    hipStream_t side[BATCH_STREAMS] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[BATCH_STREAMS] = {};
    // persistent form (mode 1)
    int mode = 0;
    bool persist_ok = false;       // every problem box-free
    int2 *d_pitems = nullptr;      // all tiers' items, tier after tier
    int *d_units = nullptr, *d_code = nullptr;
    unsigned *d_counters = nullptr;  // head[3], probs_done, done[nprob]
    int pfirst[PTIERS] = {}, pcount[PTIERS] = {}, pgrid[PTIERS] = {};
};

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Spread the classes over ns side streams: largest work first, each onto
// the least loaded stream.
void assign_streams(empc_batch *b, int ns) {
    b->nstreams = std::max(1, std::min<int>(ns, (int)b->classes.size()));
    std::vector<int> order(b->classes.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(),
              [&](int x, int y) { return b->classes[x].work > b->classes[y].work; });
    std::vector<double> load(b->nstreams, 0.0);
    for (int ci : order) {
        const int st = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->classes[ci].stream = st;
        load[st] += b->classes[ci].work;
    }
}

// The rollouts of one generation: fork the side streams from s, each class
// on its stream, join them back into s.
hipError_t rollout_phase(empc_batch *b, int g, hipStream_t s) {
    hipError_t e = hipEventRecord(b->fork, s);
    for (int i = 0; i < b->nstreams && e == hipSuccess; ++i)
        e = hipStreamWaitEvent(b->side[i], b->fork, 0);
    if (e != hipSuccess) return e;
    for (const BatchClass &c : b->classes)
        launch_class(c, c.variant, b->d_slots, b->d_items, b->pop, g, b->side[c.stream]);
    for (int i = 0; i < b->nstreams && e == hipSuccess; ++i) {
        e = hipEventRecord(b->join[i], b->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[i], 0);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

// selection launch over `count` problems (items NULL: problems 0..count-1)
void launch_batch_select(const empc_batch *b, const int *items, int count, int g, int last,
                         hipStream_t st) {
    const int64_t pop = b->pop, per = (pop + SEL_THREADS - 1) / SEL_THREADS;
    const int k = b->ga.n_elite;
    if (per <= 4)
        hipLaunchKernelGGL((batch_select<float, uint32_t, 4>), dim3(count), dim3(SEL_THREADS), 0, st,
                           b->d_slots, items, pop, k, g, last);
    else if (per <= 16)
        hipLaunchKernelGGL((batch_select<float, uint32_t, 16>), dim3(count), dim3(SEL_THREADS), 0,
                           st, b->d_slots, items, pop, k, g, last);
    else
        hipLaunchKernelGGL((batch_select<float, uint32_t, 0>), dim3(count), dim3(SEL_THREADS), 0, st,
                           b->d_slots, items, pop, k, g, last);
}

// One generation's rollouts and selections in the persistent form: the
// tiers' kernels on side streams forked from s and joined back into it.
hipError_t persist_phase(empc_batch *b, int g, int last, hipStream_t s) {
    hipError_t e = hipEventRecord(b->fork, s);
    int used = 0;
    for (int t = 0; t < PTIERS && e == hipSuccess; ++t) {
        if (!b->pcount[t]) continue;
        hipStream_t st = b->side[used];
        e = hipStreamWaitEvent(st, b->fork, 0);
        if (e != hipSuccess) break;
        PersistArgs A;
        A.slots = b->d_slots;
        A.items = b->d_pitems + b->pfirst[t];
        A.units = b->d_units;
        A.code = b->d_code;
        A.head = b->d_counters + t;
        A.probs_done = b->d_counters + PTIERS;
        A.done = b->d_counters + PTIERS + 1;
        A.tick = b->d_tick;
        A.nitems = b->pcount[t];
        A.nprob = b->nprob;
        A.k = b->ga.n_elite;
        A.g = g;
        A.last = last;
        A.pop = b->pop;
        const dim3 grid(b->pgrid[t]), block(64);
        void (*kern)(PersistArgs) =
            t == 0 ? batch_persist<0>
                   : (t == 1 ? batch_persist<1> : (t == 2 ? batch_persist<2> : batch_persist<3>));
        hipLaunchKernelGGL(kern, grid, block, 0, st, A);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(b->join[used], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[used], 0);
        ++used;
    }
    return e;
}

// Work items of the persistent form: tier, kind and units of every problem,
// items of a tier heaviest problem first; grids sized so that the tiers'
// kernels share the chip in proportion to their work.
hipError_t build_persistent(empc_batch *b, const empc_problem *probs) {
    const int nprob = b->nprob;
    const int64_t pop = b->pop;
    std::vector<int> units(nprob), code(nprob), tier(nprob);
    std::vector<double> wunit(nprob);
    b->persist_ok = pop <= 1024;  // the one-wavefront selection caches 16 keys per lane
    for (int i = 0; i < nprob; ++i) {
        const empc_problem &P = probs[i];
        if (P.qb) b->persist_ok = false;
        if (P.model == EMPC_LINEAR) {
            const int NT = (P.n + 15) / 16;
            code[i] = pcode(PC_LIN, NT, nu_bucket(P.m));
            tier[i] = NT >= 3 ? 0 : (NT == 2 ? 1 : 2);
            units[i] = (int)((pop + 15) / 16);
            wunit[i] = (double)P.T * NT * NT;
        } else if (P.m <= 8) {
            code[i] = pcode(PC_LANE, P.m <= 4 ? 4 : 8, 0);
            tier[i] = 3;
            units[i] = (int)((pop + 63) / 64);
            wunit[i] = (double)P.T * P.m;
        } else {
            code[i] = pcode(PC_ROW, (P.m + 15) / 16, 0);
            tier[i] = 3;
            units[i] = (int)((pop + 15) / 16);
            wunit[i] = (double)P.T * ((P.m + 15) / 16) * 4.0;
        }
    }
    std::vector<int2> items;
    double twork[PTIERS] = {0, 0, 0, 0}, total = 0;
    for (int t = 0; t < PTIERS; ++t) {
        std::vector<int> ps;
        for (int i = 0; i < nprob; ++i)
            if (tier[i] == t) ps.push_back(i);
        std::stable_sort(ps.begin(), ps.end(), [&](int x, int y) { return wunit[x] > wunit[y]; });
        b->pfirst[t] = (int)items.size();
        for (int i : ps) {
            for (int u = 0; u < units[i]; ++u) items.push_back(make_int2(i, u));
            twork[t] += wunit[i] * units[i];
        }
        b->pcount[t] = (int)items.size() - b->pfirst[t];
        total += twork[t];
    }
    int dev = 0, cus = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int occ[PTIERS] = {1, 1, 1, 1};
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], batch_persist<0>, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], batch_persist<1>, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[2], batch_persist<2>, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[3], batch_persist<3>, 64, 0);
    if (e != hipSuccess) return e;
    for (int t = 0; t < PTIERS; ++t) {
        const double share = total > 0 ? twork[t] / total : 0.0;
        int grid = (int)(share * cus * (occ[t] > 0 ? occ[t] : 1) + 0.5);
        grid = std::max(grid, 64);
        b->pgrid[t] = std::min(grid, std::max(b->pcount[t], 1));
    }
    const size_t ncounters = PTIERS + 1 + nprob;
    e = hipMalloc(&b->d_pitems, sizeof(int2) * std::max<size_t>(items.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_units, sizeof(int) * nprob);
    if (e == hipSuccess) e = hipMalloc(&b->d_code, sizeof(int) * nprob);
    if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(unsigned) * ncounters);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(b->d_pitems, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_units, units.data(), sizeof(int) * nprob, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_code, code.data(), sizeof(int) * nprob, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_counters, 0, sizeof(unsigned) * ncounters);
    return e;
}

// Per-problem workspace, after a 256-byte header holding the tick counter:
// flag (256 B), two populations [pm][pop], costs [pop], parent knots [pm][k],
// parent costs [k], parent indices [k], best index.
size_t slot_bytes(const empc_problem &P, const empc_ga &G) {
    const size_t pm = (size_t)P.p * P.m, pop = G.pop, k = G.n_elite;
    return 256 + 2 * al256(pm * pop * 4) + al256(pop * 4) + al256(k * pm * 4) + al256(k * 4) +
           al256(k * 8) + 256;
}

}  // namespace

// Validation shared with the single-problem entry points lives in capi.hip.
empc_status empc_validate_problem_internal(const empc_problem *P);
empc_status empc_validate_ga_internal(const empc_ga *G);
empc_status empc_fail_internal(empc_status s, const char *msg);

extern "C" {

size_t empc_batch_workspace_bytes(const empc_problem *probs, int32_t nprob, const empc_ga *ga) {
    if (!probs || nprob < 1 || empc_validate_ga_internal(ga)) return 0;
    size_t b = 256;
    for (int i = 0; i < nprob; ++i) {
        if (empc_validate_problem_internal(&probs[i]) || probs[i].dtype != EMPC_F32) return 0;
        b += slot_bytes(probs[i], *ga);
    }
    return b;
}

empc_status empc_batch_create(const empc_problem *probs, int32_t nprob, const empc_ga *ga,
                              void *workspace, size_t ws_bytes, const void *x0_packed,
                              void *u_star_packed, void *best_cost, empc_batch **out) {
    if (!out) return empc_fail_internal(EMPC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!probs || nprob < 1) return empc_fail_internal(EMPC_EINVAL, "need nprob >= 1 problems");
    empc_status st = empc_validate_ga_internal(ga);
    if (st) return st;
    for (int i = 0; i < nprob; ++i) {
        if ((st = empc_validate_problem_internal(&probs[i]))) return st;
        if (probs[i].dtype != EMPC_F32)
            return empc_fail_internal(EMPC_EUNSUPPORTED, "batched solves run in FP32");
        if (probs[i].Q || probs[i].R || probs[i].Qf || probs[i].q_min || probs[i].fric_c)
            return empc_fail_internal(EMPC_EUNSUPPORTED, "batched solves take diagonal weights, "
                                                         "no joint limits and no dry friction");
    }
    if (!x0_packed || !u_star_packed || !best_cost)
        return empc_fail_internal(EMPC_EINVAL, "x0_packed, u_star_packed and best_cost are required");
    const size_t need = empc_batch_workspace_bytes(probs, nprob, ga);
    if (!workspace || ws_bytes < need) return empc_fail_internal(EMPC_EWORKSPACE, "batch workspace too small");

    empc_batch *b = new empc_batch();
    b->nprob = nprob;
    b->ga = *ga;
    b->pop = ga->pop;
    std::vector<BatchSlot<float>> slots(nprob);
    char *base = (char *)workspace;
    size_t off = 256;
    const float *x0 = (const float *)x0_packed;
    float *us = (float *)u_star_packed;
    int64_t xo = 0, uo = 0;
    for (int i = 0; i < nprob; ++i) {
        const empc_problem &P = probs[i];
        const size_t pm = (size_t)P.p * P.m, pop = ga->pop, k = ga->n_elite;
        BatchSlot<float> &S = slots[i];
        S.P = view_of<float>(P);
        S.model = P.model;
        S.key_hi = (uint32_t)(ga->seed >> 32) ^ (uint32_t)i;
        S.x0 = x0 + xo;
        S.u_star = us + uo;
        S.best_cost = (float *)best_cost + i;
        xo += P.n;
        uo += P.m;
        S.has_elites = (int *)(base + off); off += 256;
        S.knots[0] = (float *)(base + off); off += al256(pm * pop * 4);
        S.knots[1] = (float *)(base + off); off += al256(pm * pop * 4);
        S.cost = (float *)(base + off); off += al256(pop * 4);
        S.elite_rows = (float *)(base + off); off += al256(k * pm * 4);
        S.elite_cost = (float *)(base + off); off += al256(k * 4);
        S.elite_idx = (int64_t *)(base + off); off += al256(k * 8);
        S.best_idx = (int64_t *)(base + off); off += 256;
    }
    // parameter groups per population thread, as in the single-problem
    // launch: 2 or 4 when the plan's population grid is large (the children's
    // shared draws are then taken by fewer workgroups; the same bits)
    int64_t wgs1 = 0;
    for (int i = 0; i < nprob; ++i) wgs1 += pop_tiles_s(ga->pop) * pop_tiles_g(probs[i].p * probs[i].m);
    b->pop_r = wgs1 >= 4096 ? 4 : wgs1 >= 2048 ? 2 : 1;
    int64_t total_wgs = 0;
    for (int i = 0; i < nprob; ++i)
        total_wgs += pop_tiles_s(ga->pop) * pop_tiles_g(probs[i].p * probs[i].m, b->pop_r);
    if (total_wgs > INT32_MAX) {
        delete b;
        return empc_fail_internal(EMPC_EUNSUPPORTED, "batch population grid above 2^31 workgroups");
    }
    b->pop_wgs = total_wgs;
    // group problems by kernel shape class
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < nprob; ++i) {
        const empc_problem &P = probs[i];
        if (P.model == EMPC_LINEAR)
            groups[std::make_tuple(0, (P.n + 15) / 16, nu_bucket(P.m), P.qb ? 1 : 0)].push_back(i);
        else
            groups[std::make_tuple(1, dmax_bucket(P.m), 0, P.qb ? 1 : 0)].push_back(i);
    }
    std::vector<int> items;
    for (auto &kv : groups) {
        BatchClass c;
        c.model = std::get<0>(kv.first) == 0 ? EMPC_LINEAR : EMPC_PENDULUM_CHAIN;
        c.a = std::get<1>(kv.first);
        c.b = std::get<2>(kv.first);
        c.box = std::get<3>(kv.first);
        c.first = (int)items.size();
        c.count = (int)kv.second.size();
        c.work = 0;
        if (c.model == EMPC_LINEAR && c.a == 1 && c.b <= 4) {
            // the VALU form's padded state count, as the single-problem
            // launch picks it from n; offered only if every problem shares it
            auto nm_of = [](int n) { return n <= 4 ? 4 : n <= 8 ? 8 : 16; };
            c.vnm = nm_of(probs[kv.second[0]].n);
            for (int i : kv.second)
                if (nm_of(probs[i].n) != c.vnm) c.vnm = 0;
        }
        for (int i : kv.second) {  // per candidate-step: MFMAs (linear), joints (chain)
            const empc_problem &P = probs[i];
            c.work += (double)P.T * (P.model == EMPC_LINEAR ? 4.0 * c.a * c.a * 8.0 : 3.0 * P.m);
        }
        // rule-based shape until the autotuner measures: the M-split form
        // while the class has fewer tiles than the chip has SIMDs
        c.variant = (c.model == EMPC_LINEAR && c.a > 1 &&
                     ((ga->pop + 15) / 16) * c.count < SPLIT_MAX_TILES) ? 3 : 0;
        items.insert(items.end(), kv.second.begin(), kv.second.end());
        b->classes.push_back(c);
    }
    std::vector<int2> popmap;
    popmap.reserve((size_t)total_wgs);
    for (int i = 0; i < nprob; ++i) {
        const int64_t wgs = pop_tiles_s(ga->pop) * pop_tiles_g(probs[i].p * probs[i].m, b->pop_r);
        for (int64_t t = 0; t < wgs; ++t) popmap.push_back(make_int2(i, (int)t));
    }
    assign_streams(b, BATCH_STREAMS);
    b->d_tick = (uint32_t *)base;
    hipError_t e = hipMalloc(&b->d_slots, sizeof(BatchSlot<float>) * nprob);
    if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(int) * items.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_popmap, sizeof(int2) * popmap.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_popmap, popmap.data(), sizeof(int2) * popmap.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_slots, slots.data(), sizeof(BatchSlot<float>) * nprob, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_items, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < BATCH_STREAMS && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = build_persistent(b, probs);
    if (e != hipSuccess) {
        (void)hipFree(b->d_slots);
        (void)hipFree(b->d_items);
        (void)hipFree(b->d_popmap);
        (void)hipFree(b->d_pitems);
        (void)hipFree(b->d_units);
        (void)hipFree(b->d_code);
        (void)hipFree(b->d_counters);
        for (int i = 0; i < BATCH_STREAMS; ++i) {
            if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
            if (b->join[i]) (void)hipEventDestroy(b->join[i]);
        }
        if (b->fork) (void)hipEventDestroy(b->fork);
        delete b;
        return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
    }
    *out = b;
    return EMPC_OK;
}

empc_status empc_solve_batched(empc_batch *b, void *stream) {
    if (!b) return empc_fail_internal(EMPC_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    const empc_ga &G = b->ga;
    const int64_t pop = b->pop;
    const uint32_t seed_lo = (uint32_t)G.seed;
    if (b->mode == 1) {
        const int ncounters = PTIERS + 1 + b->nprob;
        for (int g = 0; g < G.generations; ++g) {
            const int last = g == G.generations - 1;
            hipLaunchKernelGGL(batch_population<float>, dim3((unsigned)b->pop_wgs),
                               dim3(POP_THREADS), 0, s, b->d_slots, b->d_popmap, pop, G.n_elite,
                               G.elitism, (float)G.sigma, seed_lo, g, (const uint32_t *)b->d_tick,
                               G.shift, (float)G.sigma_min, (float)G.sigma_dist, b->pop_r,
                               b->d_counters, ncounters);
            const hipError_t fe = persist_phase(b, g, last, s);
            if (fe != hipSuccess) return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(fe));
        }
        return EMPC_OK;
    }
    for (int g = 0; g < G.generations; ++g) {
        hipLaunchKernelGGL(batch_population<float>, dim3((unsigned)b->pop_wgs), dim3(POP_THREADS), 0,
                           s, b->d_slots, b->d_popmap, pop, G.n_elite, G.elitism, (float)G.sigma,
                           seed_lo, g, (const uint32_t *)b->d_tick, G.shift, (float)G.sigma_min,
                           (float)G.sigma_dist, b->pop_r, (unsigned *)nullptr, 0);
        const hipError_t fe = rollout_phase(b, g, s);
        if (fe != hipSuccess) return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(fe));
        launch_batch_select(b, nullptr, b->nprob, g, g == G.generations - 1, s);
    }
    hipLaunchKernelGGL(batch_tick_advance, dim3(1), dim3(64), 0, s, b->d_tick);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
    return EMPC_OK;
}

empc_status empc_batch_autotune(empc_batch *b, int32_t reps, void *stream) {
    if (!b) return empc_fail_internal(EMPC_EINVAL, "batch is NULL");
    if (reps < 1) return empc_fail_internal(EMPC_EINVAL, "reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const empc_ga &G = b->ga;
    // a generation-0 population, so that the timed rollouts read defined
    // knots; the parents, costs kept across ticks and the tick counter are
    // left as they are
    hipLaunchKernelGGL(batch_population<float>, dim3((unsigned)b->pop_wgs), dim3(POP_THREADS), 0, s,
                       b->d_slots, b->d_popmap, b->pop, G.n_elite, G.elitism,
                       (float)G.sigma, (uint32_t)G.seed, 0, (const uint32_t *)b->d_tick, G.shift,
                       (float)G.sigma_min, (float)G.sigma_dist, b->pop_r, (unsigned *)nullptr, 0);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    // mean time of one launch sequence over `reps` back-to-back runs, after
    // one untimed run
    auto time_it = [&](auto &&enqueue) -> float {
        float ms = 0;
        if (e == hipSuccess) e = enqueue();
        if (e == hipSuccess) e = hipEventRecord(t0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue();
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        return ms / reps;
    };
    // each class alone: its fastest launch shape
    for (BatchClass &c : b->classes) {
        float best = 0;
        int best_v = c.variant;
        for (int v = 0; v < class_variants(c) && e == hipSuccess; ++v) {
            const float ms = time_it([&]() {
                launch_class(c, v, b->d_slots, b->d_items, b->pop, 0, s);
                return hipGetLastError();
            });
            c.tuned_us[v] = ms * 1e3f;
            if (v == 0 || ms < best) {
                best = ms;
                best_v = v;
            }
        }
        c.variant = best_v;
        c.work = best;
    }
    // then the number of side streams, with the classes spread by their
    // measured times
    int best_ns = 1;
    float best = 0;
    for (int ns = 1; ns <= std::min<int>(BATCH_STREAMS, (int)b->classes.size()) && e == hipSuccess;
         ++ns) {
        assign_streams(b, ns);
        const float ms = time_it([&]() { return rollout_phase(b, 0, s); });
        if (ns == 1 || ms < best) {
            best = ms;
            best_ns = ns;
        }
    }
    assign_streams(b, best_ns);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
    return EMPC_OK;
}

int32_t empc_batch_classes(const empc_batch *b) { return b ? (int32_t)b->classes.size() : 0; }

empc_status empc_batch_class_info(const empc_batch *b, int32_t cls, int32_t *info) {
    if (!b || !info || cls < 0 || cls >= (int32_t)b->classes.size())
        return empc_fail_internal(EMPC_EINVAL, "bad batch, class index or info pointer");
    const BatchClass &c = b->classes[cls];
    info[0] = c.model;
    info[1] = c.a;
    info[2] = c.b;
    info[3] = c.count;
    info[4] = c.variant;
    info[5] = class_variants(c);
    info[6] = c.stream;
    return EMPC_OK;
}

empc_status empc_batch_class_times(const empc_batch *b, int32_t cls, float *us) {
    if (!b || !us || cls < 0 || cls >= (int32_t)b->classes.size())
        return empc_fail_internal(EMPC_EINVAL, "bad batch, class index or output pointer");
    for (int v = 0; v < 4; ++v) us[v] = b->classes[cls].tuned_us[v];
    return EMPC_OK;
}

empc_status empc_batch_set_variant(empc_batch *b, int32_t cls, int32_t variant) {
    if (!b || cls < 0 || cls >= (int32_t)b->classes.size())
        return empc_fail_internal(EMPC_EINVAL, "bad batch or class index");
    BatchClass &c = b->classes[cls];
    if (variant < 0 || variant >= class_variants(c))
        return empc_fail_internal(EMPC_EINVAL, "no such launch shape for this class");
    c.variant = variant;
    return EMPC_OK;
}

empc_status empc_batch_destroy(empc_batch *b) {
    if (!b) return EMPC_OK;
    for (int i = 0; i < BATCH_STREAMS; ++i) {
        if (b->side[i]) (void)hipStreamSynchronize(b->side[i]);
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    (void)hipFree(b->d_slots);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_popmap);
    (void)hipFree(b->d_pitems);
    (void)hipFree(b->d_units);
    (void)hipFree(b->d_code);
    (void)hipFree(b->d_counters);
    delete b;
    return EMPC_OK;
}

empc_status empc_batch_allow_valu(empc_batch *b, int32_t allow) {
    if (!b) return empc_fail_internal(EMPC_EINVAL, "batch is NULL");
    for (BatchClass &c : b->classes) {
        c.allow_valu = allow ? 1 : 0;
        if (c.variant >= class_variants(c)) c.variant = 0;
    }
    return EMPC_OK;
}

empc_status empc_batch_set_mode(empc_batch *b, int32_t mode) {
    if (!b) return empc_fail_internal(EMPC_EINVAL, "batch is NULL");
    if (mode != 0 && mode != 1) return empc_fail_internal(EMPC_EINVAL, "mode must be 0 or 1");
    if (mode == 1 && !b->persist_ok)
        return empc_fail_internal(EMPC_EUNSUPPORTED,
                                  "the persistent form takes populations of at most 1024 and "
                                  "problems without the state box penalty");
    b->mode = mode;
    return EMPC_OK;
}

}  // extern "C"
