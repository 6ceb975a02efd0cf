// Linear-model rollout + cost kernel (gfx950 matrix cores), shared by the FP32
// and FP64 translation units.
//
// Linear model (eq. 2): the population-batched step X <- A_d X + B_d U + w_d
// is a dense contraction with M = n states, K = n + m, N = candidates, so it
// runs on the matrix cores: v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64,
// one wavefront per tile of 16 candidates.
//
// The accumulator of a 16x16x4 MFMA leaves lane l holding, in register v
// (v = 0..3), output row 4g + v (f32 instruction) or g + 4v (f64) of column
// l%16, g = l/16; the A operand takes row l%16 from lane l, the B operand row
// l/16 of column l%16.  State i of an M-tile is placed on output row i (f64)
// or on row 4 (i mod 4) + i div 4 (f32), i.e. the A operand of lane c holds
// the row of state c (f64) or of state (c div 4) + 4 (c mod 4) (f32), so that
// in both cases accumulator register v of lane group g holds state g + 4v.
// Accumulator register v of M-tile t, used as a B operand as it stands, then
// supplies the K slice of states {16t + g + 4v : g = 0..3}; the columns of
// A_d are taken in that K order (the contraction order is free), which
// chains the steps with no cross-lane data movement.  Slice v of the last
// M-tile holds states 16 (NT-1) + 4v .. + 3, so the slices past the last
// state are all padding and their MFMAs, which would only add zeros, are
// skipped (C2, n = 28: one of eight slices).  A_d, B_d live in registers as A
// operands (one value per lane per MFMA), the state lives in accumulators,
// and knot interpolation, the dynamics step and the cost are fused in one
// loop over the horizon.
#pragma once
#include <hip/hip_ext.h>
#include <math.h>

#include "internal.hpp"
#include "rollout_full.hpp"
#include "rollout_valu.hpp"

namespace empc {

// s_waitcnt operand for gfx9: vmcnt = 0, expcnt and lgkmcnt left at their
// maxima (no wait)
constexpr int VMCNT0 = 0x0F70;

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // state held by register v of lane group g, and the state whose row the
    // A operand of lane c (output row c) carries
    __device__ static constexpr int row(int g, int v) { return g + 4 * v; }
    __device__ static constexpr int mstate(int c) { return (c >> 2) + 4 * (c & 3); }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static constexpr int row(int g, int v) { return g + 4 * v; }
    __device__ static constexpr int mstate(int c) { return c; }
};

// NT = ceil(n / 16) M-tiles, NU = ceil(m / 4) input K-slices; HAS_XG: the
// problem has a state goal (else (x - g) is x itself).
//
// Work per step.  The input enters a step as B_d u_k + w_d with
// u_k = (1-c) U_a + c U_b (Sec. IV-C), so with V_j = B_d U_j + w_d computed
// once per knot j the step is x_{k+1} = A_d x_k + V_a + c (V_b - V_a): the
// accumulators start from that (NT fused multiply-adds of 4-vectors) and only
// the 4 NT^2 MFMAs of A_d x_k remain in the step.  The stage cost is summed
// per state row, S_i += (x_i - g_i)^2, and weighted by Q once at the end; the
// input cost of a segment is summed in closed form (u is affine in c there):
//   sum_k r (e0 + c_k du)^2 = r (n e0^2 + 2 e0 du sum c_k + du^2 sum c_k^2),
// with the two sums over c_k accumulated by the step loop (two VALU
// operations per step, off the MFMA chain).
// One wavefront: candidates 16*tile .. 16*tile+15 of one problem.
// BOX: the problem has a state box penalty (P.qb non-NULL); it is summed per
// state row like the stage cost, from the state at the start of each step,
// corrected for x_0 and completed with x_T at the end, and so is the count
// of steps outside the box that the step charge (P.sb) weighs.
template <typename T, int NT, int NU, bool HAS_XG, bool BOX = false>
__device__ __forceinline__ void linear_tile(const ProbView<T> &P, const T *__restrict__ x0,
                                            const T *__restrict__ knots, int64_t ld,
                                            int64_t ncand, T *__restrict__ cost, int64_t tile) {
    typedef typename Mfma<T>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int64_t cand0 = tile * 16;
    if (cand0 >= ncand) return;  // wave-uniform
    const int col = lane & 15, grp = lane >> 4;
    const int64_t cand = cand0 + col;
    const bool valid = cand < ncand;
    const int n = P.n, m = P.m;
    // K slices v >= live of the last M-tile hold only padding states
    const int live = (n - 16 * (NT - 1) + 3) / 4;

    // A operands.  aX[mt][4t+v]: A_d[16mt + M(col)][16t + R(grp, v)];
    // aU[mt][s]: B_d[16mt + M(col)][4s + grp]  (M = Mfma<T>::mstate, R = row).
    T aX[NT][4 * NT];
    T aU[NT][NU];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
        const int row = 16 * mt + Mfma<T>::mstate(col);
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
    // State, disturbance and goal in accumulator layout: row 16mt + R(grp, v).
    v4 X[NT], Wd[NT], Xg[NT];
    v4 Lo[BOX ? NT : 1], Hi[BOX ? NT : 1], Pn[BOX ? NT : 1], Cn[BOX ? NT : 1];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + Mfma<T>::row(grp, v);
            const bool in = row < n;
            X[mt][v] = in ? x0[row] : (T)0;
            Wd[mt][v] = (in && P.wd) ? P.wd[row] : (T)0;
            Xg[mt][v] = (in && HAS_XG && P.xg) ? P.xg[row] : (T)0;
            if (BOX) {  // padding rows: a box around their zero state
                Lo[mt][v] = in ? P.xlo[row] : (T)-1;
                Hi[mt][v] = in ? P.xhi[row] : (T)1;
                Pn[mt][v] = -box_pen(X[mt][v], Lo[mt][v], Hi[mt][v]);
                Cn[mt][v] = -box_out(X[mt][v], Lo[mt][v], Hi[mt][v]);
            }
        }

    // the model operands and the initial state are needed by the first
    // step: wait for them here, before any knot load is in flight, so that
    // no wait in the step loop has to drain the knot prefetches with them
    __builtin_amdgcn_s_waitcnt(VMCNT0);
    const int p = P.p, Tn = P.Tn;
    // Loads are unconditional and unmasked, so that each use waits only for
    // its own load: a padded input row (j >= m) reads the candidate's own
    // input m-1 (it meets zero B_d columns and zero R weights), a knot index
    // past the last reads the last knot (it only ever meets c = 0), and a lane
    // past the last candidate reads the last candidate (its cost is not
    // stored).  A candidate's values thus only reach its own cost.
    const int64_t cand_c = valid ? cand : ncand - 1;
    auto load_knot = [&](int kn_idx, T *dst) {
        const int kc = kn_idx < p ? kn_idx : p - 1;
#pragma unroll
        for (int s = 0; s < NU; ++s) {
            const int j = 4 * s + grp;
            dst[s] = knots[(int64_t)(kc * m + (j < m ? j : m - 1)) * ld + cand_c];
        }
    };
    // V = B_d U + w_d for one knot (input slices as B operands), even and
    // odd slices in two accumulator chains
    auto knot_response = [&](const T *U, v4 *V) {
        v4 V1[NT];
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
            V[mt] = Mfma<T>::op(aU[mt][0], U[0], Wd[mt]);
            if (NU > 1) V1[mt] = Mfma<T>::op(aU[mt][1 % NU], U[1 % NU], v4{0, 0, 0, 0});
        }
#pragma unroll
        for (int s = 2; s < NU; ++s)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) {
                if (s & 1)
                    V1[mt] = Mfma<T>::op(aU[mt][s], U[s], V1[mt]);
                else
                    V[mt] = Mfma<T>::op(aU[mt][s], U[s], V[mt]);
            }
        if (NU > 1)
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) V[mt] += V1[mt];
    };
    // Knot registers: four sets K0..K3 hold knots a..a+3 while segment a runs.
    // The segment loop is unrolled four ways with the sets' roles rotating in
    // the source, so that no register is copied: segment a refills the set it
    // used for knot a with knot a+4, which is first read three segments later.
    T K0[NU], K1[NU], K2[NU], K3[NU];
    load_knot(0, K0);
    load_knot(1, K1);
    load_knot(2, K2);
    load_knot(3, K3);
    T Rw[NU], Ug[NU];
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        const int j = 4 * s + grp;
        Rw[s] = j < m ? P.r[j] : (T)0;
        Ug[s] = (j < m && P.ug) ? P.ug[j] : (T)0;
    }
    v4 Va[NT], Vb[NT], dV[NT];
    knot_response(K0, Va);
    knot_response(p > 1 ? K1 : K0, Vb);

    const T inv_den = Tn > 1 ? (T)1 / (T)(Tn - 1) : (T)0;
    // per-row stage-cost sums; starting from -(x_0 - g)^2 cancels exactly the
    // term the first step adds for x_0, so that S sums x_1 .. x_T
    v4 S[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const T e = X[mt][v] - Xg[mt][v];
            S[mt][v] = -(e * e);
        }
    // input cost, input slice s summed into Ju[s mod NT] (the share of
    // M-tile s mod NT in the M-split form)
    T Ju[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) Ju[mt] = 0;
    int k = 0;
    // segment a: steps with idx1 = a, knots ua = U_a, ub = U_min(a+1, p-1)
    // (ub of the last segment is unused: c = 0 there); un = U_{a+2}
    auto segment = [&](int a, T *ua, T *ub, T *un) {
        // first step of segment a+1: ceil((a+1)(T-1)/(p-1))
        const int kend = (p == 1 || a == p - 1) ? Tn
                                                : ((a + 1) * (Tn - 1) + (p - 2)) / (p - 1);
        const int nseg = kend - k;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) dV[mt] = Vb[mt] - Va[mt];
        T C1 = 0, C2 = 0;  // sums of c and c^2 over the segment
        for (; k < kend; ++k) {
            const int rem = (p == 1 || Tn == 1) ? 0 : k * (p - 1) - a * (Tn - 1);
            const T c = (T)rem * inv_den;
            C1 += c;
            C2 += c * c;
            // two partial sums per M-tile (even / odd K slices): 2 NT
            // independent accumulator chains, issued round-robin, so that no
            // MFMA waits on the one just before it
            v4 acc[NT][2];
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) {
                acc[mt][0] = Va[mt] + c * dV[mt];
                acc[mt][1] = v4{0, 0, 0, 0};
            }
            // slot (i, v): for every M-tile mt the MFMA of K slice (t, v),
            // t = (mt + i) mod NT (the K order of the M-split form, so that
            // both forms round identically), then one row of the stage-cost
            // sums, so VALU and matrix work alternate
#pragma unroll
            for (int i = 0; i < NT; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
#pragma unroll
                    for (int mt = 0; mt < NT; ++mt) {
                        const int t = (mt + i) % NT;
                        if (t == NT - 1 && v >= live) continue;  // padding slice
                        acc[mt][v & 1] = Mfma<T>::op(aX[mt][4 * t + v], X[t][v], acc[mt][v & 1]);
                    }
                    const T e = HAS_XG ? X[i][v] - Xg[i][v] : X[i][v];
                    S[i][v] += e * e;
                    if (BOX) {
                        Pn[i][v] += box_pen(X[i][v], Lo[i][v], Hi[i][v]);
                        Cn[i][v] += box_out(X[i][v], Lo[i][v], Hi[i][v]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
            for (int mt = 0; mt < NT; ++mt) X[mt] = acc[mt][0] + acc[mt][1];
        }
        // input cost of the segment: u is affine in c on it, so
        //   sum_k r (e0 + c_k du)^2 = r (nseg e0^2 + 2 e0 du sum c_k + du^2 sum c_k^2)
#pragma unroll
        for (int s = 0; s < NU; ++s) {
            const T e0 = ua[s] - Ug[s];
            const T du = (a == p - 1) ? (T)0 : ub[s] - ua[s];
            Ju[s % NT] += Rw[s] * ((T)nseg * e0 * e0 + (T)2 * e0 * du * C1 + du * du * C2);
        }
        // next segment's second knot response, from knot a+2
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) Va[mt] = Vb[mt];
        knot_response(un, Vb);
        // the set of knot a is free: refill it with knot a+4
        load_knot(a + 4, ua);
    };
    for (int a = 0; a < p; a += 4) {
        segment(a, K0, K1, K2);
        if (a + 1 < p) segment(a + 1, K1, K2, K3);
        if (a + 2 < p) segment(a + 2, K2, K3, K0);
        if (a + 3 < p) segment(a + 3, K3, K0, K1);
    }
    // x_T: stage and terminal weights; weights applied to the row sums.
    // Per M-tile partial costs, reduced over the tile's rows and then summed
    // in tile order, as the M-split form does.
    T J = 0;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
        T Jm = Ju[mt];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + Mfma<T>::row(grp, v);
            const bool in = row < n;
            const T e = X[mt][v] - Xg[mt][v];
            const T q = in ? P.q[row] : (T)0;
            const T qf = (in && P.qf) ? P.qf[row] : (T)0;
            Jm += q * (S[mt][v] + e * e) + qf * e * e;
            if (BOX) {
                const T qb = in ? P.qb[row] : (T)0;
                Jm += qb * (Pn[mt][v] + box_pen(X[mt][v], Lo[mt][v], Hi[mt][v]));
                const T sb = (in && P.sb) ? P.sb[row] : (T)0;
                Jm += sb * (Cn[mt][v] + box_out(X[mt][v], Lo[mt][v], Hi[mt][v]));
            }
        }
        Jm += __shfl_xor(Jm, 16, 64);
        Jm += __shfl_xor(Jm, 32, 64);
        J = mt == 0 ? Jm : J + Jm;
    }
    if (grp == 0 && valid) cost[cand] = J;
}

template <typename T, int NT, int NU, int WPB, bool HAS_XG, bool BOX>
__global__ __launch_bounds__(64 * WPB) void roll_linear_mfma(ProbView<T> P,
                                                             const T *__restrict__ x0,
                                                             const T *__restrict__ knots,
                                                             int64_t ld, int64_t ncand,
                                                             T *__restrict__ cost) {
    linear_tile<T, NT, NU, HAS_XG, BOX>(P, x0, knots, ld, ncand, cost,
                                   xcd_swizzle(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// M-split form: one workgroup of NT wavefronts per tile of 16 candidates,
// wavefront w owning state rows 16w..16w+15 (M-tile w).  Each step a
// wavefront runs the 4 NT MFMAs of its own rows (instead of 4 NT^2) and
// publishes its new rows through LDS; the next step reads the other tiles
// back.  One LDS round trip and one barrier per step, hidden behind the four
// MFMAs of the wavefront's own K slices, which need no exchanged data: the
// new rows are written as soon as they are summed, the first two own MFMAs
// of the next step cover the write, the barrier follows them, and the last
// two cover the read (placing the barrier before all four, or after them,
// measured 8 % slower per launch).
// A tile thus runs on NT SIMDs instead of one, which is what a population of
// a few thousand candidates needs to occupy the chip.
//
// Registers are indexed by slot i = 0..NT-1 holding M-tile (w + i) mod NT, so
// slot 0 is always the wavefront's own tile and every register index stays a
// compile-time constant; A_d's columns are loaded in the same rotated order.
__device__ inline void lds_barrier() {
    // orders LDS accesses only: outstanding global loads (knot prefetches)
    // are not waited for
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One workgroup of 64 NT threads: candidates 16*tile .. 16*tile+15 (tile
// must hold at least one candidate: the whole workgroup takes part in every
// barrier).
template <typename T, int NT, int NU, bool HAS_XG, bool BOX = false>
__device__ __forceinline__ void linear_tile_split(const ProbView<T> &P, const T *__restrict__ x0,
                                                  const T *__restrict__ knots, int64_t ld,
                                                  int64_t ncand, T *__restrict__ cost,
                                                  int64_t tile) {
    typedef typename Mfma<T>::v4 v4;
    __shared__ v4 xs[2][NT][64];
    __shared__ T part[NT][16];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t cand0 = tile * 16;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t cand = cand0 + col;
    const bool valid = cand < ncand;
    const int n = P.n, m = P.m;
    const int row_own = 16 * w + Mfma<T>::mstate(col);  // state of this lane's A-operand row
    const int live = (n - 16 * (NT - 1) + 3) / 4;      // live K slices of the last M-tile

    // aX[4i+v] = A_d[16w + col][16 t_i + R(grp, v)], t_i = (w + i) mod NT
    T aX[4 * NT];
    T aU[NU];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int t = (w + i) % NT;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = 16 * t + Mfma<T>::row(grp, v);
            aX[4 * i + v] = (row_own < n && kk < n) ? P.Ad[row_own * n + kk] : (T)0;
        }
    }
#pragma unroll
    for (int s2 = 0; s2 < NU; ++s2) {
        const int j = 4 * s2 + grp;
        aU[s2] = (row_own < n && j < m) ? P.Bd[row_own * m + j] : (T)0;
    }
    // state of every tile by slot; disturbance and goal of the own tile
    v4 X[NT], Wd, Xg;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int t = (w + i) % NT;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * t + Mfma<T>::row(grp, v);
            X[i][v] = row < n ? x0[row] : (T)0;
        }
    }
    v4 Lo, Hi, Pn, Cn;  // state box penalty and step charge of the own rows (BOX)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 16 * w + Mfma<T>::row(grp, v);
        const bool in = row < n;
        Wd[v] = (in && P.wd) ? P.wd[row] : (T)0;
        Xg[v] = (in && HAS_XG && P.xg) ? P.xg[row] : (T)0;
        if (BOX) {  // padding rows: a box around their zero state
            Lo[v] = in ? P.xlo[row] : (T)-1;
            Hi[v] = in ? P.xhi[row] : (T)1;
            Pn[v] = -box_pen(X[0][v], Lo[v], Hi[v]);
            Cn[v] = -box_out(X[0][v], Lo[v], Hi[v]);
        }
    }

    // the model operands and the initial state are needed by the first
    // step: wait for them here, before any knot load is in flight, so that
    // no wait in the step loop has to drain the knot prefetches with them
    __builtin_amdgcn_s_waitcnt(VMCNT0);
    const int p = P.p, Tn = P.Tn;
    // unconditional clamped loads, as in the one-wavefront form
    const int64_t cand_c = valid ? cand : ncand - 1;
    auto load_knot = [&](int kn_idx, T *dst) {
        const int kc = kn_idx < p ? kn_idx : p - 1;
#pragma unroll
        for (int s2 = 0; s2 < NU; ++s2) {
            const int j = 4 * s2 + grp;
            dst[s2] = knots[(int64_t)(kc * m + (j < m ? j : m - 1)) * ld + cand_c];
        }
    };
    // own rows of V = B_d U + w_d, even and odd slices in two chains
    auto knot_response = [&](const T *U) -> v4 {
        v4 V = Mfma<T>::op(aU[0], U[0], Wd);
        if (NU == 1) return V;
        v4 V1 = Mfma<T>::op(aU[1 % NU], U[1 % NU], v4{0, 0, 0, 0});
#pragma unroll
        for (int s2 = 2; s2 < NU; ++s2) {
            if (s2 & 1)
                V1 = Mfma<T>::op(aU[s2], U[s2], V1);
            else
                V = Mfma<T>::op(aU[s2], U[s2], V);
        }
        return V + V1;
    };
    T K0[NU], K1[NU], K2[NU], K3[NU];
    load_knot(0, K0);
    load_knot(1, K1);
    load_knot(2, K2);
    load_knot(3, K3);
    T Rw[NU], Ug[NU];
#pragma unroll
    for (int s2 = 0; s2 < NU; ++s2) {
        const int j = 4 * s2 + grp;
        Rw[s2] = j < m ? P.r[j] : (T)0;
        Ug[s2] = (j < m && P.ug) ? P.ug[j] : (T)0;
    }
    v4 Va = knot_response(K0);
    v4 Vb = knot_response(p > 1 ? K1 : K0);
    v4 dV;

    const T inv_den = Tn > 1 ? (T)1 / (T)(Tn - 1) : (T)0;
    v4 S;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const T e = X[0][v] - Xg[v];
        S[v] = -(e * e);
    }
    T Ju = 0;
    int k = 0, buf = 0;
    if (NT > 1) xs[0][w][lane] = X[0];  // read back by the first step
    auto segment = [&](int a, T *ua, T *ub, T *un) {
        const int kend = (p == 1 || a == p - 1) ? Tn
                                                : ((a + 1) * (Tn - 1) + (p - 2)) / (p - 1);
        const int nseg = kend - k;
        dV = Vb - Va;
        T C1 = 0, C2 = 0;  // sums of c and c^2 over the segment
        for (; k < kend; ++k) {
            const int rem = (p == 1 || Tn == 1) ? 0 : k * (p - 1) - a * (Tn - 1);
            const T c = (T)rem * inv_den;
            C1 += c;
            C2 += c * c;
            v4 acc0 = Va + c * dV, acc1 = v4{0, 0, 0, 0};
            // own K slices first (no exchanged data), with the stage cost of
            // the own rows between them and the exchange of the previous
            // step's rows after the second; then the other tiles' slices
#pragma unroll
            for (int i = 0; i < NT; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (NT > 1 && i == 0 && v == 2) {
                        lds_barrier();
#pragma unroll
                        for (int i2 = 1; i2 < NT; ++i2) X[i2] = xs[buf][(w + i2) % NT][lane];
                        buf ^= 1;
                    }
                    const bool pad = (w + i) % NT == NT - 1 && v >= live;
                    if (pad) {
                        // padding slice: its products are zero
                    } else if (v & 1) {
                        acc1 = Mfma<T>::op(aX[4 * i + v], X[i][v], acc1);
                    } else {
                        acc0 = Mfma<T>::op(aX[4 * i + v], X[i][v], acc0);
                    }
                    if (i == 0) {
                        const T e = HAS_XG ? X[0][v] - Xg[v] : X[0][v];
                        S[v] += e * e;
                        if (BOX) {
                            Pn[v] += box_pen(X[0][v], Lo[v], Hi[v]);
                            Cn[v] += box_out(X[0][v], Lo[v], Hi[v]);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            X[0] = acc0 + acc1;
            // buffer buf was last read in the previous step, before every
            // wavefront passed this step's barrier
            if (NT > 1) xs[buf][w][lane] = X[0];
        }
        // input cost of the segment in closed form (u is affine in c on
        // it); the input slices are shared out over the wavefronts
#pragma unroll
        for (int s2 = 0; s2 < NU; ++s2) {
            if (s2 % NT != w) continue;
            const T e0 = ua[s2] - Ug[s2];
            const T du = (a == p - 1) ? (T)0 : ub[s2] - ua[s2];
            Ju += Rw[s2] * ((T)nseg * e0 * e0 + (T)2 * e0 * du * C1 + du * du * C2);
        }
        Va = Vb;
        Vb = knot_response(un);
        load_knot(a + 4, ua);
    };
    for (int a = 0; a < p; a += 4) {
        segment(a, K0, K1, K2);
        if (a + 1 < p) segment(a + 1, K1, K2, K3);
        if (a + 2 < p) segment(a + 2, K2, K3, K0);
        if (a + 3 < p) segment(a + 3, K3, K0, K1);
    }
    T J = Ju;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 16 * w + Mfma<T>::row(grp, v);
        const bool in = row < n;
        const T e = X[0][v] - Xg[v];
        const T q = in ? P.q[row] : (T)0;
        const T qf = (in && P.qf) ? P.qf[row] : (T)0;
        J += q * (S[v] + e * e) + qf * e * e;
        if (BOX) {
            const T qb = in ? P.qb[row] : (T)0;
            J += qb * (Pn[v] + box_pen(X[0][v], Lo[v], Hi[v]));
            const T sb = (in && P.sb) ? P.sb[row] : (T)0;
            J += sb * (Cn[v] + box_out(X[0][v], Lo[v], Hi[v]));
        }
    }
    J += __shfl_xor(J, 16, 64);
    J += __shfl_xor(J, 32, 64);
    if (NT == 1) {
        if (grp == 0 && valid) cost[cand] = J;
        return;
    }
    if (lane < 16) part[w][lane] = J;
    lds_barrier();
    if (w == 0 && lane < 16 && valid) {
        T tot = part[0][lane];
#pragma unroll
        for (int i = 1; i < NT; ++i) tot += part[i][lane];
        cost[cand] = tot;
    }
}

template <typename T, int NT, int NU, bool HAS_XG, bool BOX>
__global__ __launch_bounds__(64 * NT) void roll_linear_split(ProbView<T> P,
                                                             const T *__restrict__ x0,
                                                             const T *__restrict__ knots,
                                                             int64_t ld, int64_t ncand,
                                                             T *__restrict__ cost) {
    linear_tile_split<T, NT, NU, HAS_XG, BOX>(P, x0, knots, ld, ncand, cost,
                                              xcd_swizzle(blockIdx.x, gridDim.x));
}

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

// The M-split form (NT wavefronts per tile) when the one-wavefront form
// would leave SIMDs idle: fewer tiles than the chip's 1024 SIMDs.  The two
// forms round identically, so the choice never changes a result.
constexpr int64_t SPLIT_MAX_TILES = 1024;

template <typename T, int NM, int MM, bool BOX, bool FULL = false>
static hipError_t go_valu_box(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                              int64_t ld, T *cost, hipStream_t s, const Events &ev, int threads) {
    return launch_timed(roll_linear_valu<T, NM, MM, BOX, FULL>,
                        dim3((unsigned)((ncand + threads - 1) / threads)), dim3(threads), 0, s, ev,
                        P, x0, knots, ld, ncand, cost);
}
template <typename T, int NM, bool BOX>
static hipError_t go_valu_m(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                            int64_t ld, T *cost, hipStream_t s, const Events &ev, int threads) {
    if (P.m <= 4) return go_valu_box<T, NM, 4, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    if (P.m <= 8) return go_valu_box<T, NM, 8, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    return go_valu_box<T, NM, 16, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
}
template <typename T, bool BOX>
static hipError_t go_valu(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                          int64_t ld, T *cost, hipStream_t s, const Events &ev, int threads) {
    if (P.n <= 4) return go_valu_m<T, 4, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    if (P.n <= 8) return go_valu_m<T, 8, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    return go_valu_m<T, 16, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
}

// full weights (n, m <= 16): the VALU form with the matrices in LDS
template <typename T, int NM, bool BOX>
static hipError_t go_valu_full_m(const ProbView<T> &P, const T *x0, const T *knots,
                                 int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                 const Events &ev, int threads) {
    if (P.m <= 4)
        return go_valu_box<T, NM, 4, BOX, true>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    if (P.m <= 8)
        return go_valu_box<T, NM, 8, BOX, true>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    return go_valu_box<T, NM, 16, BOX, true>(P, x0, knots, ncand, ld, cost, s, ev, threads);
}
template <typename T, bool BOX>
static hipError_t go_valu_full_n(const ProbView<T> &P, const T *x0, const T *knots,
                                 int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                 const Events &ev, int threads) {
    if (P.n <= 4) return go_valu_full_m<T, 4, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    if (P.n <= 8) return go_valu_full_m<T, 8, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    return go_valu_full_m<T, 16, BOX>(P, x0, knots, ncand, ld, cost, s, ev, threads);
}
template <typename T, int J, int JM, bool BOX>
static hipError_t go_full_rows_box(const ProbView<T> &P, const T *x0, const T *knots,
                                   int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                   const Events &ev) {
    const size_t bytes = (size_t)full_rows_lds(P.n, P.m, J).total * sizeof(T);
    auto kernel = roll_linear_full_rows<T, J, JM, BOX>;
    if (bytes > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void *)kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)bytes);
        if (e != hipSuccess) return e;
    }
    return launch_timed(kernel, dim3((unsigned)((ncand + 15) / 16)), dim3(256), bytes, s, ev, P,
                        x0, knots, ld, ncand, cost);
}
template <typename T, int J, bool BOX>
static hipError_t go_full_rows_m(const ProbView<T> &P, const T *x0, const T *knots,
                                 int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                 const Events &ev) {
    if (P.m <= 16) return go_full_rows_box<T, J, 1, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
    return go_full_rows_box<T, J, 2, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
}
template <typename T, bool BOX>
static hipError_t go_full_rows(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                               int64_t ld, T *cost, hipStream_t s, const Events &ev) {
    const int J = (P.n + 15) / 16;
    if (J <= 1) return go_full_rows_m<T, 1, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
    if (J <= 2) return go_full_rows_m<T, 2, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
    if (J <= 3) return go_full_rows_m<T, 3, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
    return go_full_rows_m<T, 4, BOX>(P, x0, knots, ncand, ld, cost, s, ev);
}

// Full weights: the 16-lane row form (n <= 64, m <= 32) unless the VALU form
// (one lane per candidate, n, m <= 16) was chosen.
template <typename T>
static hipError_t go_valu_full(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                               int64_t ld, T *cost, hipStream_t s, const Events &ev, int form) {
    const bool valu = (form == RF_VALU64 || form == RF_VALU256) && P.n <= 16 && P.m <= 16;
    if (!valu) {
        if (P.qb) return go_full_rows<T, true>(P, x0, knots, ncand, ld, cost, s, ev);
        return go_full_rows<T, false>(P, x0, knots, ncand, ld, cost, s, ev);
    }
    const int threads = form == RF_VALU64 ? 64 : 256;
    if (P.qb) return go_valu_full_n<T, true>(P, x0, knots, ncand, ld, cost, s, ev, threads);
    return go_valu_full_n<T, false>(P, x0, knots, ncand, ld, cost, s, ev, threads);
}

// form: one of RolloutForm (internal.hpp); RF_RULE takes the M-split form
// below SPLIT_MAX_TILES tiles, else one wavefront per tile, four per
// workgroup.  Every matrix-core form rounds identically; the VALU forms
// (n, m <= 16 only) round differently.
template <typename T, int NT, int NU, bool HAS_XG, bool BOX>
static hipError_t go_linear_forms(const ProbView<T> &P, const T *x0, const T *knots,
                                  int64_t ncand, int64_t ld, T *cost, hipStream_t s,
                                  const Events &ev, int form) {
    const int64_t tiles = (ncand + 15) / 16;
    if ((form == RF_VALU256 || form == RF_VALU64) && P.n <= VALU_MAX && P.m <= VALU_MAX)
        return go_valu<T, BOX>(P, x0, knots, ncand, ld, cost, s, ev,
                               form == RF_VALU256 ? 256 : 64);
    if ((form == RF_RULE && NT > 1 && tiles < SPLIT_MAX_TILES) || (form == RF_SPLIT && NT > 1))
        return launch_timed(roll_linear_split<T, NT, NU, HAS_XG, BOX>, dim3((unsigned)tiles),
                            dim3(64 * NT), 0, s, ev, P, x0, knots, ld, ncand, cost);
    if (form == RF_ONE1)
        return launch_timed(roll_linear_mfma<T, NT, NU, 1, HAS_XG, BOX>, dim3((unsigned)tiles),
                            dim3(64), 0, s, ev, P, x0, knots, ld, ncand, cost);
    if (form == RF_ONE2)
        return launch_timed(roll_linear_mfma<T, NT, NU, 2, HAS_XG, BOX>,
                            dim3((unsigned)((tiles + 1) / 2)), dim3(128), 0, s, ev, P, x0, knots,
                            ld, ncand, cost);
    return launch_timed(roll_linear_mfma<T, NT, NU, 4, HAS_XG, BOX>,
                        dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, ev, P, x0, knots, ld,
                        ncand, cost);
}

// goal and state box variants: (no goal, no box), (goal, no box), (box, with
// or without a goal: a NULL goal reads as 0)
template <typename T, int NT, int NU>
static hipError_t go_linear(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                            int64_t ld, T *cost, hipStream_t s, const Events &ev, int form) {
    if (P.qb)
        return go_linear_forms<T, NT, NU, true, true>(P, x0, knots, ncand, ld, cost, s, ev, form);
    if (P.xg)
        return go_linear_forms<T, NT, NU, true, false>(P, x0, knots, ncand, ld, cost, s, ev, form);
    return go_linear_forms<T, NT, NU, false, false>(P, x0, knots, ncand, ld, cost, s, ev, form);
}

template <typename T, int NT>
static hipError_t go_linear_nu(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                               int64_t ld, T *cost, hipStream_t s, const Events &ev, int form) {
    const int nu = (P.m + 3) / 4;
    if (nu <= 1) return go_linear<T, NT, 1>(P, x0, knots, ncand, ld, cost, s, ev, form);
    if (nu <= 2) return go_linear<T, NT, 2>(P, x0, knots, ncand, ld, cost, s, ev, form);
    if (nu <= 4) return go_linear<T, NT, 4>(P, x0, knots, ncand, ld, cost, s, ev, form);
    if (nu <= 6) return go_linear<T, NT, 6>(P, x0, knots, ncand, ld, cost, s, ev, form);
    if (nu <= 8) return go_linear<T, NT, 8>(P, x0, knots, ncand, ld, cost, s, ev, form);
    return go_linear<T, NT, 10>(P, x0, knots, ncand, ld, cost, s, ev, form);
}

template <typename T>
hipError_t launch_linear(const ProbView<T> &P, const T *x0, const T *knots, int64_t ncand,
                         int64_t ld, T *cost, hipStream_t s, const Events &ev, int form) {
    if (full_weights(P)) return go_valu_full<T>(P, x0, knots, ncand, ld, cost, s, ev, form);
    const int nt = (P.n + 15) / 16;
    switch (nt) {
        case 1: return go_linear_nu<T, 1>(P, x0, knots, ncand, ld, cost, s, ev, form);
        case 2: return go_linear_nu<T, 2>(P, x0, knots, ncand, ld, cost, s, ev, form);
        case 3: return go_linear_nu<T, 3>(P, x0, knots, ncand, ld, cost, s, ev, form);
        case 4: return go_linear_nu<T, 4>(P, x0, knots, ncand, ld, cost, s, ev, form);
        default: return go_linear_nu<T, 5>(P, x0, knots, ncand, ld, cost, s, ev, form);
    }
}

}  // namespace empc
