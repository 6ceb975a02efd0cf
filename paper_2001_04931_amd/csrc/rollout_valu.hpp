// Linear-model rollout + cost on the vector ALUs, one lane per candidate
// (gfx950), for small models (n, m <= 16).
//
// A 16 x 16 matrix-core tile wastes most of its rows and K slices on a model
// of a few states (n = 4: three quarters of both), and a population of a few
// hundred candidates gives the one-wavefront MFMA form only a handful of
// wavefronts, each a chain of dependent MFMAs per step.  Here every lane
// carries one candidate's state in registers and steps it on its own
// (eq. 2, x <- A_d x + B_d u + w_d), with A_d, B_d and the weights in LDS:
// every lane of a wavefront reads the same address (a broadcast), so the
// step is n (n + m) independent FMAs per lane, the n rows giving n-way
// instruction-level parallelism.  Knots are read coalesced (candidate
// innermost) once per knot segment.  The cost is summed step by step; its
// rounding differs from the matrix-core form's (a different summation
// order), which is why the single-problem autotuner may pick this form only
// as an explicit, recorded choice.
//
// FULL: full symmetric weights Q, R, Qf (eq. 3 in general form); each stage
// adds e^T Q e + e_u^T R e_u, the end e_T^T Qf e_T, from the matrices in LDS
// (a diagonal given as a vector is expanded there).  Problems with full
// weights run this form (n, m <= 16) when the tuner picks it, else the
// 16-lane row form of rollout_full.hpp.
#pragma once
#include <math.h>

#include "internal.hpp"

namespace empc {

constexpr int VALU_MAX = 16;  // largest n and m of the VALU form (diagonal weights)

// e^T W e for W (D x D, row-major in LDS) and e in registers
template <typename T, int D>
__device__ __forceinline__ T quad_lds(const T *W, const T *e) {
    T J = 0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T y = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) y += W[r * D + c] * e[c];
        J += e[r] * y;
    }
    return J;
}

template <typename T, int NM, int MM, bool BOX, bool FULL>
__device__ __forceinline__ void valu_candidate(const ProbView<T> &P, const T *sA, const T *sB,
                                               const T *sw, const T *sq, const T *sqf,
                                               const T *sxg, const T *sr, const T *sug,
                                               const T *slo, const T *shi, const T *sqb,
                                               const T *ssb, const T *sQ, const T *sR,
                                               const T *sQf, const T *__restrict__ x0,
                                               const T *__restrict__ knots, int64_t ld,
                                               T *__restrict__ cost, int64_t cand) {
    const int m = P.m, p = P.p, Tn = P.Tn;
    T x[NM];
#pragma unroll
    for (int r = 0; r < NM; ++r) x[r] = r < P.n ? x0[r] : (T)0;
    // knots a and a+1 of the running segment in Ua / Ub; knot a+2 is loaded
    // when segment a starts and first read when it ends, so its latency
    // hides behind the segment's steps (indices past the last knot read the
    // last knot, which only ever meets c = 0)
    T Ua[MM], Ub[MM], Un[MM];
    auto load = [&](int kn, T *dst) {
        const int kc = kn < p ? kn : p - 1;
#pragma unroll
        for (int i = 0; i < MM; ++i) dst[i] = i < m ? knots[(int64_t)(kc * m + i) * ld + cand] : (T)0;
    };
    load(0, Ua);
    load(1, Ub);
    T J = 0;
    int k = 0;
    for (int a = 0; a < p; ++a) {
        load(a + 2, Un);
        // first step of segment a+1: ceil((a+1)(T-1)/(p-1))
        const int kend = (p == 1 || a == p - 1) ? Tn : ((a + 1) * (Tn - 1) + (p - 2)) / (p - 1);
        for (; k < kend; ++k) {
            const Knot s = knot_at(Tn, p, k);
            const T c = (T)s.rem / (T)s.den;
            T u[MM];
            if (FULL) {
                T eu[MM];
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    u[i] = ((T)1 - c) * Ua[i] + c * Ub[i];
                    eu[i] = u[i] - sug[i];
                }
                J += quad_lds<T, MM>(sR, eu);
            } else {
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    u[i] = ((T)1 - c) * Ua[i] + c * Ub[i];
                    const T e = u[i] - sug[i];
                    J += sr[i] * e * e;
                }
            }
            T xn[NM];
#pragma unroll
            for (int r = 0; r < NM; ++r) {
                T acc = sw[r];
#pragma unroll
                for (int j = 0; j < NM; ++j) acc += sA[r * NM + j] * x[j];
#pragma unroll
                for (int i = 0; i < MM; ++i) acc += sB[r * MM + i] * u[i];
                xn[r] = acc;
            }
            if (FULL) {
                T e[NM];
#pragma unroll
                for (int r = 0; r < NM; ++r) {
                    x[r] = xn[r];
                    e[r] = x[r] - sxg[r];
                }
                J += quad_lds<T, NM>(sQ, e);
            }
#pragma unroll
            for (int r = 0; r < NM; ++r) {
                if (!FULL) {
                    x[r] = xn[r];
                    const T e = x[r] - sxg[r];
                    J += sq[r] * e * e;
                }
                if (BOX) {
                    J += sqb[r] * box_pen(x[r], slo[r], shi[r]);
                    J += ssb[r] * box_out(x[r], slo[r], shi[r]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            Ua[i] = Ub[i];
            Ub[i] = Un[i];
        }
    }
    if (FULL) {
        T e[NM];
#pragma unroll
        for (int r = 0; r < NM; ++r) e[r] = x[r] - sxg[r];
        J += quad_lds<T, NM>(sQf, e);
    } else {
#pragma unroll
        for (int r = 0; r < NM; ++r) {
            const T e = x[r] - sxg[r];
            J += sqf[r] * e * e;
        }
    }
    cost[cand] = J;
}

// One candidate per thread; the model and weights staged in LDS, zero-padded
// to NM x NM and NM x MM so every loop is unrolled with no bounds tests.
// Every thread of the workgroup takes part in the staging (candidate `cand`
// of the workgroup's problem; none past ncand).
template <typename T, int NM, int MM, bool BOX, bool FULL>
__device__ __forceinline__ void valu_block(const ProbView<T> &P, const T *__restrict__ x0,
                                           const T *__restrict__ knots, int64_t ld, int64_t ncand,
                                           T *__restrict__ cost, int64_t cand) {
    __shared__ T sA[NM * NM], sB[NM * MM];
    __shared__ T sw[NM], sq[NM], sqf[NM], sxg[NM], sr[MM], sug[MM];
    __shared__ T slo[BOX ? NM : 1], shi[BOX ? NM : 1], sqb[BOX ? NM : 1], ssb[BOX ? NM : 1];
    __shared__ T sQ[FULL ? NM * NM : 1], sR[FULL ? MM * MM : 1], sQf[FULL ? NM * NM : 1];
    const int n = P.n, m = P.m;
    for (int e = threadIdx.x; e < NM * NM; e += blockDim.x) {
        const int r = e / NM, c = e % NM;
        sA[e] = (r < n && c < n) ? P.Ad[r * n + c] : (T)0;
    }
    for (int e = threadIdx.x; e < NM * MM; e += blockDim.x) {
        const int r = e / MM, i = e % MM;
        sB[e] = (r < n && i < m) ? P.Bd[r * m + i] : (T)0;
    }
    for (int r = threadIdx.x; r < NM; r += blockDim.x) {
        const bool in = r < n;
        sw[r] = (in && P.wd) ? P.wd[r] : (T)0;
        sq[r] = (in && P.q) ? P.q[r] : (T)0;
        sqf[r] = (in && P.qf) ? P.qf[r] : (T)0;
        sxg[r] = (in && P.xg) ? P.xg[r] : (T)0;
        if (BOX) {  // padding rows: a box around their zero state, no weight
            slo[r] = in ? P.xlo[r] : (T)-1;
            shi[r] = in ? P.xhi[r] : (T)1;
            sqb[r] = in ? P.qb[r] : (T)0;
            ssb[r] = (in && P.sb) ? P.sb[r] : (T)0;
        }
    }
    if (FULL) {  // full matrices, or the diagonal vectors on the diagonal
        for (int e = threadIdx.x; e < NM * NM; e += blockDim.x) {
            const int r = e / NM, c = e % NM;
            const bool in = r < n && c < n;
            sQ[e] = !in ? (T)0 : P.Qm ? P.Qm[r * n + c] : (r == c ? P.q[r] : (T)0);
            sQf[e] = !in ? (T)0
                   : P.Qfm ? P.Qfm[r * n + c]
                           : ((r == c && P.qf) ? P.qf[r] : (T)0);
        }
        for (int e = threadIdx.x; e < MM * MM; e += blockDim.x) {
            const int r = e / MM, c = e % MM;
            const bool in = r < m && c < m;
            sR[e] = !in ? (T)0 : P.Rm ? P.Rm[r * m + c] : (r == c ? P.r[r] : (T)0);
        }
    }
    for (int i = threadIdx.x; i < MM; i += blockDim.x) {
        sr[i] = (i < m && P.r) ? P.r[i] : (T)0;
        sug[i] = (i < m && P.ug) ? P.ug[i] : (T)0;
    }
    __syncthreads();
    if (cand >= ncand) return;
    valu_candidate<T, NM, MM, BOX, FULL>(P, sA, sB, sw, sq, sqf, sxg, sr, sug, slo, shi, sqb, ssb,
                                         sQ, sR, sQf, x0, knots, ld, cost, cand);
}

template <typename T, int NM, int MM, bool BOX, bool FULL = false>
__global__ __launch_bounds__(256) void roll_linear_valu(ProbView<T> P, const T *__restrict__ x0,
                                                        const T *__restrict__ knots, int64_t ld,
                                                        int64_t ncand, T *__restrict__ cost) {
    valu_block<T, NM, MM, BOX, FULL>(P, x0, knots, ld, ncand, cost,
                                     (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

}  // namespace empc
