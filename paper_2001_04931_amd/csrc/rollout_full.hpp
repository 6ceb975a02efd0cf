// Linear-model rollout + cost with full weights Q, R, Qf (eq. 3 in general
// form), 16 lanes per candidate (gfx950).
//
// With one candidate per lane (rollout_valu.hpp) a population of a few
// thousand is only a few dozen wavefronts, each stepping through n (n + m)
// + n^2 multiply-adds per step in sequence.  Here a 16-lane row of a
// wavefront carries one candidate (4 per wavefront, 16 per workgroup of
// 256): lane r owns state rows r, r + 16, .. (J of them, n <= 16 J) and
// inputs r, r + 16, .. (JM, m <= 16 JM).  A_d, B_d, Q and R sit in LDS
// (shared by the workgroup's candidates, rows padded to an odd stride so
// the row's 16 lanes hit 16 banks); the state goes through LDS once per
// step: every lane writes its rows, then reads the whole vector back (a
// row lies inside one wavefront, whose LDS operations complete in order,
// so no barrier is needed), and one pass over it gives both the next state
// rows (A_d x + the knot term) and the rows of Q (x - g) for the stage cost
// of x.  The knot term is precomputed per knot (V_a = B_d U_a + w_d, the
// lane's rows), the input cost of a knot segment is summed in closed form
// (u is affine in c there): nseg e0^T R e0 + 2 C1 e0^T R du + C2 du^T R du
// with e0 = U_a - u_g, du = U_b - U_a, each lane taking its inputs' rows of
// R.  The terminal weight Qf is read from global memory once.  The row's
// partial costs are summed over its 16 lanes at the end.
#pragma once
#include <math.h>

#include "internal.hpp"

namespace empc {

constexpr int FULL_ROWS_NMAX = 64;  // states of the 16-lane full-weight form
constexpr int FULL_ROWS_MMAX = 32;  // inputs

// LDS layout of the form (elements of T): A [nr][sa], B [nr][sb], Q [nr][sa],
// R [m][sr], the goals x_g [n] and u_g [m], the workgroup's states xs
// [16][nr] and knots us [16][2][m]; nr = 16 J rows, the rows past n zero, so
// that the step loop runs with no guard (a padding row stays at zero).
struct FullRowsLds {
    int sa, sb, sr;
    int oA, oB, oQ, oR, oG, oUg, oX, oU, total;
};
__host__ __device__ inline FullRowsLds full_rows_lds(int n, int m, int J) {
    FullRowsLds L;
    const int nr = 16 * J;
    L.sa = n | 1;
    L.sb = m | 1;
    L.sr = m | 1;
    L.oA = 0;
    L.oB = L.oA + nr * L.sa;
    L.oQ = L.oB + nr * L.sb;
    L.oR = L.oQ + nr * L.sa;
    L.oG = L.oR + m * L.sr;
    L.oUg = L.oG + n;
    L.oX = L.oUg + m;
    L.oU = L.oX + 16 * nr;
    L.total = L.oU + 16 * 2 * m;
    return L;
}

template <typename T, int J, int JM, bool BOX>
__global__ __launch_bounds__(256) void roll_linear_full_rows(ProbView<T> P,
                                                             const T *__restrict__ x0,
                                                             const T *__restrict__ knots,
                                                             int64_t ld, int64_t ncand,
                                                             T *__restrict__ cost) {
    extern __shared__ __align__(16) unsigned char full_smem[];
    T *sm = (T *)full_smem;
    const int n = P.n, m = P.m, p = P.p, Tn = P.Tn;
    constexpr int NR = 16 * J;
    const FullRowsLds L = full_rows_lds(n, m, J);
    T *sA = sm + L.oA, *sB = sm + L.oB, *sQ = sm + L.oQ, *sR = sm + L.oR;
    T *sG = sm + L.oG, *sUg = sm + L.oUg;
    for (int i = threadIdx.x; i < n; i += blockDim.x) sG[i] = P.xg ? P.xg[i] : (T)0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) sUg[i] = P.ug ? P.ug[i] : (T)0;
    // stage A_d, B_d, Q, R (a diagonal given as a vector goes on the diagonal)
    for (int e = threadIdx.x; e < NR * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        const bool in = i < n;
        sA[i * L.sa + j] = in ? P.Ad[e] : (T)0;
        sQ[i * L.sa + j] = !in ? (T)0 : P.Qm ? P.Qm[e] : (i == j ? P.q[i] : (T)0);
    }
    for (int e = threadIdx.x; e < NR * m; e += blockDim.x)
        sB[(e / m) * L.sb + e % m] = e < n * m ? P.Bd[e] : (T)0;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e % m;
        sR[i * L.sr + j] = P.Rm ? P.Rm[e] : (i == j ? P.r[i] : (T)0);
    }
    __syncthreads();
    const int r = threadIdx.x & 15, slot = threadIdx.x >> 4;  // lane in row, row in workgroup
    const int64_t cand0 = (int64_t)blockIdx.x * 16;
    if (cand0 + (threadIdx.x >> 6) * 4 >= ncand) return;  // whole wavefront past the end
    const int64_t cand = cand0 + slot;
    const bool valid = cand < ncand;
    const int64_t cc = valid ? cand : ncand - 1;  // loads stay in bounds
    T *xs = sm + L.oX + slot * NR;
    T *ua = sm + L.oU + slot * 2 * m, *ub = ua + m;

    // the lane's rows: goal, disturbance, box
    T g[J], w[J], lo[J], hi[J], qb[J], sbw[J];
#pragma unroll
    for (int t = 0; t < J; ++t) {
        const int i = r + 16 * t;
        const bool in = i < n;
        g[t] = (in && P.xg) ? P.xg[i] : (T)0;
        w[t] = (in && P.wd) ? P.wd[i] : (T)0;
        lo[t] = (BOX && in) ? P.xlo[i] : (T)0;
        hi[t] = (BOX && in) ? P.xhi[i] : (T)0;
        qb[t] = (BOX && in) ? P.qb[i] : (T)0;
        sbw[t] = (BOX && in && P.sb) ? P.sb[i] : (T)0;
    }
    T gu[JM];
#pragma unroll
    for (int t = 0; t < JM; ++t) {
        const int i = r + 16 * t;
        gu[t] = (i < m && P.ug) ? P.ug[i] : (T)0;
    }
    // knots a (ua) and a+1 (ub) of the candidate in LDS, the lane's inputs
    // loaded by the lane; knot a+2 is loaded into registers (pre) when
    // segment a starts and stored to LDS when it ends, so the load's
    // latency hides behind the segment's steps
    T pre[JM];
    auto fetch_knot = [&](int kn) {
        const int kc = kn < p ? kn : p - 1;
#pragma unroll
        for (int t = 0; t < JM; ++t) {
            const int i = r + 16 * t;
            pre[t] = i < m ? knots[(int64_t)(kc * m + i) * ld + cc] : (T)0;
        }
    };
    auto store_knot = [&](T *dst) {
#pragma unroll
        for (int t = 0; t < JM; ++t) {
            const int i = r + 16 * t;
            if (i < m) dst[i] = pre[t];
        }
    };
    // V = B_d U + w_d for the lane's rows from a knot in LDS (padding rows:
    // zero rows of B_d, w = 0)
    auto response = [&](const T *u, T *V) {
#pragma unroll
        for (int t = 0; t < J; ++t) V[t] = w[t];
        for (int l = 0; l < m; ++l) {
            const T ul = u[l];
#pragma unroll
            for (int t = 0; t < J; ++t) V[t] += sB[(r + 16 * t) * L.sb + l] * ul;
        }
    };
    // the lane's share of the segment input cost
    auto input_cost = [&](int nseg, T C1, T C2, bool last) -> T {
        T s = 0;
#pragma unroll
        for (int t = 0; t < JM; ++t) {
            const int i = r + 16 * t;
            if (i < m) {
                T re = 0, rd = 0;
                for (int l = 0; l < m; ++l) {
                    const T e0l = ua[l] - sUg[l];
                    const T dul = last ? (T)0 : ub[l] - ua[l];
                    re += sR[i * L.sr + l] * e0l;
                    rd += sR[i * L.sr + l] * dul;
                }
                const T e0 = ua[i] - gu[t], du = last ? (T)0 : ub[i] - ua[i];
                s += (T)nseg * e0 * re + (T)2 * C1 * e0 * rd + C2 * du * rd;
            }
        }
        return s;
    };
    // x_0 into LDS (padding rows: 0)
#pragma unroll
    for (int t = 0; t < J; ++t) {
        const int i = r + 16 * t;
        xs[i] = i < n ? x0[i] : (T)0;
    }
    fetch_knot(0);
    store_knot(ua);
    fetch_knot(1);
    store_knot(ub);
    // Q g for the lane's rows
    T qg[J];
#pragma unroll
    for (int t = 0; t < J; ++t) qg[t] = 0;
    for (int j = 0; j < n; ++j) {
        const T gj = sG[j];
#pragma unroll
        for (int t = 0; t < J; ++t) qg[t] += sQ[(r + 16 * t) * L.sa + j] * gj;
    }
    T Va[J], Vb[J];
    response(ua, Va);
    response(ub, Vb);
    T Jc = 0;
    int a = 0, k = 0;
    // knot position of step k kept incrementally: k (p-1) = a (T-1) + rem
    const int den = Tn > 1 ? Tn - 1 : 1;
    const T inv_den = (T)1 / (T)den;
    int rem = 0;
    for (; a < p; ++a) {
        // steps of segment a: k .. kend-1 (first step of segment a+1:
        // ceil((a+1)(T-1)/(p-1)))
        const int kend = (p == 1 || a == p - 1) ? Tn : ((a + 1) * (Tn - 1) + (p - 2)) / (p - 1);
        if (a + 2 < p + 1) fetch_knot(a + 2);
        int nseg = 0;
        T C1 = 0, C2 = 0;
        for (; k < kend; ++k) {
            const T c = (p > 1 && Tn > 1) ? (T)rem * inv_den : (T)0;
            if (p > 1 && Tn > 1) {
                rem += p - 1;
                if (rem >= den) rem -= den;
            }
            C1 += c;
            C2 += c * c;
            ++nseg;
            // one pass over x_k: next rows and (for k > 0) Q (x_k - g) rows
            // (Q x - Q g, Q g precomputed), eight columns in flight
            T xn[J], qe[J];
#pragma unroll
            for (int t = 0; t < J; ++t) {
                xn[t] = Va[t] + c * (Vb[t] - Va[t]);
                qe[t] = -qg[t];
            }
#pragma unroll 8
            for (int j = 0; j < n; ++j) {
                const T xj = xs[j];
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    const int i = r + 16 * t;
                    xn[t] += sA[i * L.sa + j] * xj;
                    qe[t] += sQ[i * L.sa + j] * xj;
                }
            }
            if (k > 0) {  // stage cost of x_k (padding rows add zero)
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    const T xi = xs[r + 16 * t];  // x_k, this lane's own row
                    Jc += (xi - g[t]) * qe[t];
                    if (BOX) Jc += qb[t] * box_pen(xi, lo[t], hi[t]) + sbw[t] * box_out(xi, lo[t], hi[t]);
                }
            }
            // every lane of the row has read x_k (program order): store x_{k+1}
#pragma unroll
            for (int t = 0; t < J; ++t) xs[r + 16 * t] = xn[t];
        }
        Jc += input_cost(nseg, C1, C2, a == p - 1);
        if (a + 1 < p) {
            // next segment: knot a+1 becomes the first, knot a+2 the second
#pragma unroll
            for (int t = 0; t < J; ++t) Va[t] = Vb[t];
            // all lanes have used ua / ub (program order within the row)
            for (int l = r; l < m; l += 16) ua[l] = ub[l];
            store_knot(ub);
            response(ub, Vb);
        }
    }
    // x_T: stage weight Q and terminal weight Qf (global), box
#pragma unroll
    for (int t = 0; t < J; ++t) {
        const int i = r + 16 * t;
        if (i < n) {
            T qf = 0, qs = 0;
            for (int j = 0; j < n; ++j) {
                const T ej = xs[j] - sG[j];
                qs += sQ[i * L.sa + j] * ej;
                qf += (P.Qfm ? P.Qfm[i * n + j] : ((i == j && P.qf) ? P.qf[i] : (T)0)) * ej;
            }
            const T xi = xs[i];
            Jc += (xi - g[t]) * (qs + qf);
            if (BOX) Jc += qb[t] * box_pen(xi, lo[t], hi[t]) + sbw[t] * box_out(xi, lo[t], hi[t]);
        }
    }
    Jc += __shfl_xor(Jc, 8, 16);
    Jc += __shfl_xor(Jc, 4, 16);
    Jc += __shfl_xor(Jc, 2, 16);
    Jc += __shfl_xor(Jc, 1, 16);
    if (r == 0 && valid) cost[cand] = Jc;
}

}  // namespace empc
