// Pendulum-chain rollout + cost device code (gfx950), shared by the
// single-problem kernel (rollout.hip) and the problem-batched one
// (batched.hip).  One candidate per lane, joint state in registers, the
// per-joint constants in LDS where every lane reads the same address.
#pragma once
#include <math.h>

#include "internal.hpp"

namespace empc {

// ---------------------------------------------------------------------------
// Pendulum chain.  Per-joint constants in LDS.
template <typename T>
struct JointConst {
    T cg;    // g l_r M_r (gravity coefficient of absolute angle r)
    T dtI;   // dt / I_j (the velocity update's factor)
    T kst, dmp;
    T wq, wv, wqf, wvf;  // stage and terminal weights of q_j and qd_j
    T gq, gv;            // goals of q_j and qd_j
    T wr, gu;            // input weight and goal
    T bq, bv;            // state box penalty weights of q_j and qd_j (0: none)
    T loq, hiq, lov, hiv;  // and its bounds
    T sq, sv;            // step charges outside the box (0: none)
    T qmn, qmx;          // joint limits (with impacts)
    T fc, fs;            // dry friction: sliding, breakaway torque
};

// Compile-time features of the chain forms: the state box penalty with its
// step charge, joint limits with impacts, dry friction with stiction.
constexpr int CF_BOX = 1, CF_LIMIT = 2, CF_FRIC = 4;

template <typename T>
__device__ void chain_constants_lds(const ProbView<T> &P, JointConst<T> *jc) {
    const int d = P.m;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        T tail = 0;
        for (int i = j; i < d; ++i) tail += P.mass[i];
        T inert = 0, dist = 0;
        for (int i = j; i < d; ++i) {
            dist += P.len[i];
            inert += P.mass[i] * dist * dist;
        }
        JointConst<T> c;
        c.cg = P.gravity * P.len[j] * tail;
        c.dtI = P.dt / inert;
        c.kst = P.stiff[j];
        c.dmp = P.damp[j];
        c.wq = P.q[j];
        c.wv = P.q[d + j];
        c.wqf = P.qf ? P.qf[j] : (T)0;
        c.wvf = P.qf ? P.qf[d + j] : (T)0;
        c.gq = P.xg ? P.xg[j] : (T)0;
        c.gv = P.xg ? P.xg[d + j] : (T)0;
        c.wr = P.r[j];
        c.gu = P.ug ? P.ug[j] : (T)0;
        const bool box = P.qb != nullptr;
        c.bq = box ? P.qb[j] : (T)0;
        c.bv = box ? P.qb[d + j] : (T)0;
        c.loq = box ? P.xlo[j] : (T)0;
        c.hiq = box ? P.xhi[j] : (T)0;
        c.lov = box ? P.xlo[d + j] : (T)0;
        c.hiv = box ? P.xhi[d + j] : (T)0;
        c.sq = (box && P.sb) ? P.sb[j] : (T)0;
        c.sv = (box && P.sb) ? P.sb[d + j] : (T)0;
        c.qmn = P.qlo ? P.qlo[j] : (T)0;
        c.qmx = P.qhi ? P.qhi[j] : (T)0;
        c.fc = P.fc ? P.fc[j] : (T)0;
        c.fs = P.fs ? P.fs[j] : (T)0;
        jc[j] = c;
    }
}

template <typename T>
__device__ inline T sin_of(T x);
template <>
__device__ inline float sin_of<float>(float x) { return sinf(x); }
template <>
__device__ inline double sin_of<double>(double x) { return sin(x); }

// sin for the rollout's gravity torques, of an angle given in the unit
// RolloutAngle<T>::per_rad per radian.  FP32: the hardware transcendental
// (v_sin_f32 takes its argument in revolutions; the rollout sums the
// cumulative angles in revolutions directly, q / (2 pi) folded into the sum
// as one fused multiply-add), instead of the library's range reduction and
// polynomial; its absolute error (a few 1e-7) is of the order of FP32
// rounding of the cumulative angle itself.  FP64: radians, the library sin.
template <typename T>
struct RolloutAngle;
template <>
struct RolloutAngle<float> {
    static constexpr float per_rad = 0.15915494309189535f;  // 1 / (2 pi)
    __device__ static float sin(float rev) { return __builtin_amdgcn_sinf(rev); }
};
template <>
struct RolloutAngle<double> {
    static constexpr double per_rad = 1.0;
    __device__ static double sin(double rad) { return ::sin(rad); }
};

// One thread: candidate `cand` of one problem; jc holds the problem's
// per-joint constants.  FEAT: CF_BOX (state box penalty and step charge),
// CF_LIMIT (joint limits with impacts).
template <typename T, int DMAX, int FEAT>
__device__ __forceinline__ void chain_candidate(const ProbView<T> &P, const JointConst<T> *jc,
                                                const T *__restrict__ x0,
                                                const T *__restrict__ knots, int64_t ld,
                                                T *__restrict__ cost, int64_t cand) {
    const int d = P.m;
    const T dt = P.dt;
    constexpr bool box = (FEAT & CF_BOX) != 0, limit = (FEAT & CF_LIMIT) != 0;
    constexpr bool fric = (FEAT & CF_FRIC) != 0;
    const T rest = P.rest;
    T q[DMAX], v[DMAX], ua[DMAX], ub[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        q[j] = j < d ? x0[j] : (T)0;
        v[j] = j < d ? x0[d + j] : (T)0;
    }
    const int Tn = P.Tn, p = P.p, den = Tn - 1;
    const T inv_den = Tn > 1 ? (T)1 / (T)den : (T)0;
    auto load_knot = [&](int kn, T *dst) {
        const int kc = kn < p ? kn : p - 1;
#pragma unroll
        for (int j = 0; j < DMAX; ++j)  // joints past d (never used) repeat d-1:
            // every lane issues the same loads, which keeps the waits countable
            dst[j] = knots[(int64_t)(kc * d + (j < d ? j : d - 1)) * ld + cand];
    };
    // knots a, a+1 (ub) and a+2 (un); the knot position of step k is kept
    // incrementally, k (p-1) = a (T-1) + rem (p <= T: at most one boundary
    // per step)
    T un[DMAX];
    load_knot(0, ua);
    load_knot(1, ub);
    int a = 0, rem = 0, k = 0;
    T J = 0;
    // outer loop: knot segments; inner loop: the steps of one segment.  Knot
    // a+2 is loaded when a segment starts and first used when it ends.
    for (;;) {
        load_knot(a + 2, un);
        bool adv = false;
        do {
        // re-read the per-joint constants from LDS every step instead of
        // letting them be hoisted into (and overflow) registers
        asm volatile("" ::: "memory");
        const T c = (T)rem * inv_den;
        // gravity torque: G_j = sum_{r>=j} cg_r sin(phi_r), phi_r = q_0 + .. + q_r
        // (phi summed in the unit of RolloutAngle<T>)
        T sg[DMAX];
        T phi = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (j < d) {
                phi += q[j] * RolloutAngle<T>::per_rad;
                sg[j] = jc[j].cg * RolloutAngle<T>::sin(phi);
            }
        }
        T G = 0, js = 0;
#pragma unroll
        for (int j = DMAX - 1; j >= 0; --j) {
            if (j < d) {
                const JointConst<T> cj = jc[j];
                G += sg[j];
                const T u = ((T)1 - c) * ua[j] + c * ub[j];
                // qd += dt (u - k q - b qd - G) / I, with dt / I as one factor
                const T f = u - cj.kst * q[j] - cj.dmp * v[j] - G;
                const T vf = v[j] + cj.dtI * f;
                v[j] = fric ? dry_friction(v[j], vf, f, cj.dtI, cj.fc, cj.fs) : vf;
                q[j] = q[j] + dt * v[j];
                if (limit) joint_limit(q[j], v[j], cj.qmn, cj.qmx, rest);
                const T eq = cj.gq - q[j], ev = cj.gv - v[j], eu = cj.gu - u;
                js += cj.wq * eq * eq + cj.wv * ev * ev + cj.wr * eu * eu;
                if (box) {
                    js += cj.bq * box_pen(q[j], cj.loq, cj.hiq) + cj.bv * box_pen(v[j], cj.lov, cj.hiv);
                    js += cj.sq * box_out(q[j], cj.loq, cj.hiq) + cj.sv * box_out(v[j], cj.lov, cj.hiv);
                }
            }
        }
        J += js;
        if (p > 1 && Tn > 1) {
            rem += p - 1;
            adv = rem >= den && k + 1 < Tn;
        }
        ++k;
        } while (!adv && k < Tn);
        if (!adv) break;  // k == Tn
        rem -= den;
        ++a;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            ua[j] = ub[j];
            ub[j] = un[j];
        }
    }
    T jt = 0;
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        if (j < d) {
            const T eq = jc[j].gq - q[j], ev = jc[j].gv - v[j];
            jt += jc[j].wqf * eq * eq + jc[j].wvf * ev * ev;
        }
    }
    cost[cand] = J + jt;
}

template <typename T, int DMAX, int FEAT>
__global__ __launch_bounds__(256) void roll_chain(ProbView<T> P, const T *__restrict__ x0,
                                                  const T *__restrict__ knots, int64_t ld,
                                                  int64_t ncand, T *__restrict__ cost) {
    __shared__ JointConst<T> jc[DMAX];
    chain_constants_lds(P, jc);
    __syncthreads();
    const int64_t cand = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cand >= ncand) return;
    chain_candidate<T, DMAX, FEAT>(P, jc, x0, knots, ld, cost, cand);
}

// ---------------------------------------------------------------------------
// Row layout: one candidate per 16-lane row, lane r owning joints
// r*J .. r*J+J-1 (J = ceil(d/16)).  The cumulative angles are a prefix sum
// over joints and the gravity torques a suffix sum, both done as a local sum
// over the lane's J joints plus a scan over the 16 lanes of the row with DPP
// row shifts (which never cross a row).
// One candidate per 16-lane row.  `cand` is the row's candidate; r the lane
// in the row.  Every lane of the wavefront must call this (DPP).  FEAT:
// CF_BOX, CF_LIMIT as for the lane form.
template <typename T, int J, int FEAT>
__device__ __forceinline__ void chain_row_candidate(const ProbView<T> &P, const T *__restrict__ x0,
                                                    const T *__restrict__ knots, int64_t ld,
                                                    int64_t ncand, T *__restrict__ cost,
                                                    int64_t cand, int r) {
    const int d = P.m;
    const bool valid = cand < ncand;
    const int64_t cc = valid ? cand : ncand - 1;  // loads stay in bounds
    // per-joint constants of this lane's joints (zero for joints past d)
    T q[J], v[J], cg[J], dtI[J], kst[J], dmp[J], wq[J], wv[J], gq[J], gv[J], wr[J], gu[J];
    T ua[J], ub[J];
    // state box penalty: weights, bounds and running sums; step charges and
    // the running counts of steps outside; joint limits
    constexpr bool box = (FEAT & CF_BOX) != 0, limit = (FEAT & CF_LIMIT) != 0;
    constexpr bool fric = (FEAT & CF_FRIC) != 0;
    T fcr[fric ? J : 1], fsr[fric ? J : 1];
    T bq[J], bv[J], loq[J], hiq[J], lov[J], hiv[J], Pq[J], Pv[J];
    T sq[box ? J : 1], sv[box ? J : 1], Nq[box ? J : 1], Nv[box ? J : 1];
    T qmn[limit ? J : 1], qmx[limit ? J : 1];
    const T rest = P.rest;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const int j = r * J + i;
        const bool in = j < d;
        T tail = 0, inert = 0, dist = 0;
        if (in) {
            for (int t = j; t < d; ++t) {
                tail += P.mass[t];
                dist += P.len[t];
                inert += P.mass[t] * dist * dist;
            }
        }
        cg[i] = in ? P.gravity * P.len[j] * tail : (T)0;
        dtI[i] = in ? P.dt / inert : (T)0;
        kst[i] = in ? P.stiff[j] : (T)0;
        dmp[i] = in ? P.damp[j] : (T)0;
        wq[i] = in ? P.q[j] : (T)0;
        wv[i] = in ? P.q[d + j] : (T)0;
        gq[i] = (in && P.xg) ? P.xg[j] : (T)0;
        gv[i] = (in && P.xg) ? P.xg[d + j] : (T)0;
        wr[i] = in ? P.r[j] : (T)0;
        gu[i] = (in && P.ug) ? P.ug[j] : (T)0;
        q[i] = in ? x0[j] : (T)0;
        v[i] = in ? x0[d + j] : (T)0;
        const bool bx = in && box;
        bq[i] = bx ? P.qb[j] : (T)0;
        bv[i] = bx ? P.qb[d + j] : (T)0;
        loq[i] = bx ? P.xlo[j] : (T)0;
        hiq[i] = bx ? P.xhi[j] : (T)0;
        lov[i] = bx ? P.xlo[d + j] : (T)0;
        hiv[i] = bx ? P.xhi[d + j] : (T)0;
        Pq[i] = Pv[i] = 0;
        if (box) {
            sq[i] = (bx && P.sb) ? P.sb[j] : (T)0;
            sv[i] = (bx && P.sb) ? P.sb[d + j] : (T)0;
            Nq[i] = Nv[i] = 0;
        }
        if (limit) {
            qmn[i] = in ? P.qlo[j] : (T)0;
            qmx[i] = in ? P.qhi[j] : (T)0;
        }
        if (fric) {
            fcr[i] = in ? P.fc[j] : (T)0;
            fsr[i] = in ? P.fs[j] : (T)0;
        }
    }
    const T dt = P.dt;
    const int Tn = P.Tn, p = P.p, den = Tn - 1;
    const T inv_den = Tn > 1 ? (T)1 / (T)den : (T)0;
    // knot position of step k tracked incrementally: k (p-1) = a (T-1) + rem
    int a = 0, rem = 0;
    // knots a, a+1 (b) and a+2 (prefetched) of the lane's joints
    T un[J], du[J];
    auto load_knot = [&](int kn, T *dst) {
        const int kc = kn < p ? kn : p - 1;
#pragma unroll
        for (int i = 0; i < J; ++i) {
            const int j = r * J + i;
            dst[i] = knots[(int64_t)(kc * d + (j < d ? j : d - 1)) * ld + cc];
        }
    };
    load_knot(0, ua);
    load_knot(1, ub);
#pragma unroll
    for (int i = 0; i < J; ++i) du[i] = ub[i] - ua[i];
    // stage cost: per joint sums of squared errors, weighted at the end; the
    // input cost of a knot segment in closed form (u = U_a + c dU is affine
    // in c there): sum (g - U_a - c dU)^2 = n e0^2 - 2 e0 dU C1 + dU^2 C2,
    // e0 = g - U_a, with C1, C2 the sums of c and c^2 over the segment
    T Sq[J], Sv[J];
#pragma unroll
    for (int i = 0; i < J; ++i) Sq[i] = Sv[i] = 0;
    T Ju = 0, C1 = 0, C2 = 0;
    int nseg = 0;
    auto flush_input = [&]() {
#pragma unroll
        for (int i = 0; i < J; ++i) {
            const T e0 = gu[i] - ua[i];
            Ju += wr[i] * ((T)nseg * e0 * e0 - (T)2 * e0 * du[i] * C1 + du[i] * du[i] * C2);
        }
    };
    // Outer loop: knot segments; inner loop: the steps of one segment.  Knot
    // a+2 is loaded when a segment starts and first used when it ends, and
    // nothing merges into its registers in between, so the wait for that
    // load falls at the segment's end rather than right after the load.
    int k = 0;
    for (;;) {
        load_knot(a + 2, un);
        bool adv = false;
        do {
        const T c = (T)rem * inv_den;
        C1 += c;
        C2 += c * c;
        ++nseg;
        // cumulative angles phi: local prefix over the lane's joints, then
        // the row's exclusive prefix of lane totals
        T loc[J];
        T run = q[0];
        loc[0] = run;
#pragma unroll
        for (int i = 1; i < J; ++i) {
            run += q[i];
            loc[i] = run;
        }
        const T before = (row_scan_up<T>(run) - run) * RolloutAngle<T>::per_rad;
        T sg[J];
#pragma unroll
        for (int i = 0; i < J; ++i)
            sg[i] = cg[i] * RolloutAngle<T>::sin(loc[i] * RolloutAngle<T>::per_rad + before);
        // gravity torque G_j = sum_{r >= j} cg_r sin(phi_r): local suffix plus
        // the row's exclusive suffix of lane totals
        T srun = 0, sloc[J];
#pragma unroll
        for (int i = J - 1; i >= 0; --i) {
            srun += sg[i];
            sloc[i] = srun;
        }
        const T after = row_scan_down<T>(srun) - srun;
#pragma unroll
        for (int i = 0; i < J; ++i) {
            const T G = after + sloc[i];
            const T u = ua[i] + c * du[i];
            // qd += dt (u - k q - b qd - G) / I, with dt / I as one factor
            const T f = u - kst[i] * q[i] - dmp[i] * v[i] - G;
            const T vf = v[i] + dtI[i] * f;
            v[i] = fric ? dry_friction(v[i], vf, f, dtI[i], fcr[i], fsr[i]) : vf;
            q[i] = q[i] + dt * v[i];
            if (limit) joint_limit(q[i], v[i], qmn[i], qmx[i], rest);
            const T eq = gq[i] - q[i], ev = gv[i] - v[i];
            Sq[i] += eq * eq;
            Sv[i] += ev * ev;
            if (box) {
                Pq[i] += box_pen(q[i], loq[i], hiq[i]);
                Pv[i] += box_pen(v[i], lov[i], hiv[i]);
                Nq[i] += box_out(q[i], loq[i], hiq[i]);
                Nv[i] += box_out(v[i], lov[i], hiv[i]);
            }
        }
        // advance the knot position to step k + 1 (uniform)
        if (p > 1 && Tn > 1) {
            rem += p - 1;
            adv = rem >= den && k + 1 < Tn;
        }
        ++k;
        } while (!adv && k < Tn);
        if (!adv) break;  // k == Tn
        flush_input();
        C1 = C2 = 0;
        nseg = 0;
        rem -= den;
        ++a;
#pragma unroll
        for (int i = 0; i < J; ++i) {
            ua[i] = ub[i];
            ub[i] = un[i];
            du[i] = ub[i] - ua[i];
        }
    }
    flush_input();
    T J_ = Ju;
#pragma unroll
    for (int i = 0; i < J; ++i) J_ += wq[i] * Sq[i] + wv[i] * Sv[i];
    if (box)
#pragma unroll
        for (int i = 0; i < J; ++i) {
            J_ += bq[i] * Pq[i] + bv[i] * Pv[i];
            J_ += sq[i] * Nq[i] + sv[i] * Nv[i];
        }
    T jt = 0;
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const int j = r * J + i;
        if (j < d && P.qf) {
            const T eq = gq[i] - q[i], ev = gv[i] - v[i];
            jt += P.qf[j] * eq * eq + P.qf[d + j] * ev * ev;
        }
    }
    T tot = J_ + jt;
    // sum over the row's 16 lanes
    tot += __shfl_xor(tot, 8, 16);
    tot += __shfl_xor(tot, 4, 16);
    tot += __shfl_xor(tot, 2, 16);
    tot += __shfl_xor(tot, 1, 16);
    if (r == 0 && valid) cost[cand] = tot;
}

template <typename T, int J, int FEAT>
__global__ __launch_bounds__(256) void roll_chain_rows(ProbView<T> P, const T *__restrict__ x0,
                                                       const T *__restrict__ knots, int64_t ld,
                                                       int64_t ncand, T *__restrict__ cost) {
    // blockDim.x / 16 rows (candidates) per block
    const int64_t cand0 = xcd_swizzle(blockIdx.x, gridDim.x) * (int64_t)(blockDim.x >> 4);
    if (cand0 + (threadIdx.x >> 6) * 4 >= ncand) return;  // whole wavefront past the end
    chain_row_candidate<T, J, FEAT>(P, x0, knots, ld, ncand, cost, cand0 + (threadIdx.x >> 4),
                              threadIdx.x & 15);
}

}  // namespace empc
