// Adjoint gradient of the rollout cost with respect to the knots, and Adam
// refinement built on it (gfx950).
//
// One workgroup of two wavefronts per candidate: a few dozen elites each run
// a sequential chain of dependent steps per Adam step, so the latency of one
// step is what counts.  Wavefront 0 runs the forward pass and the backward
// steps; wavefront 1 recomputes the states of the next checkpoint segment
// (into the other of two LDS buffers) while wavefront 0 walks the current one
// backward, so an Adam step is T + S + T dependent steps instead of 3T.  Linear model: lane i owns state i
// (n <= 64) and, for i < m, input i, and holds row i and column i of A_d and
// of B_d in registers; each lane publishes its state (or adjoint) to LDS and
// reads the whole vector back with broadcast 16-byte loads (the LDS
// operations of one wavefront complete in order, so no barrier is needed),
// and every dot product runs on four partial sums, so its dependent chain
// is a quarter of its length.  Pendulum chain: lane j owns joint j
// (d <= 64); the cumulative angles, gravity torques and the adjoint's
// prefix / suffix sums are wavefront scans on DPP row shifts.
//
// With lambda_k = dJ/dx_k:
//   lambda_T = 2 (Q + Q_f)(x_T - g),
//   lambda_k = 2 Q (x_k - g) + f_x(x_k, u_k)^T lambda_{k+1},
//   dJ/du_k  = 2 R (u_k - u_g) + f_u(x_k, u_k)^T lambda_{k+1},
// and dJ/du_k goes to knots idx1 and idx2 with weights 1-c and c.  States
// are stored every S = ceil(sqrt(T)) steps on the forward pass; the backward
// pass recomputes each segment of S states from its checkpoint.
#include <math.h>

#include <type_traits>

#include "internal.hpp"

namespace empc {

template <typename T>
__device__ inline T sin_f(T x);
template <>
__device__ inline float sin_f<float>(float x) { return sinf(x); }
template <>
__device__ inline double sin_f<double>(double x) { return sin(x); }
template <typename T>
__device__ inline T cos_f(T x);
template <>
__device__ inline float cos_f<float>(float x) { return cosf(x); }
template <>
__device__ inline double cos_f<double>(double x) { return cos(x); }

// LDS plan (element counts), shared with the host-side size check.
struct GradPlan {
    int S, nchk, us;  // us: row stride of the input table (m rounded up to 4)
    size_t oU, oG, oM1, oM2, oXb, oChk, oSeg, oUk, oBu, oC, total;
};
inline GradPlan grad_plan(int model, int n, int m, int T, int p) {
    GradPlan g;
    g.S = 1;
    while (g.S * g.S < T) ++g.S;
    g.nchk = (T + g.S - 1) / g.S;
    const size_t pm = (size_t)p * m;
    size_t o = 0;
    g.oU = o; o += pm;
    g.oG = o; o += pm;
    g.oM1 = o; o += pm;
    g.oM2 = o; o += pm;
    g.oXb = o; o += 128;  // broadcast slots of the two wavefronts: states (or adjoints)
    g.oChk = o; o += (size_t)g.nchk * n;
    g.oSeg = o; o += (size_t)2 * g.S * n;  // two recomputed segments
    // per-step tables of the current knots: inputs u_k (rows of us, plus
    // 64 of padding for whole-vector reads of the last row), the linear
    // model's B_d u_k + w_d, and the blend weights c_k
    g.us = (m + 3) / 4 * 4;
    o = (o + 3) / 4 * 4;  // 16-byte aligned rows (whole-vector reads)
    g.oUk = o; o += (size_t)T * g.us + 64;
    g.oBu = o; o += model == EMPC_LINEAR ? (size_t)T * n : 0;
    g.oC = o; o += (size_t)T;
    g.total = o;
    return g;
}

template <typename T>
struct Lane {
    // per-lane constants (linear: state/input role; chain: joint role)
    T q, qf, xg, r, ug, w;                // linear state i / input i
    T cg, invI, kst, dmp, wq, wv, wqf, wvf, gq, gv, wr, gu;  // chain joint j
    T lo, hi, bq;                         // state box penalty: linear state i, chain q_j
    T lov, hiv, bv;                       // chain qd_j
    T sq, sv;                             // step charges outside the box (no derivative)
};

// LIN: linear model with NMAX >= n and MMAX >= m (register operand
// lengths); else the pendulum chain (NMAX, MMAX unused).
template <typename T, bool LIN, int NMAX, int MMAX>
__global__ __launch_bounds__(128) void adjoint_kernel(ProbView<T> P, GradPlan G,
                                                     const T *__restrict__ x0,
                                                     const T *__restrict__ knots, int64_t ld,
                                                     T *__restrict__ dJ, T *__restrict__ cost,
                                                     int steps, T lr, T *__restrict__ knots_io,
                                                     T *__restrict__ cost_io) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = (T *)smem_raw;
    T *sU = sm + G.oU, *sG = sm + G.oG;
    T *sM1 = sm + G.oM1, *sM2 = sm + G.oM2;
    T *sChk = sm + G.oChk;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    T *sXb = sm + G.oXb + 64 * wave;  // this wavefront's broadcast slots
    T *sUk = sm + G.oUk, *sBu = sm + G.oBu, *sC = sm + G.oC;
    const int64_t cand = blockIdx.x;
    const int n = P.n, m = P.m, pm = P.p * P.m, Tn = P.Tn, S = G.S;
    constexpr bool lin = LIN;
    const bool refine = steps > 0;

    // ---- load: row and column `lane` of A_d and B_d (zero padded)
    constexpr int NR = LIN ? NMAX : 4;
    constexpr int MR = LIN ? MMAX : 4;
    T aRow[NR], aCol[NR], bRow[MR], bCol[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        aRow[j] = (LIN && lane < n && j < n) ? P.Ad[lane * n + j] : (T)0;
        aCol[j] = (LIN && lane < n && j < n) ? P.Ad[j * n + lane] : (T)0;
        bCol[j] = (LIN && lane < m && j < n) ? P.Bd[j * m + lane] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < MR; ++j) bRow[j] = (LIN && lane < n && j < m) ? P.Bd[lane * m + j] : (T)0;
    const T *src = refine ? knots_io : knots;
    for (int j = threadIdx.x; j < pm; j += 128) {
        sU[j] = src[(int64_t)j * ld + cand];
        sM1[j] = 0;
        sM2[j] = 0;
    }
    Lane<T> L;
    if (lin) {
        const bool si = lane < n, ui = lane < m;
        L.q = si ? P.q[lane] : (T)0;
        L.qf = (si && P.qf) ? P.qf[lane] : (T)0;
        L.xg = (si && P.xg) ? P.xg[lane] : (T)0;
        L.w = (si && P.wd) ? P.wd[lane] : (T)0;
        L.r = ui ? P.r[lane] : (T)0;
        L.ug = (ui && P.ug) ? P.ug[lane] : (T)0;
        const bool bx = si && P.qb;
        L.bq = bx ? P.qb[lane] : (T)0;
        L.lo = bx ? P.xlo[lane] : (T)0;
        L.hi = bx ? P.xhi[lane] : (T)0;
        L.sq = (bx && P.sb) ? P.sb[lane] : (T)0;
        L.sv = 0;
    } else {
        const int d = m;
        const bool in = lane < d;
        T tail = 0, inert = 0, dist = 0;
        if (in) {
            for (int i = lane; i < d; ++i) {
                tail += P.mass[i];
                dist += P.len[i];
                inert += P.mass[i] * dist * dist;
            }
        }
        L.cg = in ? P.gravity * P.len[lane] * tail : (T)0;
        L.invI = in ? (T)1 / inert : (T)0;
        L.kst = in ? P.stiff[lane] : (T)0;
        L.dmp = in ? P.damp[lane] : (T)0;
        L.wq = in ? P.q[lane] : (T)0;
        L.wv = in ? P.q[d + lane] : (T)0;
        L.wqf = (in && P.qf) ? P.qf[lane] : (T)0;
        L.wvf = (in && P.qf) ? P.qf[d + lane] : (T)0;
        L.gq = (in && P.xg) ? P.xg[lane] : (T)0;
        L.gv = (in && P.xg) ? P.xg[d + lane] : (T)0;
        L.wr = in ? P.r[lane] : (T)0;
        L.gu = (in && P.ug) ? P.ug[lane] : (T)0;
        const bool bx = in && P.qb;
        L.bq = bx ? P.qb[lane] : (T)0;
        L.lo = bx ? P.xlo[lane] : (T)0;
        L.hi = bx ? P.xhi[lane] : (T)0;
        L.bv = bx ? P.qb[d + lane] : (T)0;
        L.lov = bx ? P.xlo[d + lane] : (T)0;
        L.hiv = bx ? P.xhi[d + lane] : (T)0;
        L.sq = (bx && P.sb) ? P.sb[lane] : (T)0;
        L.sv = (bx && P.sb) ? P.sb[d + lane] : (T)0;
    }
    __syncthreads();

    const int d = m;  // chain joints
    const bool box = P.qb != nullptr;  // state box penalty (uniform)
    // lane-owned state: linear xi (state lane); chain (q, v) of joint lane
    // sum_j c[j] v_j with v_j published by lane j: one LDS store per lane,
    // then every lane reads the vector back 16 bytes at a time (broadcast
    // reads).  The LDS operations of a wavefront complete in order, so the
    // reads see the stores; the next store comes after these values are used.
    typedef T vec __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int VW = 16 / sizeof(T);
    // acc + sum_{j < N} c[j] w_j over the vector published at `slot`, in
    // four partial sums (term j goes to sum j mod 4), added pairwise
    auto slot_dot = [&](const T *slot, const T *c, auto NC, T acc) -> T {
        constexpr int N = decltype(NC)::value;
        T a[4] = {acc, (T)0, (T)0, (T)0};
#pragma unroll
        for (int j = 0; j < N; j += VW) {
            const vec w = *reinterpret_cast<const vec *>(slot + j);
#pragma unroll
            for (int q = 0; q < VW; ++q) a[(j + q) & 3] += c[j + q] * w[q];
        }
        return (a[0] + a[1]) + (a[2] + a[3]);
    };
    // Tables of the current knots, built before each forward pass (the
    // iterations are independent, so they pipeline): c_k, the lane's input
    // u_k, and for the linear model B_d u_k + w_d.  The step chains then
    // read them instead of interpolating and multiplying.  (Each lane reads
    // the u_k rows it needs only after its own writes and those of the other
    // lanes: the LDS operations of a wavefront complete in order.)
    auto tabulate = [&]() {
        for (int k = lane; k < Tn; k += 64) {
            const Knot kn = knot_at(Tn, P.p, k);
            sC[k] = (T)kn.rem / (T)kn.den;
        }
        for (int k = 0; k < Tn; ++k) {
            const Knot kn = knot_at(Tn, P.p, k);
            const T c = sC[k];
            if (lane < G.us)
                sUk[k * G.us + lane] =
                    lane < m ? ((T)1 - c) * sU[kn.a * m + lane] + c * sU[kn.b * m + lane] : (T)0;
        }
        sUk[Tn * G.us + lane] = 0;  // padding read by the last row's vector loads
        if (lin)
            for (int k = 0; k < Tn; ++k) {
                const T bu = slot_dot(sUk + k * G.us, bRow, std::integral_constant<int, MR>(), L.w);
                if (lane < n) sBu[k * n + lane] = bu;
            }
    };
    // the lane's input at step k (0 for lanes >= m)
    auto input_at = [&](int k) -> T { return sUk[k * G.us + lane]; };
    // one linear step: xi <- A x + (B u_k + w)
    auto lin_step = [&](T xi, int k) -> T {
        sXb[lane] = lane < n ? xi : (T)0;
        const T ax = slot_dot(sXb, aRow, std::integral_constant<int, NR>(), (T)0);
        return lane < n ? ax + sBu[k * n + lane] : (T)0;
    };
    auto chain_step = [&](T &q, T &v, T u) {
        const T phi = wave_scan_up<T>(q);
        const T sg = L.cg * sin_f<T>(phi);
        const T Gj = wave_scan_down<T>(sg);
        const T acc = (u - L.kst * q - L.dmp * v - Gj) * L.invI;
        v = v + P.dt * acc;
        q = q + P.dt * v;
    };

    // forward pass: returns J; stores checkpoints when chk != 0
    auto forward = [&](bool chk, T &xi, T &qj, T &vj) -> T {
        tabulate();
        T J = 0;
        xi = (lin && lane < n) ? x0[lane] : (T)0;
        qj = (!lin && lane < d) ? x0[lane] : (T)0;
        vj = (!lin && lane < d) ? x0[d + lane] : (T)0;
        for (int k = 0; k < Tn; ++k) {
            if (chk && k % S == 0) {
                if (lin) {
                    if (lane < n) sChk[(k / S) * n + lane] = xi;
                } else if (lane < d) {
                    sChk[(k / S) * n + lane] = qj;
                    sChk[(k / S) * n + d + lane] = vj;
                }
            }
            const T u = input_at(k);
            if (lin) {
                xi = lin_step(xi, k);
                const T e = L.xg - xi, eu = L.ug - u;
                J += L.q * e * e + L.r * eu * eu;
                if (box) J += L.bq * box_pen(xi, L.lo, L.hi) + L.sq * box_out(xi, L.lo, L.hi);
            } else {
                chain_step(qj, vj, u);
                const T eq = L.gq - qj, ev = L.gv - vj, eu = L.gu - u;
                J += L.wq * eq * eq + L.wv * ev * ev + L.wr * eu * eu;
                if (box) {
                    J += L.bq * box_pen(qj, L.lo, L.hi) + L.bv * box_pen(vj, L.lov, L.hiv);
                    J += L.sq * box_out(qj, L.lo, L.hi) + L.sv * box_out(vj, L.lov, L.hiv);
                }
            }
        }
        if (lin) {
            const T e = L.xg - xi;
            J += L.qf * e * e;
        } else {
            const T eq = L.gq - qj, ev = L.gv - vj;
            J += L.wqf * eq * eq + L.wvf * ev * ev;
        }
        return wave_total<T>(J);
    };

    // states x_k0 .. x_{k1-1} of checkpoint segment sg, recomputed into seg
    auto recompute = [&](int sg, T *seg) {
        const int k0 = sg * S, k1 = min(k0 + S, Tn);
        T xi = 0, qj = 0, vj = 0;
        if (lin) {
            if (lane < n) xi = sChk[sg * n + lane];
        } else if (lane < d) {
            qj = sChk[sg * n + lane];
            vj = sChk[sg * n + d + lane];
        }
        for (int k = k0; k < k1; ++k) {
            if (lin) {
                if (lane < n) seg[(k - k0) * n + lane] = xi;
            } else if (lane < d) {
                seg[(k - k0) * n + lane] = qj;
                seg[(k - k0) * n + d + lane] = vj;
            }
            if (k + 1 < k1) {
                if (lin) {
                    xi = lin_step(xi, k);
                } else {
                    chain_step(qj, vj, input_at(k));
                }
            }
        }
    };

    // backward pass from the final state (wavefront 0's xT / qT, vT): fills
    // sG with dJ/dknots.  Both wavefronts call it: wavefront 0 walks the
    // segments backward, wavefront 1 recomputes one segment ahead of it.
    auto backward = [&](T xT, T qT, T vT) {
        for (int j = threadIdx.x; j < pm; j += 128) sG[j] = 0;
        T lam = 0, lq = 0, lv = 0;
        if (lin) {
            lam = (T)2 * (L.q + L.qf) * (xT - L.xg);
            if (box) lam += box_pen_grad(xT, L.lo, L.hi, L.bq);
        } else {
            lq = (T)2 * (L.wq + L.wqf) * (qT - L.gq);
            lv = (T)2 * (L.wv + L.wvf) * (vT - L.gv);
            if (box) {
                lq += box_pen_grad(qT, L.lo, L.hi, L.bq);
                lv += box_pen_grad(vT, L.lov, L.hiv, L.bv);
            }
        }
        // the two segment buffers (offsets from the LDS base, not a table
        // of pointers, so that their accesses compile to LDS operations)
        auto segbuf = [&](int b) { return sm + G.oSeg + (b ? (size_t)S * n : (size_t)0); };
        if (wave == 1) recompute(G.nchk - 1, segbuf((G.nchk - 1) & 1));
        __syncthreads();
        // dJ/du_k goes to knots a and b of step k with weights 1-c and c;
        // summed in registers while the knot pair stays, then added to sG
        int cur_a = -1, cur_b = -1;
        T gA = 0, gB = 0;
        auto flush = [&]() {
            if (cur_a >= 0 && lane < m) {
                sG[cur_a * m + lane] += gA;
                sG[cur_b * m + lane] += gB;
            }
        };
        for (int sg = G.nchk - 1; sg >= 0; --sg) {
            if (wave == 1) {
                if (sg > 0) recompute(sg - 1, segbuf((sg - 1) & 1));
            } else {
                const int k0 = sg * S, k1 = min(k0 + S, Tn);
                const T *sSeg = segbuf(sg & 1);
                for (int k = k1 - 1; k >= k0; --k) {
                    const Knot kn = knot_at(Tn, P.p, k);
                    const T c = sC[k];
                    const T u = input_at(k);
                    T gu;
                    if (lin) {
                        // B^T lambda and A^T lambda, lambda_i published by lane i
                        sXb[lane] = lane < n ? lam : (T)0;
                        const T bu = slot_dot(sXb, bCol, std::integral_constant<int, NR>(), (T)0);
                        const T ax = slot_dot(sXb, aCol, std::integral_constant<int, NR>(), (T)0);
                        gu = (T)2 * L.r * (u - L.ug) + bu;
                        if (k >= 1 && lane < n) {
                            const T xk = sSeg[(k - k0) * n + lane];
                            lam = (T)2 * L.q * (xk - L.xg) + ax;
                            if (box) lam += box_pen_grad(xk, L.lo, L.hi, L.bq);
                        }
                    } else {
                        const T qk = lane < d ? sSeg[(k - k0) * n + lane] : (T)0;
                        const T vk = lane < d ? sSeg[(k - k0) * n + d + lane] : (T)0;
                        const T phi = wave_scan_up<T>(qk);
                        const T Sv = wave_scan_down<T>(L.cg * cos_f<T>(phi));
                        const T mu = lv + P.dt * lq;
                        const T nu = mu * L.invI;
                        const T pf = wave_scan_up<T>(nu);
                        const T sn = Sv * nu;
                        const T R = wave_scan_down<T>(sn) - sn;
                        const T dadq = -L.kst * nu - (Sv * pf + R);
                        const T lq_n = lq + P.dt * dadq;
                        const T lv_n = mu - P.dt * L.dmp * nu;
                        gu = (T)2 * L.wr * (u - L.gu) + P.dt * nu;
                        if (k >= 1) {
                            lq = lq_n + (T)2 * L.wq * (qk - L.gq);
                            lv = lv_n + (T)2 * L.wv * (vk - L.gv);
                            if (box) {
                                lq += box_pen_grad(qk, L.lo, L.hi, L.bq);
                                lv += box_pen_grad(vk, L.lov, L.hiv, L.bv);
                            }
                        }
                    }
                    if (kn.a != cur_a) {  // uniform
                        flush();
                        cur_a = kn.a;
                        cur_b = kn.b;
                        gA = 0;
                        gB = 0;
                    }
                    gA += ((T)1 - c) * gu;
                    gB += c * gu;
                }
            }
            // segment sg - 1 recomputed, segment sg walked: the buffers swap
            __syncthreads();
        }
        if (wave == 0) flush();
        __syncthreads();
    };

    // wavefront 0 owns the forward passes; both take part in the backward
    // passes and the Adam updates (barriers between the phases)
    T xi = 0, qj = 0, vj = 0;
    if (!refine) {
        T J = 0;
        if (wave == 0) J = forward(true, xi, qj, vj);
        __syncthreads();  // checkpoints and input tables
        backward(xi, qj, vj);
        for (int j = threadIdx.x; j < pm; j += 128) dJ[(int64_t)j * ld + cand] = sG[j];
        if (cost && threadIdx.x == 0) cost[cand] = J;
        return;
    }
    // Adam (Kingma & Ba 2015), bias-corrected, clamp after each update
    const T b1 = (T)0.9, b2 = (T)0.999, eps = (T)1e-8;
    T b1t = 1, b2t = 1;
    T J0 = 0;  // cost of the entry knots by this kernel's own forward pass
    for (int t = 1; t <= steps; ++t) {
        if (wave == 0) {
            const T Jt = forward(true, xi, qj, vj);
            if (t == 1) J0 = Jt;
        }
        __syncthreads();  // checkpoints and input tables
        backward(xi, qj, vj);
        b1t *= b1;
        b2t *= b2;
        for (int j = threadIdx.x; j < pm; j += 128) {
            const T g = sG[j];
            const T m1 = b1 * sM1[j] + ((T)1 - b1) * g;
            const T m2 = b2 * sM2[j] + ((T)1 - b2) * g * g;
            sM1[j] = m1;
            sM2[j] = m2;
            const T mh = m1 / ((T)1 - b1t), vh = m2 / ((T)1 - b2t);
            T U = sU[j] - lr * mh / (sqrt(vh) + eps);
            const int i = j % m;
            U = U < P.umin[i] ? P.umin[i] : U;
            U = U > P.umax[i] ? P.umax[i] : U;
            sU[j] = U;
        }
        __syncthreads();
    }
    if (wave == 0) {
        // accept the refined knots only if they cost less: both costs come
        // from the same forward pass code (in FP32 the rollout kernels take
        // the hardware sine, this pass the library one, so cost_io is not
        // the value to compare against)
        const T Jn = forward(false, xi, qj, vj);
        if (Jn < J0) {  // uniform: Jn and J0 are wave sums
            for (int j = lane; j < pm; j += 64) knots_io[(int64_t)j * ld + cand] = sU[j];
            if (lane == 0) cost_io[cand] = Jn;
        }
    }
}

size_t grad_smem_bytes(int model, int n, int m, int T, int p, size_t esize) {
    return grad_plan(model, n, m, T, p).total * esize;
}

template <typename T>
hipError_t launch_grad(const ProbView<T> &P, int model, const T *x0, const T *knots, int64_t ncand,
                       int64_t ld, T *dJ, T *cost, int refine_steps, T lr, T *knots_io,
                       T *cost_io, hipStream_t s) {
    const GradPlan G = grad_plan(model, P.n, P.m, P.Tn, P.p);
    const size_t bytes = G.total * sizeof(T);
    auto go = [&](auto kernel) {
        if (bytes > 65536) {
            hipError_t e = hipFuncSetAttribute((const void *)kernel,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)bytes);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kernel, dim3((unsigned)ncand), dim3(128), bytes, s, P, G, x0, knots, ld,
                           dJ, cost, refine_steps, lr, knots_io, cost_io);
        return hipGetLastError();
    };
    if (model != EMPC_LINEAR) return go(adjoint_kernel<T, false, 4, 4>);
    // register operand lengths: n and m each rounded up to 16, 32 or 64
    const int nb = P.n <= 16 ? 16 : P.n <= 32 ? 32 : 64;
    const int mb = P.m <= 16 ? 16 : P.m <= 32 ? 32 : 64;
    switch (nb * 100 + mb) {
        case 1616: return go(adjoint_kernel<T, true, 16, 16>);
        case 3216: return go(adjoint_kernel<T, true, 32, 16>);
        case 3232: return go(adjoint_kernel<T, true, 32, 32>);
        case 6416: return go(adjoint_kernel<T, true, 64, 16>);
        case 6432: return go(adjoint_kernel<T, true, 64, 32>);
        default: return go(adjoint_kernel<T, true, 64, 64>);
    }
}
template hipError_t launch_grad<float>(const ProbView<float> &, int, const float *, const float *,
                                       int64_t, int64_t, float *, float *, int, float, float *,
                                       float *, hipStream_t);
template hipError_t launch_grad<double>(const ProbView<double> &, int, const double *,
                                        const double *, int64_t, int64_t, double *, double *, int,
                                        double, double *, double *, hipStream_t);

}  // namespace empc
