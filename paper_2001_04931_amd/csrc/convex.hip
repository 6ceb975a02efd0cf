// Parameterized small-matrix convex MPC on the GPU (gfx950): the paper's
// other method (Sec. IV-B small-matrix formulation, parameterized as in
// Sec. IV-E), for linear problems.  With z the knot vector, the states
// x_1..x_T = S z + v and the cost of eq. 3 is J(z) = z^T P z + 2 q^T z + c;
// the knot bounds make the MPC a box-constrained QP.
//  - qp_traj_kernel: S and v.  One workgroup per column: the response of
//    unit knot j from rest (column j of S, built step by step as the paper
//    describes, each row the previous one times A_d plus B_d in the knot's
//    proportions), and one workgroup for the free response v from x0 with
//    w_d; one thread per state row, the state exchanged through LDS each
//    step (the paper's own thread-per-state layout: the work is tiny).
//  - qp_gram_kernel: P = S^T Qb S + Phi^T Rb Phi, 16 x 16 output tiles with
//    the shared dimension T n staged through LDS; the input part in closed
//    form from the knot weights.  qp_lin_kernel: q and c.
//  - qp_box_kernel: the box QP by the projected Newton method (Bertsekas
//    1982): Newton steps of the quadratic restricted to the variables off
//    their bounds (Cholesky solves), an Armijo search along the projection
//    arc; one workgroup.
// Every step computes in FP64; inputs and outputs are in the problem dtype.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.hpp"

namespace empc {

namespace {

constexpr int TRAJ_THREADS = 128;  // >= the largest linear state count (80)
constexpr int QP_THREADS = 1024;
constexpr int QP_MAX_PM = 1024;    // one knot parameter per QP thread

// weight of knot a at step k (u_k = (1-c) U_idx1 + c U_idx2)
__device__ inline double knot_weight(int T, int p, int k, int a) {
    const Knot s = knot_at(T, p, k);
    const double c = (double)s.rem / (double)s.den;
    return (a == s.a ? 1.0 - c : 0.0) + (a == s.b ? c : 0.0);
}

template <typename T>
__global__ __launch_bounds__(TRAJ_THREADS) void qp_traj_kernel(ProbView<T> P,
                                                               const T *__restrict__ x0,
                                                               double *__restrict__ S,
                                                               double *__restrict__ v) {
    __shared__ double x[2][TRAJ_THREADS];
    const int n = P.n, m = P.m, pm = P.p * P.m, r = threadIdx.x;
    const int j = blockIdx.x;  // column; j == pm: the free response
    const bool free_resp = j == pm;
    const int aj = free_resp ? 0 : j / m, ij = free_resp ? 0 : j % m;
    if (r < n) x[0][r] = free_resp ? (double)x0[r] : 0.0;
    __syncthreads();
    for (int k = 0; k < P.Tn; ++k) {
        const double *xc = x[k & 1];
        if (r < n) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += (double)P.Ad[r * n + c] * xc[c];
            if (free_resp) {
                if (P.wd) s += (double)P.wd[r];
            } else {
                s += (double)P.Bd[r * m + ij] * knot_weight(P.Tn, P.p, k, aj);
            }
            x[(k + 1) & 1][r] = s;
            if (free_resp)
                v[(int64_t)k * n + r] = s;
            else
                S[((int64_t)k * n + r) * pm + j] = s;
        }
        __syncthreads();
    }
}

// weight of state row K = k n + r of the stacked cost: q_r (+ qf_r at x_T)
template <typename T>
__device__ inline double row_weight(const ProbView<T> &P, int K) {
    const int k = K / P.n, r = K % P.n;
    double w = (double)P.q[r];
    if (k == P.Tn - 1 && P.qf) w += (double)P.qf[r];
    return w;
}

// Partial Gram products over a slice of the stacked state rows (split K):
// blockIdx.z = slice; Ppart[z][i][j] = sum over the slice's rows K of
// w_K S[K][i] S[K][j].
constexpr int GRAM_SPLIT = 8;
template <typename T>
__global__ __launch_bounds__(256) void qp_gram_kernel(ProbView<T> P, const double *__restrict__ S,
                                                      double *__restrict__ Ppart) {
    __shared__ double As[16][17], Bs[16][17];
    const int pm = P.p * P.m, K = P.Tn * P.n;
    const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
    const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
    const int kb = (int)((int64_t)K * blockIdx.z / GRAM_SPLIT);
    const int ke = (int)((int64_t)K * (blockIdx.z + 1) / GRAM_SPLIT);
    double acc = 0.0;
    for (int k0 = kb; k0 < ke; k0 += 16) {
        // thread (ti, tj) stages row k0 + ti, columns i0 + tj / j0 + tj
        const int kr = k0 + ti;
        double a = 0.0, b = 0.0;
        if (kr < ke) {
            const double w = row_weight(P, kr);
            if (i0 + tj < pm) a = w * S[(int64_t)kr * pm + i0 + tj];
            if (j0 + tj < pm) b = S[(int64_t)kr * pm + j0 + tj];
        }
        As[ti][tj] = a;
        Bs[ti][tj] = b;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc += As[kk][ti] * Bs[kk][tj];
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i < pm && j < pm) Ppart[((int64_t)blockIdx.z * pm + i) * pm + j] = acc;
}

// P = the partial products summed in slice order, plus the input part
// sum_k w_k(knot of i) w_k(knot of j) r_input on matching inputs.
template <typename T>
__global__ __launch_bounds__(256) void qp_gram_sum_kernel(ProbView<T> P,
                                                          const double *__restrict__ Ppart,
                                                          T *__restrict__ Pout) {
    const int pm = P.p * P.m, m = P.m;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)pm * pm) return;
    const int i = (int)(e / pm), j = (int)(e % pm);
    double acc = 0.0;
#pragma unroll
    for (int z = 0; z < GRAM_SPLIT; ++z) acc += Ppart[(int64_t)z * pm * pm + e];
    if (i % m == j % m) {
        double s = 0.0;
        for (int k = 0; k < P.Tn; ++k)
            s += knot_weight(P.Tn, P.p, k, i / m) * knot_weight(P.Tn, P.p, k, j / m);
        acc += s * (double)P.r[i % m];
    }
    Pout[e] = (T)acc;
}

// q_i (block i < pm) and c (block pm): sums over the stacked state rows
// K = k n + r, spread over the workgroup's threads and reduced in LDS.
template <typename T>
__global__ __launch_bounds__(256) void qp_lin_kernel(ProbView<T> P, const double *__restrict__ S,
                                                     const double *__restrict__ v,
                                                     T *__restrict__ qout, T *__restrict__ cout) {
    __shared__ double part[256];
    const int pm = P.p * P.m, K = P.Tn * P.n, m = P.m;
    const int i = blockIdx.x;
    double s = 0.0;
    if (i < pm) {
        for (int kr = threadIdx.x; kr < K; kr += blockDim.x) {
            const double g = P.xg ? (double)P.xg[kr % P.n] : 0.0;
            s += S[(int64_t)kr * pm + i] * row_weight(P, kr) * (v[kr] - g);
        }
        if (P.ug && threadIdx.x == 0) {
            double wsum = 0.0;
            for (int k = 0; k < P.Tn; ++k) wsum += knot_weight(P.Tn, P.p, k, i / m);
            s -= wsum * (double)P.r[i % m] * (double)P.ug[i % m];
        }
    } else {
        for (int kr = threadIdx.x; kr < K; kr += blockDim.x) {
            const double e = v[kr] - (P.xg ? (double)P.xg[kr % P.n] : 0.0);
            s += row_weight(P, kr) * e * e;
        }
        if (P.ug)
            for (int ii = threadIdx.x; ii < m; ii += blockDim.x)
                s += (double)P.Tn * (double)P.r[ii] * (double)P.ug[ii] * (double)P.ug[ii];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (i < pm)
            qout[i] = (T)part[0];
        else
            *cout = (T)part[0];
    }
}

// Adam refinement of k parents on the quadratic J(z) = z^T P z + 2 q^T z + c
// of a linear problem without the state box: its gradient 2 (P z + q) is
// the rollout cost's gradient exactly (the value the adjoint builds step by
// step), so an Adam step is one product with the symmetric P.  The Adam of
// the adjoint kernel: moments from zero, bias correction, a clamp to the
// knot bounds after every update, and the result kept only if its cost (by
// the same quadratic) is below the entry cost.  The parents are read from
// the population (parameter j of parent b at knots[j ld + idx[b]]) and
// written, refined or not, to Z: [pm][k]; cost_io [k] takes the refined
// costs.  One workgroup per parent, up to QP_MAX_PM parameters.  When P fits
// in the workgroup's LDS (dynamic size pm^2 elements) it is staged there
// once and every product reads it from LDS; otherwise from global memory.
// LS: rows per lane of the product (pm <= 64 LS), a compile-time count so
// the slot loops carry no runtime guards.
constexpr int REF_THREADS = 256, REF_WAVES = REF_THREADS / 64;
constexpr size_t REF_LDS_MAX = 96 * 1024;  // bytes of P staged in LDS at most
template <typename T, int LS>
__global__ __launch_bounds__(REF_THREADS) void qp_refine_kernel(
    int pm, int m, int k, const T *__restrict__ Pg, const T *__restrict__ qv,
    const T *__restrict__ cp, const T *__restrict__ umin, const T *__restrict__ umax, int steps,
    T lr, const T *__restrict__ knots, int64_t ld, const int64_t *__restrict__ idx,
    T *__restrict__ Z, T *__restrict__ cost_io, int p_in_lds) {
    constexpr int REF_SLOTS = (64 * LS + REF_THREADS - 1) / REF_THREADS;
    constexpr int NP = 64 * LS;  // parameters at most
    extern __shared__ __align__(16) unsigned char ref_smem[];
    // the knots in two buffers: an Adam step writes the other one, so one
    // barrier separates it from the next product's reads
    __shared__ T zbuf[2][NP];
    int cur = 0;
    __shared__ double part[REF_WAVES][NP];
    __shared__ double red[REF_WAVES];
    const int tid = threadIdx.x, b = blockIdx.x, lane = tid & 63, wv = tid >> 6;
    T *Pl = (T *)ref_smem;
    const int64_t src = idx[b];
    for (int i = tid; i < pm; i += REF_THREADS) zbuf[0][i] = knots[(int64_t)i * ld + src];
    if (p_in_lds) {
        // P is copied as a flat array: 16-byte pieces, sixteen loads in
        // flight per thread, then their stores (a 140 x 140 FP32 form takes
        // two such rounds per thread); the scalar tail, and every element
        // when P is not 16-byte aligned, one at a time
        typedef T v16 __attribute__((ext_vector_type(16 / sizeof(T))));
        constexpr int W = 16 / sizeof(T);
        const int tot = pm * pm;
        const int nv = (reinterpret_cast<uintptr_t>(Pg) & 15) == 0 ? tot / W : 0;
        const v16 *Pv = reinterpret_cast<const v16 *>(Pg);
        v16 *Lv = reinterpret_cast<v16 *>(Pl);
        for (int e0 = tid; e0 < nv; e0 += 16 * REF_THREADS) {
            v16 t16[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * REF_THREADS;
                if (e < nv) t16[u] = Pv[e];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * REF_THREADS;
                if (e < nv) Lv[e] = t16[u];
            }
        }
        for (int e = nv * W + tid; e < tot; e += REF_THREADS) Pl[e] = Pg[e];
    }
    // this thread's parameters: linear term and bounds in registers
    T qr[REF_SLOTS], lo[REF_SLOTS], hi[REF_SLOTS];
#pragma unroll
    for (int sl = 0; sl < REF_SLOTS; ++sl) {
        const int i = tid + REF_THREADS * sl;
        qr[sl] = i < pm ? qv[i] : (T)0;
        lo[sl] = i < pm ? umin[i % m] : (T)0;
        hi[sl] = i < pm ? umax[i % m] : (T)0;
    }
    const double c0 = (double)*cp;
    __syncthreads();
    // y = P z: wavefront w sums the columns j of its quarter of 0..pm-1
    // for every row i = lane + 64 s (P symmetric: column j read as row j,
    // contiguous over the lanes), the quarters added in LDS; then, when
    // asked for (the first and the last product: the Adam steps in between
    // need only the gradient), J = sum_i z_i (y_i + 2 q_i) + c over the
    // workgroup.  Each thread returns y for its parameters
    // i = tid + REF_THREADS s.
    double y[REF_SLOTS];
    const int jb = pm * wv / REF_WAVES, je = pm * (wv + 1) / REF_WAVES;
    auto product = [&](bool want_J) {
        // partial sums in the problem's precision, eight columns per pass
        // so that their loads are in flight together
        T acc[LS];
#pragma unroll
        for (int sl = 0; sl < LS; ++sl) acc[sl] = 0;
        // P from LDS or from global memory, each loop on its own pointer so
        // that the LDS one compiles to LDS reads
        auto columns = [&](const T *Pp) {
#pragma unroll 8
            for (int j = jb; j < je; ++j) {
                const T zj = zbuf[cur][j];
                const T *row = Pp + (int64_t)j * pm;
#pragma unroll
                for (int sl = 0; sl < LS; ++sl) {
                    const int i = lane + 64 * sl;
                    acc[sl] += (i < pm ? row[i] : (T)0) * zj;
                }
            }
        };
        if (p_in_lds)
            columns(Pl);
        else
            columns(Pg);
#pragma unroll
        for (int sl = 0; sl < LS; ++sl) {
            const int i = lane + 64 * sl;
            if (i < pm) part[wv][i] = (double)acc[sl];
        }
        __syncthreads();
        double pj = 0.0;
#pragma unroll
        for (int sl = 0; sl < REF_SLOTS; ++sl) {
            const int i = tid + REF_THREADS * sl;
            double a = 0.0;
            if (i < pm) {
#pragma unroll
                for (int w2 = 0; w2 < REF_WAVES; ++w2) a += part[w2][i];
                pj += (double)zbuf[cur][i] * (a + 2.0 * (double)qr[sl]);
            }
            y[sl] = a;
        }
        if (!want_J) return 0.0;  // uniform over the workgroup
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) pj += __shfl_xor(pj, o, 64);
        if (lane == 0) red[wv] = pj;
        __syncthreads();
        double J = c0;
#pragma unroll
        for (int w2 = 0; w2 < REF_WAVES; ++w2) J += red[w2];
        return J;
    };
    const T b1 = (T)0.9, b2 = (T)0.999, eps = (T)1e-8;
    T b1t = 1, b2t = 1;
    T m1[REF_SLOTS], m2[REF_SLOTS];
#pragma unroll
    for (int sl = 0; sl < REF_SLOTS; ++sl) m1[sl] = m2[sl] = 0;
    double J0 = 0.0;
    for (int t = 1; t <= steps; ++t) {
        const double Jt = product(t == 1);
        if (t == 1) J0 = Jt;
        b1t *= b1;
        b2t *= b2;
        T U[REF_SLOTS];
#pragma unroll
        for (int sl = 0; sl < REF_SLOTS; ++sl) {
            const int i = tid + REF_THREADS * sl;
            if (i < pm) {
                const T g = (T)(2.0 * (y[sl] + (double)qr[sl]));
                m1[sl] = b1 * m1[sl] + ((T)1 - b1) * g;
                m2[sl] = b2 * m2[sl] + ((T)1 - b2) * g * g;
                const T mh = m1[sl] / ((T)1 - b1t), vh = m2[sl] / ((T)1 - b2t);
                T u = zbuf[cur][i] - lr * mh / (sqrt(vh) + eps);
                u = u < lo[sl] ? lo[sl] : u;
                u = u > hi[sl] ? hi[sl] : u;
                U[sl] = u;
            }
        }
        // every read of the current buffer lies before this step's product
        // barrier or is this thread's own; the next product reads the other
#pragma unroll
        for (int sl = 0; sl < REF_SLOTS; ++sl) {
            const int i = tid + REF_THREADS * sl;
            if (i < pm) zbuf[cur ^ 1][i] = U[sl];
        }
        cur ^= 1;
        __syncthreads();
    }
    const double Jn = product(true);
    const bool keep = steps > 0 && Jn < J0;  // uniform over the workgroup
    for (int i = tid; i < pm; i += REF_THREADS)
        Z[(int64_t)i * k + b] = keep ? zbuf[cur][i] : knots[(int64_t)i * ld + src];
    if (keep && tid == 0) cost_io[b] = (T)Jn;
}

// sum over the workgroup (every thread gets it)
__device__ inline double block_sum(double x, double *red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = QP_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// max over the workgroup (every thread gets it)
__device__ inline double block_max(double x, double *red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = QP_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Box QP min f(z) = z^T P z + 2 q^T z, lo <= z <= hi, by Bertsekas' projected
// Newton method (SIAM J. Control Optim. 20, 1982): with g = 2 (P z + q) and
// w = |z - clip(z - g)|_inf, the variables within min(eps, w) of a bound
// whose gradient points out of the box are held on a scaled gradient step,
// the rest take the Newton step of the reduced quadratic (a Cholesky solve
// of P on the free variables), and the step is cut back along the
// projection arc until the Armijo condition f(z) - f(z') >= sigma g^T (z -
// z') holds.  Globally convergent for a positive definite P; once the active
// set is the optimal one the full Newton step lands on the minimizer.
template <typename T>
__global__ __launch_bounds__(QP_THREADS) void qp_box_kernel(
    int pm, int m, const T *__restrict__ umin, const T *__restrict__ umax,
    const T *__restrict__ Pm, const T *__restrict__ qv, const T *__restrict__ cp, int max_iter,
    double *__restrict__ H, T *__restrict__ zout, T *__restrict__ cost, int *__restrict__ info) {
    __shared__ double z[QP_MAX_PM], d[QP_MAX_PM], y[QP_MAX_PM], red[QP_THREADS];
    __shared__ int act[QP_MAX_PM], idx[QP_MAX_PM], s_nfree;
    const int i = threadIdx.x;
    const bool mine = i < pm;
    const double lo = mine ? (double)umin[i % m] : 0.0, hi = mine ? (double)umax[i % m] : 0.0;
    const double qi = mine ? (double)qv[i] : 0.0;
    const double pii = mine ? (double)Pm[(int64_t)i * pm + i] : 1.0;
    auto clip = [&](double v) { return v < lo ? lo : (v > hi ? hi : v); };
    // (P v)_i for v in LDS
    auto pdot = [&](const double *v) {
        double s = 0.0;
        if (mine)
            for (int j = 0; j < pm; ++j) s += (double)Pm[(int64_t)i * pm + j] * v[j];
        return s;
    };
    if (mine) z[i] = clip(0.0);
    __syncthreads();
    double pz = pdot(z);
    double f = block_sum(mine ? z[i] * (pz + 2.0 * qi) : 0.0, red);
    int it = 0, converged = 0;
    const double eps0 = 1e-3;
    for (; it < max_iter; ++it) {
        const double g = mine ? 2.0 * (pz + qi) : 0.0;
        const double w = block_max(mine ? fabs(z[i] - clip(z[i] - g)) : 0.0, red);
        const double gs = block_max(mine ? fabs(g) : 0.0, red);
        if (w <= 1e-14 * (1.0 + gs)) {
            converged = 1;
            break;
        }
        const double eps = w < eps0 ? w : eps0;
        int a = 0;
        if (mine) a = (z[i] <= lo + eps && g > 0.0) || (z[i] >= hi - eps && g < 0.0);
        if (mine) act[i] = a;
        __syncthreads();
        if (i == 0) {
            int c = 0;
            for (int t = 0; t < pm; ++t)
                if (!act[t]) idx[c++] = t;
            s_nfree = c;
        }
        __syncthreads();
        const int nf = s_nfree;
        // Newton step on the free variables: P_FF d_F = -(P z + q)_F
        for (int e = i; e < nf * nf; e += QP_THREADS) {
            const int r = e / nf, c = e % nf;
            H[e] = (double)Pm[(int64_t)idx[r] * pm + idx[c]];
        }
        if (mine && !a) d[i] = -(pz + qi);  // gathered below
        if (mine && a) d[i] = -g / (2.0 * pii);
        __syncthreads();
        if (i < nf) y[i] = d[idx[i]];
        __syncthreads();
        for (int k = 0; k < nf; ++k) {
            if (i == 0) H[k * nf + k] = sqrt(H[k * nf + k]);
            __syncthreads();
            const double dk = H[k * nf + k];
            for (int r = k + 1 + i; r < nf; r += QP_THREADS) H[r * nf + k] /= dk;
            __syncthreads();
            const int wdt = nf - k - 1;
            for (int e = i; e < wdt * wdt; e += QP_THREADS) {
                const int r = k + 1 + e / wdt, c = k + 1 + e % wdt;
                if (c <= r) H[r * nf + c] -= H[r * nf + k] * H[c * nf + k];
            }
            __syncthreads();
        }
        for (int k = 0; k < nf; ++k) {
            if (i == 0) y[k] /= H[k * nf + k];
            __syncthreads();
            for (int r = k + 1 + i; r < nf; r += QP_THREADS) y[r] -= H[r * nf + k] * y[k];
            __syncthreads();
        }
        for (int k = nf - 1; k >= 0; --k) {
            if (i == 0) y[k] /= H[k * nf + k];
            __syncthreads();
            for (int r = i; r < k; r += QP_THREADS) y[r] -= H[k * nf + r] * y[k];
            __syncthreads();
        }
        if (i < nf) d[idx[i]] = y[i];
        __syncthreads();
        // Armijo search along the projection arc
        const double z_old = mine ? z[i] : 0.0;
        double alpha = 1.0, pz_new = pz, f_new = f;
        bool moved = false;
        for (int ls = 0; ls < 60; ++ls) {
            const double zt = mine ? clip(z_old + alpha * d[i]) : 0.0;
            __syncthreads();
            if (mine) y[i] = zt;
            __syncthreads();
            pz_new = pdot(y);
            f_new = block_sum(mine ? zt * (pz_new + 2.0 * qi) : 0.0, red);
            const double dec = block_sum(mine ? g * (z_old - zt) : 0.0, red);
            if (f - f_new >= 1e-4 * dec) {
                moved = true;
                break;
            }
            alpha *= 0.5;
        }
        if (!moved) {  // no decrease left at rounding level
            converged = 1;
            break;
        }
        // a step below rounding of z: nothing left to gain
        const double step = block_max(mine ? fabs(y[i] - z_old) : 0.0, red);
        const double zmax = block_max(mine ? fabs(z_old) : 0.0, red);
        if (mine) z[i] = y[i];
        pz = pz_new;
        f = f_new;
        __syncthreads();
        if (step <= 1e-15 * (1.0 + zmax)) {
            converged = 1;
            ++it;
            break;
        }
    }
    if (mine) zout[i] = (T)z[i];
    if (i == 0) {
        *cost = (T)(f + (double)*cp);
        info[0] = it;
        info[1] = converged;
    }
}

}  // namespace

// workspace of the form, in doubles: S [T n][pm], v [T n], the split-K
// partial Gram products [GRAM_SPLIT][pm][pm]; the box solver adds H [pm][pm]
static size_t form_doubles(int n, int T, int pm) {
    const size_t S = (size_t)T * n * pm, v = (size_t)T * n;
    const size_t G = (size_t)GRAM_SPLIT * pm * pm;
    return (S + 31) / 32 * 32 + (v + 31) / 32 * 32 + (G + 31) / 32 * 32;
}

size_t qp_workspace_bytes(int n, int T, int pm) {
    return (form_doubles(n, T, pm) + (size_t)pm * pm) * sizeof(double);
}

template <typename T>
hipError_t launch_qp_form(const ProbView<T> &P, const T *x0, void *ws, T *Pout, T *qout, T *cout,
                          hipStream_t s) {
    const int pm = P.p * P.m, n = P.n;
    double *S = (double *)ws;
    double *v = S + ((size_t)P.Tn * n * pm + 31) / 32 * 32;
    double *Gp = v + ((size_t)P.Tn * n + 31) / 32 * 32;
    hipLaunchKernelGGL(qp_traj_kernel<T>, dim3(pm + 1), dim3(TRAJ_THREADS), 0, s, P, x0, S, v);
    const unsigned tiles = (unsigned)((pm + 15) / 16);
    hipLaunchKernelGGL(qp_gram_kernel<T>, dim3(tiles, tiles, GRAM_SPLIT), dim3(256), 0, s, P, S,
                       Gp);
    hipLaunchKernelGGL(qp_gram_sum_kernel<T>, dim3((unsigned)(((int64_t)pm * pm + 255) / 256)),
                       dim3(256), 0, s, P, Gp, Pout);
    hipLaunchKernelGGL(qp_lin_kernel<T>, dim3(pm + 1), dim3(256), 0, s, P, S, v, qout, cout);
    return hipGetLastError();
}

size_t qp_form_bytes(int n, int T, int pm) { return form_doubles(n, T, pm) * sizeof(double); }

template <typename T>
hipError_t launch_qp_refine(const ProbView<T> &P, const T *Pm, const T *q, const T *c,
                            const T *knots, int64_t ld, const int64_t *idx, T *Z, int k,
                            int steps, T lr, T *cost_io, hipStream_t s) {
    const int pm = P.p * P.m;
    const size_t bytes = (size_t)pm * pm * sizeof(T);
    const int in_lds = bytes <= REF_LDS_MAX ? 1 : 0;
    const size_t dyn = in_lds ? bytes : 0;
    auto go = [&](auto kernel) {
        if (dyn > 65536) {
            const hipError_t e = hipFuncSetAttribute((const void *)kernel,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)dyn);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kernel, dim3(k), dim3(REF_THREADS), dyn, s, pm, P.m, k, Pm, q, c,
                           P.umin, P.umax, steps, lr, knots, ld, idx, Z, cost_io, in_lds);
        return hipGetLastError();
    };
    if (pm <= 64) return go(qp_refine_kernel<T, 1>);
    if (pm <= 128) return go(qp_refine_kernel<T, 2>);
    if (pm <= 256) return go(qp_refine_kernel<T, 4>);
    if (pm <= 512) return go(qp_refine_kernel<T, 8>);
    return go(qp_refine_kernel<T, 16>);
}
template hipError_t launch_qp_refine<float>(const ProbView<float> &, const float *, const float *,
                                            const float *, const float *, int64_t,
                                            const int64_t *, float *, int, int, float, float *,
                                            hipStream_t);
template hipError_t launch_qp_refine<double>(const ProbView<double> &, const double *,
                                             const double *, const double *, const double *,
                                             int64_t, const int64_t *, double *, int, int, double,
                                             double *, hipStream_t);

template <typename T>
hipError_t launch_qp_solve(const ProbView<T> &P, const T *Pm, const T *q, const T *c, void *ws,
                           int max_iter, T *z, T *cost, int *info, hipStream_t s) {
    const int pm = P.p * P.m, n = P.n;
    double *H = (double *)ws + form_doubles(n, P.Tn, pm);
    hipLaunchKernelGGL(qp_box_kernel<T>, dim3(1), dim3(QP_THREADS), 0, s, pm, P.m, P.umin, P.umax,
                       Pm, q, c, max_iter, H, z, cost, info);
    return hipGetLastError();
}

template hipError_t launch_qp_form<float>(const ProbView<float> &, const float *, void *, float *,
                                          float *, float *, hipStream_t);
template hipError_t launch_qp_form<double>(const ProbView<double> &, const double *, void *,
                                           double *, double *, double *, hipStream_t);
template hipError_t launch_qp_solve<float>(const ProbView<float> &, const float *, const float *,
                                           const float *, void *, int, float *, float *, int *,
                                           hipStream_t);
template hipError_t launch_qp_solve<double>(const ProbView<double> &, const double *,
                                            const double *, const double *, void *, int, double *,
                                            double *, int *, hipStream_t);

}  // namespace empc

using namespace empc;

empc_status empc_validate_problem_internal(const empc_problem *P);
empc_status empc_fail_internal(empc_status s, const char *msg);

namespace {

empc_status check_qp_problem(const empc_problem *P) {
    empc_status st = empc_validate_problem_internal(P);
    if (st) return st;
    if (P->model != EMPC_LINEAR)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "the convex form needs a linear model");
    if (P->qb) return empc_fail_internal(EMPC_EUNSUPPORTED, "the state box penalty is not quadratic");
    if (P->Q || P->R || P->Qf)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "the convex form takes diagonal weights");
    if (P->p * P->m > QP_MAX_PM)
        return empc_fail_internal(EMPC_EUNSUPPORTED, "more than 1024 knot parameters");
    return EMPC_OK;
}

empc_status qp_launched(hipError_t e) {
    if (e == hipSuccess) return EMPC_OK;
    return empc_fail_internal(EMPC_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t empc_qp_workspace_bytes(const empc_problem *prob) {
    if (check_qp_problem(prob)) return 0;
    return qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m);
}

empc_status empc_qp_form(const empc_problem *prob, const void *x0, void *workspace,
                         size_t ws_bytes, void *P, void *q, void *c, void *stream) {
    empc_status st = check_qp_problem(prob);
    if (st) return st;
    if (!x0 || !P || !q || !c) return empc_fail_internal(EMPC_EINVAL, "x0, P, q and c are required");
    if (!workspace || ws_bytes < qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m))
        return empc_fail_internal(EMPC_EWORKSPACE, "convex workspace too small");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qp_launched(e);
    hipStream_t s = (hipStream_t)stream;
    if (prob->dtype == EMPC_F32)
        e = launch_qp_form<float>(view_of<float>(*prob), (const float *)x0, workspace, (float *)P,
                                  (float *)q, (float *)c, s);
    else
        e = launch_qp_form<double>(view_of<double>(*prob), (const double *)x0, workspace,
                                   (double *)P, (double *)q, (double *)c, s);
    return qp_launched(e);
}

empc_status empc_qp_solve(const empc_problem *prob, const void *P, const void *q, const void *c,
                          void *workspace, size_t ws_bytes, int32_t max_iter, void *z, void *cost,
                          int32_t *info, void *stream) {
    empc_status st = check_qp_problem(prob);
    if (st) return st;
    if (!P || !q || !c || !z || !cost || !info)
        return empc_fail_internal(EMPC_EINVAL, "P, q, c, z, cost and info are required");
    if (max_iter < 1) return empc_fail_internal(EMPC_EINVAL, "max_iter must be >= 1");
    if (!workspace || ws_bytes < qp_workspace_bytes(prob->n, prob->T, prob->p * prob->m))
        return empc_fail_internal(EMPC_EWORKSPACE, "convex workspace too small");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qp_launched(e);
    hipStream_t s = (hipStream_t)stream;
    if (prob->dtype == EMPC_F32)
        e = launch_qp_solve<float>(view_of<float>(*prob), (const float *)P, (const float *)q,
                                   (const float *)c, workspace, max_iter, (float *)z,
                                   (float *)cost, (int *)info, s);
    else
        e = launch_qp_solve<double>(view_of<double>(*prob), (const double *)P, (const double *)q,
                                    (const double *)c, workspace, max_iter, (double *)z,
                                    (double *)cost, (int *)info, s);
    return qp_launched(e);
}

}  // extern "C"
