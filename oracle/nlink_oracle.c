/*
 * N-link planar robot oracle (FP64, single-threaded).  TEST INFRASTRUCTURE
 * ONLY: loaded by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg, never by the HIP library.
 *
 * The robot of the paper's convex-solver and EMPC experiments (Sec. IV-F
 * setup, Sec. VI-A): N revolute joints in a chain whose plane is
 * perpendicular to gravity (no gravity torque), canonical dynamics
 *     M(q) qdd + C(q, qd) + b qd = tau
 * with viscous damping b.  Reading taken here: each link is massless with a
 * point mass m_i at its far end (the single pendulum of eq. 5 is that case
 * for N = 1), joint angles relative, q_1 measured from a fixed axis.
 *
 * Written from Lagrangian mechanics, not from a recursive algorithm:
 *  - mass point i sits at p_i = sum_{j<=i} l_j (cos phi_j, sin phi_j),
 *    phi_j = q_1 + ... + q_j, so dp_i/dq_k = sum_{j=k..i} l_j (-sin, cos)(phi_j)
 *    and the kinetic energy 1/2 qd^T M qd gives
 *      M_kl = sum_{j>=k} sum_{j'>=l} l_j l_j' mu_max(j,j') cos(phi_j - phi_j'),
 *    mu_r = sum_{i>=r} m_i (the mass at or beyond the end of link r);
 *  - C_k = sum_{i,j} Gamma_kij qd_i qd_j with the Christoffel symbols
 *    Gamma_kij = 1/2 (dM_kj/dq_i + dM_ki/dq_j - dM_ij/dq_k), the derivatives
 *    of M written out from the cosine sum above;
 *  - qdd = M^-1 (tau - C - b qd) by Gaussian elimination.
 * Every function is written over complex numbers so that the Jacobian of the
 * state derivative can be taken by the complex step (Squire & Trapp 1998):
 * df/dx_s = Im f(x + i h e_s) / h with h = 1e-30, exact to rounding because
 * no difference of nearby values is formed.
 *
 * Parity pins (tests): the two-link closed form of M and C of the robotics
 * textbooks (point masses), eq. 5 without gravity for one link, the kinetic
 * energy from the mass points' velocities against 1/2 qd^T M qd, energy
 * conservation of the undamped, unforced robot, power balance, and central
 * differences of the state derivative against the complex-step Jacobian.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define NL_MAX 16

/* mu_r = sum_{i>=r} m_i */
static void tail_masses(int N, const double *mass, double *mu) {
    double s = 0.0;
    for (int r = N - 1; r >= 0; --r) {
        s += mass[r];
        mu[r] = s;
    }
}

/* M(q) and dM[s][k][l] = dM_kl/dq_s, complex arguments */
static void mass_matrix_c(int N, const double *mass, const double *len, const cplx *q, cplx *M,
                          cplx *dM) {
    double mu[NL_MAX];
    cplx phi[NL_MAX];
    tail_masses(N, mass, mu);
    cplx acc = 0;
    for (int j = 0; j < N; ++j) {
        acc += q[j];
        phi[j] = acc;
    }
    for (int k = 0; k < N; ++k)
        for (int l = 0; l < N; ++l) {
            cplx s = 0;
            for (int j = k; j < N; ++j)
                for (int jp = l; jp < N; ++jp) {
                    int hi = j > jp ? j : jp;
                    s += len[j] * len[jp] * mu[hi] * ccos(phi[j] - phi[jp]);
                }
            M[k * N + l] = s;
        }
    if (!dM) return;
    /* d cos(phi_j - phi_j')/dq_s = -sin(phi_j - phi_j') ([s<=j] - [s<=j']) */
    for (int s = 0; s < N; ++s)
        for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l) {
                cplx acc2 = 0;
                for (int j = k; j < N; ++j)
                    for (int jp = l; jp < N; ++jp) {
                        int dj = (s <= j) - (s <= jp);
                        if (!dj) continue;
                        int hi = j > jp ? j : jp;
                        acc2 -= len[j] * len[jp] * mu[hi] * csin(phi[j] - phi[jp]) * (double)dj;
                    }
                dM[(s * N + k) * N + l] = acc2;
            }
}

/* C(q, qd) by the Christoffel symbols of M */
static void coriolis_c(int N, const cplx *dM, const cplx *qd, cplx *C) {
    for (int k = 0; k < N; ++k) {
        cplx s = 0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                cplx g = 0.5 * (dM[(i * N + k) * N + j] + dM[(j * N + k) * N + i] -
                                dM[(k * N + i) * N + j]);
                s += g * qd[i] * qd[j];
            }
        C[k] = s;
    }
}

/* solve A y = r (A n x n, copied) by Gaussian elimination without pivoting:
 * A = M(q) is symmetric positive definite */
static void solve_c(int n, const cplx *A_in, const cplx *r, cplx *y) {
    cplx A[NL_MAX * NL_MAX], b[NL_MAX];
    memcpy(A, A_in, sizeof(cplx) * n * n);
    memcpy(b, r, sizeof(cplx) * n);
    for (int c = 0; c < n; ++c)
        for (int rr = c + 1; rr < n; ++rr) {
            cplx f = A[rr * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[rr * n + k] -= f * A[c * n + k];
            b[rr] -= f * b[c];
        }
    for (int c = n - 1; c >= 0; --c) {
        cplx s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * y[k];
        y[c] = s / A[c * n + c];
    }
}

/* state derivative f(x, tau) = [qd; qdd], x = [q; qd] (2N), complex */
static void deriv_c(int N, const double *mass, const double *len, double b, const cplx *x,
                    const cplx *tau, cplx *f) {
    cplx M[NL_MAX * NL_MAX], C[NL_MAX], r[NL_MAX], qdd[NL_MAX];
    cplx *dM = (cplx *)malloc(sizeof(cplx) * N * N * N);
    mass_matrix_c(N, mass, len, x, M, dM);
    coriolis_c(N, dM, x + N, C);
    free(dM);
    for (int k = 0; k < N; ++k) r[k] = tau[k] - C[k] - b * x[N + k];
    solve_c(N, M, r, qdd);
    for (int k = 0; k < N; ++k) {
        f[k] = x[N + k];
        f[N + k] = qdd[k];
    }
}

static int bad_n(int N) { return N < 1 || N > NL_MAX; }

/* ---------------------------------------------------------------------------
 * Real-valued entry points. */

int or_nlink_mass_matrix(int N, const double *mass, const double *len, const double *q,
                         double *M, double *C_out, const double *qd) {
    if (bad_n(N)) return 1;
    cplx qc[NL_MAX], Mc[NL_MAX * NL_MAX], qdc[NL_MAX], Cc[NL_MAX];
    for (int i = 0; i < N; ++i) qc[i] = q[i];
    cplx *dM = (cplx *)malloc(sizeof(cplx) * N * N * N);
    mass_matrix_c(N, mass, len, qc, Mc, dM);
    for (int i = 0; i < N * N; ++i) M[i] = creal(Mc[i]);
    if (C_out && qd) {
        for (int i = 0; i < N; ++i) qdc[i] = qd[i];
        coriolis_c(N, dM, qdc, Cc);
        for (int i = 0; i < N; ++i) C_out[i] = creal(Cc[i]);
    }
    free(dM);
    return 0;
}

/* kinetic energy from the velocities of the mass points (no M involved):
 * v_i = sum_{j<=i} l_j omega_j (-sin phi_j, cos phi_j), omega_j = qd_1+..+qd_j */
double or_nlink_kinetic(int N, const double *mass, const double *len, const double *q,
                        const double *qd) {
    double phi = 0, om = 0, vx = 0, vy = 0, e = 0;
    for (int i = 0; i < N; ++i) {
        phi += q[i];
        om += qd[i];
        vx += -len[i] * om * sin(phi);
        vy += len[i] * om * cos(phi);
        e += 0.5 * mass[i] * (vx * vx + vy * vy);
    }
    return e;
}

int or_nlink_deriv(int N, const double *mass, const double *len, double b, const double *x,
                   const double *tau, double *f) {
    if (bad_n(N)) return 1;
    cplx xc[2 * NL_MAX], tc[NL_MAX], fc[2 * NL_MAX];
    for (int i = 0; i < 2 * N; ++i) xc[i] = x[i];
    for (int i = 0; i < N; ++i) tc[i] = tau[i];
    deriv_c(N, mass, len, b, xc, tc, fc);
    for (int i = 0; i < 2 * N; ++i) f[i] = creal(fc[i]);
    return 0;
}

/* Jacobians of f at (x, tau) by the complex step: A (2N x 2N) = df/dx,
 * B (2N x N) = df/dtau, row-major; f0 = f(x, tau). */
int or_nlink_jacobian(int N, const double *mass, const double *len, double b, const double *x,
                      const double *tau, double *A, double *B, double *f0) {
    if (bad_n(N)) return 1;
    const double h = 1e-30;
    const int n = 2 * N;
    cplx xc[2 * NL_MAX], tc[NL_MAX], fc[2 * NL_MAX];
    or_nlink_deriv(N, mass, len, b, x, tau, f0);
    for (int s = 0; s < n + N; ++s) {
        for (int i = 0; i < n; ++i) xc[i] = x[i];
        for (int i = 0; i < N; ++i) tc[i] = tau[i];
        if (s < n)
            xc[s] += I * h;
        else
            tc[s - n] += I * h;
        deriv_c(N, mass, len, b, xc, tc, fc);
        for (int r = 0; r < n; ++r) {
            double d = cimag(fc[r]) / h;
            if (s < n)
                A[r * n + s] = d;
            else
                B[r * N + (s - n)] = d;
        }
    }
    return 0;
}

/* The simulated robot: `substeps` classical Runge-Kutta steps of length
 * dt / substeps with tau held constant (zero-order hold), from x to x_next. */
int or_nlink_rk4(int N, const double *mass, const double *len, double b, const double *x,
                 const double *tau, double dt, int substeps, double *x_next) {
    if (bad_n(N) || substeps < 1) return 1;
    const int n = 2 * N;
    const double h = dt / substeps;
    double y[2 * NL_MAX], k1[2 * NL_MAX], k2[2 * NL_MAX], k3[2 * NL_MAX], k4[2 * NL_MAX],
        t[2 * NL_MAX];
    memcpy(y, x, sizeof(double) * n);
    for (int s = 0; s < substeps; ++s) {
        or_nlink_deriv(N, mass, len, b, y, tau, k1);
        for (int i = 0; i < n; ++i) t[i] = y[i] + 0.5 * h * k1[i];
        or_nlink_deriv(N, mass, len, b, t, tau, k2);
        for (int i = 0; i < n; ++i) t[i] = y[i] + 0.5 * h * k2[i];
        or_nlink_deriv(N, mass, len, b, t, tau, k3);
        for (int i = 0; i < n; ++i) t[i] = y[i] + h * k3[i];
        or_nlink_deriv(N, mass, len, b, t, tau, k4);
        for (int i = 0; i < n; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    memcpy(x_next, y, sizeof(double) * n);
    return 0;
}
