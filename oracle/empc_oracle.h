/*
 * EMPC oracle: plain, slow, single-threaded FP64 reference of the
 * parameterized Evolutionary MPC hot path (Hyatt, Williams, Killpack,
 * "Parameterized and GPU-Parallelized Real-Time Model Predictive Control for
 * High Degree of Freedom Robots", 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library) shares no code, header or constant with it.
 *
 * Parity status per function (what pins it, see the tests):
 *   or_philox4x32_10   pinned: published Philox known-answer vectors and an
 *                      independent library implementation.
 *   or_knot_weights    pinned: worked example T=5, p=3 of Sec. IV-D.
 *   or_rollout_cost    linear: pinned by the small-matrix closed form
 *                      (Sec. IV-B) and the quadratic form of J;
 *                      pendulum chain: pinned by energy / equilibrium /
 *                      single-pendulum (eq. 5) special cases and the
 *                      gravity-torque finite-difference check.
 *   or_select          pinned: a library sort on (isnan(J), J, index).
 *   or_next_population pinned: statistics of the draws, bounds, elitism.
 *   or_solve           pinned: brute-force box-QP bound on tiny problems;
 *                      multi-generation trajectories beyond one generation
 *                      are parity unpinned against the paper (the paper gives
 *                      no numbers for them).
 *   or_grad            pinned: central finite differences, and 2 P U + 2 q
 *                      of the small-matrix form for linear models.
 *   or_refine          pinned: Adam (Kingma & Ba 2015) on a one-parameter
 *                      quadratic: the first update equals -lr g/(|g|+eps),
 *                      later updates equal the bias-corrected recursion in
 *                      high-precision decimal arithmetic, the clamp acts
 *                      after every update, moments start at zero per call,
 *                      worse candidates are rejected; plus or_grad's pins.
 *   or_nlink_*         (nlink_oracle.c, the N-link planar robot of the
 *                      paper's Sec. IV-F setup) pinned: the two-link
 *                      closed form of M and C, eq. 5 without gravity for one
 *                      link (and its zero-order-hold closed form), kinetic
 *                      energy from the mass points' velocities, energy
 *                      conservation, power balance and Lagrange's equation
 *                      by differences in time, the complex-step Jacobian by
 *                      central differences, the hold against a fine RK4 of
 *                      the affine expansion, third-order local error of the
 *                      linearized step, fourth-order convergence of RK4.
 */
#ifndef EMPC_ORACLE_H
#define EMPC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_LINEAR = 0, OR_PENDULUM_CHAIN = 1 };

/* Problem statement of eq. 3 with the knot parameterization of Sec. III-B.
 * All arrays are host memory, float64, owned by the caller. */
typedef struct {
    int model;              /* OR_LINEAR or OR_PENDULUM_CHAIN                  */
    int n, m, T, p;         /* states, inputs, horizon steps, knots per input  */
    const double *Ad;       /* linear: n*n row-major                           */
    const double *Bd;       /* linear: n*m row-major                           */
    const double *wd;       /* linear: n, may be NULL (= 0)                    */
    const double *stiff;    /* chain (d = m, n = 2d): joint stiffness, d       */
    const double *damp;     /* chain: joint viscous damping, d                 */
    const double *mass;     /* chain: link point mass, d                       */
    const double *len;      /* chain: link length, d                           */
    double gravity, dt;     /* chain: gravity and integration step             */
    const double *q, *r;    /* diagonal stage weights: n, m                    */
    const double *qf;       /* diagonal terminal weight: n, may be NULL (= 0)  */
    const double *x_goal;   /* n, may be NULL (= 0)                            */
    const double *u_goal;   /* m, may be NULL (= 0)                            */
    const double *u_min, *u_max; /* m                                          */
    /* state box as a soft constraint (NULL qb: none): each of x_1..x_T adds
     * sum_i qb_i (max(0, x_i - x_max_i)^2 + max(0, x_min_i - x_i)^2)      */
    const double *x_min, *x_max, *qb; /* n                                     */
    /* non-smooth terms (Sec. V-A: branches in the simulation and costs that
     * need not be continuous), NULL = none:
     * sb (with the state box): sb_i for every state x_1..x_T outside
     *   [x_min_i, x_max_i], a discontinuous cost;
     * q_min, q_max (chain, d each): joint limits with impacts; after each
     *   step a joint past a limit is put back on it and its rate, if it
     *   still points outward, reversed and scaled by the restitution.      */
    const double *sb;                 /* n                                     */
    const double *q_min, *q_max;      /* d                                     */
    double restitution;               /* in [0, 1]                             */
    /* full symmetric weights (linear model), row-major, replacing the
     * diagonal q, r, qf when given: (x-g)^T Q (x-g) + (u-ug)^T R (u-ug) per
     * stage and (x_T-g)^T Qf (x_T-g) at the end (eq. 3 with full Q, R).   */
    const double *Q, *R, *Qf;         /* n*n, m*m, n*n                          */
    /* chain dry friction (d each, NULL = none): sliding torque fric_c,
     * breakaway torque fric_s >= fric_c; a joint at rest stays at rest
     * while the other torques stay within fric_s (stick-slip, a
     * history-dependent branch).                                           */
    const double *fric_c, *fric_s;
} or_problem;

/* Tunables of Alg. 1: numSims (pop), numParents (n_elite), sigma_noise. */
typedef struct {
    int pop, n_elite, generations, elitism;
    double sigma;
    uint64_t seed;
    int shift;          /* 1: move the carried parents one step later per solve */
    double sigma_min;   /* noise at the goal (sigma_dist > 0)                    */
    double sigma_dist;  /* > 0: distance-dependent noise, see or_sigma_at        */
} or_ga;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_knot_weights(int T, int p, int k, int *a, int *b, double *c);
void or_input_at(const or_problem *P, const double *knots, int64_t ld, int64_t cand, int k,
                 double *u);
void or_step(const or_problem *P, const double *x, const double *u, double *x_next);
double or_rollout_one(const or_problem *P, const double *x0, const double *knots, int64_t ld,
                      int64_t cand, double *traj);
void or_rollout_cost(const or_problem *P, const double *x0, const double *knots, int64_t ncand,
                     int64_t ld, double *cost);
void or_select(const double *cost, int64_t pop, int k, int64_t *elite_idx, int64_t *best);
void or_next_population(const or_problem *P, const or_ga *G, const double *elite_knots, int cold,
                        uint32_t tick, uint32_t gen, double *knots, int64_t ld);
void or_shift_knots(const or_problem *P, double *rows, int k);
double or_sigma_at(const or_problem *P, const or_ga *G, const double *x0);
int or_solve(const or_problem *P, const or_ga *G, double *elite_knots, int *has_elites,
             const double *x0, uint32_t tick, double *u_star, double *best_cost,
             double *gen_best, double *knots_ws, double *cost_ws, int64_t *idx_ws, int refine,
             double lr, int adam_steps);
void or_grad(const or_problem *P, const double *x0, const double *knots, int64_t ncand,
             int64_t ld, double *dJ, double *cost);
void or_refine(const or_problem *P, const double *x0, double *knots, int64_t ncand, int64_t ld,
               double *cost, double lr, int steps);
void or_plant_step(const or_problem *P, const double *x, const double *u, const double *noise,
                   double *x_next);

#ifdef __cplusplus
}
#endif
#endif
