/*
 * empc.h — C ABI of the MI355X (gfx950) EMPC library, libempc.so.
 *
 * Parameterized Evolutionary Model Predictive Control, after Hyatt,
 * Williams, Killpack, "Parameterized and GPU-Parallelized Real-Time Model
 * Predictive Control for High Degree of Freedom Robots" (2020): a population
 * of candidate input trajectories, each described by p knots per input
 * (Sec. III-B, interpolation of Sec. IV-C), is simulated through the discrete
 * model (eq. 2), scored by the quadratic cost of eq. 3, and evolved by
 * selection, crossover and mutation (Sec. V, Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Memory: every array argument is a DEVICE pointer owned by the caller,
 *    unless a comment says "host".  The library never frees caller memory.
 *  - Precision: problem->dtype (EMPC_F32 or EMPC_F64) is the element type of
 *    every floating-point array of the problem and of x0, knots, costs,
 *    gradients, u* and noise.  Index outputs are int64.
 *  - Knot layout: structure of arrays.  Parameter j = knot * m + input of
 *    candidate c lives at knots[j * ld + c], ld >= number of candidates.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *    are asynchronous; results are valid once the stream has synchronised.
 *  - Errors: arguments are validated on the host before anything is
 *    launched; a bad argument returns EMPC_EINVAL and launches nothing.  A
 *    HIP launch error, or an asynchronous fault of earlier work, returns
 *    EMPC_EDEVICE.  empc_last_error() describes the last failure of the
 *    calling thread.  Nothing throws across this ABI.
 *  - Costs that are NaN rank after every finite or infinite cost.
 *  - Limits of the library: n <= 80, m <= 40 for LINEAR; d = m <= 40 joints
 *    (n = 2d) for PENDULUM_CHAIN; 1 <= p <= T; n_elite <= 256;
 *    pop <= 2^24.  Larger problems return EMPC_EUNSUPPORTED.
 */
#ifndef EMPC_H
#define EMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EMPC_OK = 0,
    EMPC_EINVAL = 1,       /* invalid argument; nothing was launched             */
    EMPC_EDEVICE = 2,      /* HIP runtime error or earlier asynchronous fault    */
    EMPC_EUNSUPPORTED = 3, /* valid problem outside the library's limits        */
    EMPC_EWORKSPACE = 4    /* workspace NULL or smaller than required            */
} empc_status;

typedef enum { EMPC_F32 = 0, EMPC_F64 = 1 } empc_dtype;

/* EMPC_LINEAR: x_{k+1} = A_d x_k + B_d u_k + w_d (eq. 2).
 * EMPC_PENDULUM_CHAIN: d = m joints, state x = [q; qd] (n = 2d), relative
 *   angles from the downward vertical; the single pendulum of eq. 5 extended
 *   joint by joint with joint stiffness, gravity torque of the cumulative
 *   angles G_j = g sum_{r>=j} l_r (sum_{i>=r} m_i) sin(q_0 + ... + q_r), and
 *   the constant diagonal inertia of the straight chain
 *   I_j = sum_{i>=j} m_i (l_j + ... + l_i)^2;
 *   qdd = (u - k q - b qd - G) / I, semi-implicit Euler with step dt.
 *   FP32 rollouts take the sine from the hardware instruction, whose input
 *   domain is +-256 revolutions: each cumulative angle q_0 + ... + q_r must
 *   stay within +-1608 rad (FP64 rollouts, the adjoint and the plant use
 *   the library sine and have no such limit). */
typedef enum { EMPC_LINEAR = 0, EMPC_PENDULUM_CHAIN = 1 } empc_model;

/* The MPC problem of eq. 3 (diagonal weights, or full Q, R, Qf below) with
 * the optional non-smooth terms below.  Pointers are device pointers of
 * problem->dtype elements. */
typedef struct {
    int32_t n, m;          /* states, inputs                                     */
    int32_t T;             /* horizon steps                                      */
    int32_t p;             /* knots per input, 1 <= p <= T                       */
    int32_t dtype;         /* empc_dtype                                         */
    int32_t model;         /* empc_model                                         */
    const void *Ad;        /* LINEAR: n*n row-major                              */
    const void *Bd;        /* LINEAR: n*m row-major                              */
    const void *wd;        /* LINEAR: n; NULL = 0                                */
    const void *stiffness; /* CHAIN: d joint stiffness                           */
    const void *damping;   /* CHAIN: d joint damping                             */
    const void *mass;      /* CHAIN: d link point masses                         */
    const void *length;    /* CHAIN: d link lengths                              */
    double gravity;        /* CHAIN: gravitational acceleration                  */
    double dt;             /* CHAIN: integration step                            */
    const void *q;         /* n  stage state weight (diagonal of Q)              */
    const void *r;         /* m  stage input weight (diagonal of R)              */
    const void *qf;        /* n  terminal state weight; NULL = 0                 */
    const void *x_goal;    /* n; NULL = 0                                        */
    const void *u_goal;    /* m; NULL = 0                                        */
    const void *u_min;     /* m  input lower bounds                              */
    const void *u_max;     /* m  input upper bounds                              */
    /* State box as a soft constraint (a variant, not in the paper's cost;
     * Sec. VII names constraints and non-smooth costs among what a sampling
     * method admits).  qb NULL: none.  Else x_min, x_max (n each) are
     * required and every state x_1..x_T adds
     *   sum_i qb_i (max(0, x_i - x_max_i)^2 + max(0, x_min_i - x_i)^2)
     * to the cost (and its derivative to the adjoint).  The arrays live on
     * the device and are not read on the host: x_min <= x_max and qb >= 0
     * are the caller's to keep (infinite bounds are allowed and cost
     * nothing). */
    const void *x_min;     /* n  state lower bounds (with qb)                    */
    const void *x_max;     /* n  state upper bounds (with qb)                    */
    const void *qb;        /* n  weights of the box penalty; NULL = none         */
    /* Non-smooth terms: Sec. V-A names effects placed in if/else branches
     * of the simulation (contact, impacts) and costs that need not be
     * continuous as what the evolutionary method admits.  NULL: none.
     * sb (needs the state box: qb, x_min, x_max; qb may be zeros): a
     *   constant sb_i for every state x_1..x_T outside [x_min_i, x_max_i],
     *   a discontinuous cost (with a box around the goal: the number of
     *   steps spent outside a tolerance band, a settling-time cost).  The
     *   adjoint takes its derivative as zero (it has none off the faces).
     * q_min, q_max (PENDULUM_CHAIN, d each, both or neither): joint limits
     *   with impacts.  After every step a joint past a limit is put back on
     *   it and its rate, if it still points outward, reversed and scaled by
     *   `restitution` (0 plastic, 1 elastic; [0, 1] is checked).  The
     *   adjoint, refinement and the batched plan refuse such problems
     *   (EMPC_EUNSUPPORTED); FP32 rollouts decide each impact in FP32. */
    const void *sb;        /* n  charge per step outside the box; NULL = none    */
    const void *q_min;     /* CHAIN: d joint lower limits; NULL = none           */
    const void *q_max;     /* CHAIN: d joint upper limits; NULL = none           */
    double restitution;    /* CHAIN: impact restitution in [0, 1]                */
    /* Full weights of eq. 3 (LINEAR only): symmetric row-major Q (n*n),
     * R (m*m), Qf (n*n) replacing q, r, qf respectively when non-NULL
     * (q, r may then be NULL); each stage adds (x-g)^T Q (x-g) +
     * (u-ug)^T R (u-ug), the end (x_T-g)^T Qf (x_T-g).  Such problems
     * run on a vector-ALU rollout with 16 lanes per candidate (n <= 64,
     * m <= 32, else EMPC_EUNSUPPORTED; for n, m <= 16 the tuner may pick
     * one lane per candidate);
     * the adjoint, refinement, the convex solver and the batched plan
     * refuse them (EMPC_EUNSUPPORTED). */
    const void *Q;         /* LINEAR: n*n full stage state weight; NULL = q      */
    const void *R;         /* LINEAR: m*m full stage input weight; NULL = r      */
    const void *Qf;        /* LINEAR: n*n full terminal weight; NULL = qf        */
    /* Dry friction with stiction (PENDULUM_CHAIN, d each, both or neither):
     * a joint at rest stays at rest while the other torques on it stay
     * within fric_s; it breaks away against fric_c, which then slows it, and
     * it sticks where that (or a holding torque within fric_s) turns it
     * round: stick-slip, a history-dependent branch of the kind Sec. V-A
     * names.  0 <= fric_c <= fric_s is the caller's to keep (device arrays,
     * not read on the host).  The adjoint, refinement and the batched plan
     * refuse such problems (EMPC_EUNSUPPORTED); FP32 rollouts decide each
     * branch in FP32. */
    const void *fric_c;    /* CHAIN: d sliding friction torques; NULL = none     */
    const void *fric_s;    /* CHAIN: d breakaway torques; NULL = none            */
} empc_problem;

/* Tunables of Alg. 1: numSims = pop, numParents = n_elite, sigma_noise. */
typedef struct {
    int32_t pop;         /* candidates per generation                            */
    int32_t n_elite;     /* parents kept by selection, 1 <= n_elite <= pop       */
    int32_t generations; /* generations per solve (one control tick)             */
    int32_t elitism;     /* 1: parents re-enter the next generation in slots     */
                         /*    0..n_elite-1; 0: every slot is a child            */
    double sigma;        /* standard deviation of the mutation noise             */
    uint64_t seed;       /* key of the counter-based random streams              */
    /* Warm-start and exploration variants (all 0: the plain method).
     * shift = 1: at the first generation of a warm-started solve the carried
     *   parents are moved one control step later in time, knot j taking the
     *   carried input at its time plus one step, (1-d) U_j + d U_{j+1} with
     *   d = (p-1)/(T-1), and the last knot held; the parents kept by elitism
     *   are the moved ones (the receding horizon advances by one step per
     *   tick).
     * sigma_dist > 0: the mutation noise of a solve is
     *   sigma_min + (sigma - sigma_min) min(1, |x0 - x_goal|_2 / sigma_dist),
     *   smaller near the goal (Sec. VII); otherwise sigma is used as is. */
    int32_t shift;
    double sigma_min;    /* noise at the goal, 0 <= sigma_min                    */
    double sigma_dist;   /* distance at which the noise reaches sigma, >= 0      */
} empc_ga;

/* Human-readable name of a status code (static string). */
const char *empc_status_str(empc_status s);

/* Message describing the last failure on the calling thread (static
 * thread-local buffer; "" if none). */
const char *empc_last_error(void);

/* Rollout and cost (Alg. 1 simulation loop; cost of eq. 3 charged on
 * x_1..x_T and u_0..u_{T-1}, plus the terminal weight on x_T).
 * x0: n.  knots: [p*m][ld].  cost: ncand outputs.  ncand >= 0; ncand = 0 is
 * a no-op.  Candidates' knots are used as given (no clamping). */
empc_status empc_rollout_cost(const empc_problem *prob, const void *x0, const void *knots,
                              int64_t ncand, int64_t ld, void *cost, void *stream);

/* One evolutionary step (Sec. V): select the n_elite lowest (cost, index)
 * candidates of knots_in / cost_in (ga->pop candidates, leading dimension
 * ld_in) and write the next population to knots_out ([p*m][ld_out]): parents
 * in slots 0..n_elite-1 when ga->elitism, children elsewhere (two parents
 * drawn uniformly with replacement, one crossover bit per parameter, one
 * mutation flag per input with N(0, sigma^2) noise on each knot of a flagged
 * input, clamp to [u_min, u_max]).  knots_in = NULL and cost_in = NULL give a
 * cold start (every knot uniform in its bounds).  elite_idx (n_elite
 * outputs, ascending index order) is required for a warm start and unused by
 * a cold start; best_idx (1 output) may be NULL.  knots_out must not overlap
 * knots_in.  (tick, gen) select the random stream. */
empc_status empc_generation(const empc_problem *prob, const empc_ga *ga, const void *knots_in,
                            int64_t ld_in, const void *cost_in, void *knots_out, int64_t ld_out,
                            int64_t *elite_idx, int64_t *best_idx, uint32_t tick, uint32_t gen,
                            void *stream);

/* Bytes of the workspace that empc_solve and empc_solve_refined need for
 * (prob, ga).  For a linear problem without the state box or full weights
 * it includes room for the problem's quadratic form (Sec. IV-B, knots of
 * Sec. IV-E) when that fits in 48 MiB: empc_solve_refined then refines on
 * it. */
size_t empc_workspace_bytes(const empc_problem *prob, const empc_ga *ga);

/* One control tick of EMPC: ga->generations rounds of {population, rollout
 * and cost, selection}, then u* = knot 0 of the best candidate (Alg. 1,
 * u* = get_u_from_U(U_best, 0)).  The workspace (device, ws_bytes >=
 * empc_workspace_bytes) carries the parents from tick to tick (warm start,
 * Sec. V); a zero-filled workspace cold-starts.  x0: n.  u_star: m.
 * best_cost: 1.  Consecutive ticks must use the same prob shape and ga. */
empc_status empc_solve(const empc_problem *prob, const empc_ga *ga, void *workspace,
                       size_t ws_bytes, const void *x0, uint32_t tick, void *u_star,
                       void *best_cost, void *stream);

/* Gradient-refined tick: as empc_solve, but after every selection the
 * parents are refined by `adam_steps` Adam updates (empc_refine semantics,
 * learning rate lr) before they breed the next generation; u* and the best
 * cost come from the best refined parent.  Same workspace as empc_solve.
 * A linear problem whose workspace holds its quadratic form forms P, q, c
 * once per call (at this x0) and takes the gradient 2 (P z + q), which is
 * the rollout cost's gradient exactly, with acceptance on the quadratic's
 * own costs; any other problem uses the adjoint (the limits of empc_grad). */
empc_status empc_solve_refined(const empc_problem *prob, const empc_ga *ga, void *workspace,
                               size_t ws_bytes, const void *x0, uint32_t tick, double lr,
                               int32_t adam_steps, void *u_star, void *best_cost, void *stream);

/* empc_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a static device array of
 * EMPC_STATIC_SCRATCH_BYTES bytes inside the library, one per GPU, held from
 * the library's load to the end of the process; the call itself allocates
 * nothing.  The array keeps the last call's contents, which is what carries
 * the parents from tick to tick: cold = 1 clears the warm-start state first
 * (a cold start, as a zero-filled workspace does for empc_solve), cold = 0
 * continues from whatever solve ran last on this GPU.  Every call on one GPU
 * shares the array, so calls that overlap on one GPU (other streams, other
 * threads) race, and a warm call after a solve of a different problem shape
 * reads that solve's parents: use cold = 1 whenever the shape or ga changes.
 * Arguments as empc_solve.  A problem whose workspace (empc_workspace_bytes)
 * exceeds the array returns EMPC_EUNSUPPORTED; cold outside {0, 1} returns
 * EMPC_EINVAL. */
#define EMPC_STATIC_SCRATCH_BYTES (64ull << 20)
empc_status empc_solve_static(const empc_problem *prob, const empc_ga *ga, const void *x0,
                              uint32_t tick, int32_t cold, void *u_star, void *best_cost,
                              void *stream);

/* Autotuner of the single-problem path.  empc_autotune times, on a
 * cold-start population of (prob, ga), every rollout launch shape of the
 * problem's kernel family (linear: one wavefront per 16-candidate tile with
 * 1, 2 or 4 per workgroup, the M-split form for more than 16 states, and,
 * if allow_valu, the vector-ALU form with one lane per candidate for n, m <=
 * 16; pendulum chain: three workgroup sizes) and the population kernel's
 * 16, 32 or 64 parameters per workgroup, then records the fastest in a
 * process-wide tuning table keyed by the problem's shape (model, dtype, n,
 * m, T, p, which optional terms are present) and the population.  Later
 * empc_solve, empc_solve_refined, empc_solve_static and empc_rollout_cost
 * calls of that shape (rollout_cost: with ncand equal to the population)
 * use the recorded choice; other shapes keep the fixed rules.  The
 * matrix-core shapes and the population choices give the same bits as the
 * rules; the vector-ALU form sums the cost in another order, so its costs
 * differ by rounding (within the FP32 / FP64 parity tolerances), which is
 * why it is only tried with allow_valu.  info (host, float[5], may be NULL):
 * the chosen rollout form (RolloutForm codes: 1..3 one wavefront per tile
 * with 1/2/4 per workgroup, 4 M-split, 5/6 vector-ALU in workgroups of
 * 256/64, 11..13 chain workgroups of 64/128/256), the chosen parameter
 * groups, its mean rollout time and the fixed rule's (us), and the chosen
 * population time (us).  A host call that allocates scratch buffers,
 * launches on `stream` and blocks until the timing is done.
 * empc_autotune_set records a choice by hand (form one of the codes above
 * or 0 for the fixed rule; groups 1, 2, 4 or 0 for the rule): EMPC_EINVAL
 * for a code the model does not have, EMPC_EUNSUPPORTED for the vector-ALU
 * form above 16 states or inputs or the M-split form at 16 states or less.
 * empc_autotune_reset clears the table. */
empc_status empc_autotune(const empc_problem *prob, const empc_ga *ga, int32_t reps,
                          int32_t allow_valu, float *info, void *stream);
empc_status empc_autotune_set(const empc_problem *prob, const empc_ga *ga, int32_t form,
                              int32_t groups);
empc_status empc_autotune_reset(void);

/* Gradient of the rollout cost with respect to the knots by a hand-written
 * adjoint pass (states recomputed from checkpoints every ceil(sqrt(T))
 * steps).  dJ: [p*m][ld].  cost: ncand (may be NULL). */
empc_status empc_grad(const empc_problem *prob, const void *x0, const void *knots, int64_t ncand,
                      int64_t ld, void *dJ, void *cost, void *stream);

/* Gradient refinement: `steps` Adam updates (beta1 0.9, beta2 0.999, eps
 * 1e-8, learning rate lr) of each candidate's knots, each followed by a clamp
 * to [u_min, u_max]; a refined candidate replaces the original only if its
 * cost is lower than the cost of its entry knots (both evaluated by the
 * refinement's own forward pass).  knots [p*m][ld] and cost (ncand) are
 * updated in place; cost is written only for replaced candidates. */
empc_status empc_refine(const empc_problem *prob, const void *x0, void *knots, int64_t ncand,
                        int64_t ld, void *cost, double lr, int32_t steps, void *stream);

/* One step of the model, x_next = f(x, u) + noise (noise may be NULL):
 * the simulated plant of a closed-loop run.  x, x_next: n.  u: m. */
empc_status empc_plant_step(const empc_problem *prob, const void *x, const void *u,
                            const void *noise, void *x_next, void *stream);

/* Parameterized small-matrix convex MPC (Sec. IV-B small-matrix formulation
 * with the knot parameterization of Sec. IV-E), the paper's other method,
 * for EMPC_LINEAR problems without the state box penalty: with z the knot
 * vector [p*m] (z[j*m + i] = knot j of input i), the states x_1..x_T are
 * S z + v and the cost of eq. 3 is J(z) = z^T P z + 2 q^T z + c;
 * u_min <= z <= u_max (each input's bounds on each of its knots) keeps
 * every interpolated input in bounds, so the MPC is a box-constrained QP.
 * Limits: p*m <= 1024 (more: EMPC_EUNSUPPORTED); FP64 arithmetic inside,
 * arrays in the problem dtype.
 * empc_qp_workspace_bytes(prob): device workspace of both calls (0 for an
 *   invalid or unsupported problem).
 * empc_qp_form: P [p*m][p*m] row-major, q [p*m], c [1] at state x0 [n] (the
 *   "MPC solve time" matrix formation: S from the responses to unit knots,
 *   then S^T Qb S plus the input term).
 * empc_qp_solve: the minimizer z [p*m] of z^T P z + 2 q^T z over the box by
 *   the projected Newton method (Bertsekas 1982: Newton steps on the
 *   variables off their bounds by Cholesky solves of P restricted to them,
 *   an Armijo search along the projection arc), stopping when the projected
 *   gradient vanishes to rounding or after max_iter iterations; cost [1] =
 *   J(z) including c; info (device, int32[2]) = {iterations, converged}.
 *   P must be positive definite (r > 0 for every input suffices).  u* is
 *   the first m entries of z (knot 0). */
size_t empc_qp_workspace_bytes(const empc_problem *prob);
empc_status empc_qp_form(const empc_problem *prob, const void *x0, void *workspace,
                         size_t ws_bytes, void *P, void *q, void *c, void *stream);
empc_status empc_qp_solve(const empc_problem *prob, const void *P, const void *q, const void *c,
                          void *workspace, size_t ws_bytes, int32_t max_iter, void *z, void *cost,
                          int32_t *info, void *stream);

/* The N-link planar robot of the paper's convex-solver and EMPC experiments
 * (Sec. IV-F setup, used again in Sec. VI-A): N revolute joints in a plane
 * perpendicular to gravity, M(q) qdd + C(q, qd) + b qd = tau, each link
 * massless with a point mass at its far end (N = 1 is the pendulum of eq. 5
 * with g = 0), relative joint angles, state x = [q; qd] (2N), input tau (N).
 * EMPC controls it through the linear model of eq. 2, relinearized at the
 * current state every tick (Sec. VI-A: the dynamics matrices are computed
 * from the current conditions).  Every array of the robot, x, u and the
 * outputs has robot->dtype elements; the kernels compute in FP64. */
typedef struct {
    int32_t links;      /* N, 1 <= N <= 16 (more: EMPC_EUNSUPPORTED)            */
    int32_t dtype;      /* empc_dtype                                           */
    const void *mass;   /* N point masses (device)                              */
    const void *length; /* N link lengths (device)                              */
    double damping;     /* viscous joint damping b                              */
} empc_nlink;

/* Discrete affine model x_{k+1} = A_d x_k + B_d u_k + w_d (eq. 2) of the robot
 * at (x, u): the exact Jacobians A = df/dx, B = df/du of f = [qd; qdd], the
 * offset w = f(x, u) - A x - B u of the first-order expansion, and the
 * zero-order hold over dt (the exponential of [[A, B, w], [0, 0, 0]] dt).
 * Ad: 2N x 2N, Bd: 2N x N row-major, wd: 2N, ready to be pointed at by an
 * empc_problem of model EMPC_LINEAR.  dt finite and > 0. */
empc_status empc_nlink_linearize(const empc_nlink *robot, double dt, const void *x,
                                 const void *u, void *Ad, void *Bd, void *wd, void *stream);

/* The robot itself over dt with u held: `substeps` classical Runge-Kutta
 * steps (the simulated plant of a closed loop).  x, x_next: 2N (x_next may
 * be x: the state is read before anything is written); u: N. */
empc_status empc_nlink_step(const empc_nlink *robot, double dt, int32_t substeps, const void *x,
                            const void *u, void *x_next, void *stream);

/* Batched solve: many independent problems (each its own empc_problem, all
 * FP32, possibly of different model, size, horizon and knot count) advance
 * one control tick together under one empc_ga.  Problem i draws from the
 * Philox key (seed low word, seed high word XOR i), so it evolves exactly as
 * empc_solve would with that seed.
 *
 * empc_batch_workspace_bytes(probs (host array), nprob, ga) -> bytes of
 *   device workspace (0 if an argument is invalid).
 * empc_batch_create binds the problems, the workspace (device, zero-filled
 *   for a cold start; it also holds the tick counter, starting at 0), the
 *   packed initial states x0_packed (device, sum of n, problem after
 *   problem; the caller may rewrite them between ticks), the packed outputs
 *   u_star_packed (device, sum of m) and best_cost (device, nprob) into a
 *   plan.  Host call; allocates the plan's small device tables.
 * empc_solve_batched(plan, stream) runs one tick: ga->generations x
 *   {population, rollout + cost, selection} for every problem, then
 *   increments the device tick counter, so that a HIP graph captured from
 *   one call replays tick after tick.  Allocates nothing.
 * empc_batch_destroy frees the plan (not the caller's buffers). */
typedef struct empc_batch empc_batch;
size_t empc_batch_workspace_bytes(const empc_problem *probs, int32_t nprob, const empc_ga *ga);
empc_status empc_batch_create(const empc_problem *probs, int32_t nprob, const empc_ga *ga,
                              void *workspace, size_t ws_bytes, const void *x0_packed,
                              void *u_star_packed, void *best_cost, empc_batch **out);
empc_status empc_solve_batched(empc_batch *plan, void *stream);
empc_status empc_batch_destroy(empc_batch *plan);

/* Launch-shape autotuner of a batch plan.  The plan groups its problems into
 * classes that share a rollout kernel (linear: state tiles of 16 and input
 * slices of 4; chain: joints per lane); each class has a few launch shapes
 * (linear: one wavefront per 16-candidate tile with 4, 2 or 1 wavefronts per
 * workgroup, or the M-split form with one wavefront per state tile; chain:
 * workgroup sizes), and every shape of a class runs the same per-candidate
 * arithmetic, so the shape changes the time, never a result (the VALU form
 * that empc_batch_allow_valu offers is the one exception).
 * empc_batch_create picks shapes by a fixed rule.  empc_batch_autotune(plan,
 * reps, stream) times every shape of every class on the plan's own problems
 * (one untimed and `reps` timed launches each, on `stream`, after one
 * generation-0 population), keeps the fastest per class, then times the
 * generation's rollouts with 1..4 side streams, the classes spread over them
 * by their measured times, and keeps the fastest count.  Host call that
 * blocks until the timing is done; it overwrites only the generation-0
 * population and the costs in the workspace (the next solve rewrites both),
 * so the warm-start state and the tick counter are unchanged.  Call it
 * before capturing a graph of empc_solve_batched.  EMPC_EINVAL for a NULL
 * plan or reps < 1.
 * empc_batch_classes(plan) -> number of classes (0 for NULL).
 * empc_batch_class_info(plan, cls, info[7]) fills model, the two shape
 *   parameters (linear: state tiles, input-slice bucket; chain: joint
 *   bucket, 0), problem count, chosen shape, number of shapes, side stream.
 * empc_batch_class_times(plan, cls, us[4]) gives the mean launch time in
 *   microseconds the autotuner measured for each shape (-1: not measured).
 * empc_batch_set_variant(plan, cls, variant) sets a class's shape by hand
 *   (EMPC_EINVAL if out of range).
 * empc_batch_allow_valu(plan, allow) offers (allow != 0) or withdraws the
 *   vector-ALU form, one lane per candidate, as shape 3 of every linear class
 *   of at most 16 states whose inputs are at most 16 and whose problems share
 *   the form's padded state count (4, 8 or 16); a problem solved in that form
 *   gives the bits of its single solve with the form pinned (RF_VALU64), not
 *   those of the matrix-core shapes (its cost is summed in another order),
 *   which is why the plan starts without it.  Withdrawing it puts a class
 *   that uses it back on shape 0.  Host call; EMPC_EINVAL for a NULL plan. */
empc_status empc_batch_autotune(empc_batch *plan, int32_t reps, void *stream);
int32_t empc_batch_classes(const empc_batch *plan);
empc_status empc_batch_class_info(const empc_batch *plan, int32_t cls, int32_t *info);
empc_status empc_batch_class_times(const empc_batch *plan, int32_t cls, float *us);
empc_status empc_batch_set_variant(empc_batch *plan, int32_t cls, int32_t variant);
empc_status empc_batch_allow_valu(empc_batch *plan, int32_t allow);

/* Launch form of a batch plan's ticks.  Mode 0 (the default): per
 * generation, one population launch, one rollout launch per class (on side
 * streams), one selection launch over all problems, then a tick-advance
 * launch.  Mode 1, the persistent work-queue form: per generation, one
 * population launch and one persistent kernel per register tier (linear
 * problems of more than 32 states; of 17..32 states; of at most 16 states;
 * pendulum chains), whose one-wavefront workgroups
 * take (problem, candidate tile) items from an atomic queue, the heaviest
 * problems first; the wave that finishes a problem's last tile runs its
 * selection, and the one that finishes the last selection advances the
 * tick, so no wave ever waits for another.  Both forms give the same bits.
 * Mode 1 takes populations of at most 1024 and problems without the state
 * box penalty (else EMPC_EUNSUPPORTED); EMPC_EINVAL for a NULL plan or
 * another mode. */
empc_status empc_batch_set_mode(empc_batch *plan, int32_t mode);

/* Kernel timing.  empc_profile_begin(max_launches) creates a pool of HIP
 * event pairs (host call, may allocate); until empc_profile_end, every
 * rollout launch made by empc_rollout_cost and empc_solve (at most
 * max_launches of them) carries an event pair stamped at the start and end
 * of the kernel's own dispatch (no extra packets on the stream).
 * empc_profile_end waits for the recorded events and returns the number of
 * timed launches and their summed duration in milliseconds, then stops
 * timing.  Not thread-safe: one profiling session per process. */
empc_status empc_profile_begin(int32_t max_launches);
empc_status empc_profile_end(int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* EMPC_H */
