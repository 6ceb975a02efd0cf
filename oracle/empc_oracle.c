/*
 * EMPC oracle (FP64, single-threaded).  TEST INFRASTRUCTURE ONLY: see
 * empc_oracle.h for who may load it and how each function is pinned.
 *
 * Conventions taken where the paper is silent or inconsistent (each one is
 * listed with its reason in the design notes of the repository):
 *  - cost (eq. 3 vs Alg. 1 vs the small-matrix form of Sec. IV-B): the stage
 *    cost is charged on x_1..x_T with u_0..u_{T-1}; a diagonal terminal
 *    weight Q_f (default 0) stands for the undefined terminal_cost;
 *  - knot interpolation (Sec. IV-C): idx1 and c are computed in exact integer
 *    arithmetic (k*(p-1) against T-1) because Delta T is rarely
 *    representable; idx2 is clamped to p-1 where c = 0; p = 1 holds the
 *    single knot constant;
 *  - evolutionary step (Sec. V, Alg. 1): elites kept in slots 0..k-1; one
 *    crossover bit per parameter; one mutation flag per (child, input);
 *    Gaussian noise on each knot of a flagged input; clamp to the input
 *    bounds; random numbers from Philox4x32-10 (Salmon et al., SC'11) with
 *    Box-Muller normals, in the counter layout documented below.
 */
#include "empc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10, Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11.  Round: two 32x32->64 products of the even counter
 * words with the multipliers, outputs permuted and xored with the odd counter
 * words and the key; the key advances by the Weyl constants between rounds.
 */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        philox_round(c, k);
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    memcpy(out, c, sizeof c);
}

/* Counter layout of the evolutionary draws.  Block (slot, gen, tick, w3) with
 * w3 = stream << 24 | block index; key = (seed low word, seed high word).
 * Warm start (stream 0):
 *   block 0                      words 0,1 -> parent draws P1, P2
 *   blocks 1 ..                  mutation flag of input i: block 1 + i/128,
 *                                word (i/32) % 4, bit i % 32
 *   blocks XB = 1+ceil(m/128) .. crossover bit of parameter j: block
 *                                XB + j/128, word (j/32) % 4, bit j % 32
 *   blocks NB = XB+ceil(pm/128)  normal of parameter j: block NB + j/4; words
 *                                (0,1) give the Box-Muller pair of j%4 in
 *                                {0,1}, words (2,3) that of j%4 in {2,3}
 * Cold start (stream 1): parameter j uses block j/4, word j%4. */
static void ga_block(const or_ga *G, uint32_t slot, uint32_t gen, uint32_t tick, uint32_t stream,
                     uint32_t block, uint32_t out[4]) {
    uint32_t ctr[4] = {slot, gen, tick, (stream << 24) | block};
    uint32_t key[2] = {(uint32_t)G->seed, (uint32_t)(G->seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* Uniform on (0,1) from the top 23 bits of a word: (2*(w>>9)+1) * 2^-24,
 * exactly representable in binary32 and binary64. */
static double uni23(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Integer in [0, k) by the multiply-shift map floor(w * k / 2^32). */
static int64_t draw_index(uint32_t w, int k) { return (int64_t)(((uint64_t)w * (uint64_t)k) >> 32); }

static int bit_of(const uint32_t blk[4], int j) { return (int)((blk[(j / 32) % 4] >> (j % 32)) & 1u); }

/* ---------------------------------------------------------------------------
 * Knot interpolation, Sec. IV-C: Delta T = (T-1)/(p-1), idx1 = floor(k /
 * Delta T), idx2 = idx1 + 1, c = (k - idx1 Delta T) / Delta T and
 * u = (1-c) U_idx1 + c U_idx2.  Multiplying through by (p-1) keeps idx1 exact:
 * k / Delta T = k (p-1) / (T-1). */
void or_knot_weights(int T, int p, int k, int *a, int *b, double *c) {
    if (p == 1 || T == 1) {
        *a = 0; *b = 0; *c = 0.0;
        return;
    }
    long num = (long)k * (long)(p - 1);
    long den = (long)(T - 1);
    long idx1 = num / den;
    long rem = num - idx1 * den;
    *a = (int)idx1;
    *b = (int)(idx1 + 1 < p ? idx1 + 1 : p - 1);
    *c = (double)rem / (double)den;
}

/* get_u_from_U (Sec. V): input vector at step k of candidate `cand`.
 * Knots are stored SoA: parameter (knot*m + i) of candidate c at [.*ld + c]. */
void or_input_at(const or_problem *P, const double *knots, int64_t ld, int64_t cand, int k,
                 double *u) {
    int a, b;
    double c;
    or_knot_weights(P->T, P->p, k, &a, &b, &c);
    for (int i = 0; i < P->m; ++i) {
        double Ua = knots[(int64_t)(a * P->m + i) * ld + cand];
        double Ub = knots[(int64_t)(b * P->m + i) * ld + cand];
        u[i] = (1.0 - c) * Ua + c * Ub;
    }
}

/* ---------------------------------------------------------------------------
 * Dynamics.
 * Linear: eq. 2, x_{k+1} = A_d x_k + B_d u_k + w_d.
 * Pendulum chain (the paper's single pendulum of eq. 5, m l^2 qdd + b qd +
 * m g l sin q = tau, extended joint by joint): relative joint angles q_j
 * measured from the downward vertical, absolute angle phi_r = sum_{s<=r} q_s,
 * tail mass M_r = sum_{i>=r} m_i, gravity torque
 *   G_j = g sum_{r>=j} l_r M_r sin(phi_r)   (the gradient of the potential),
 * constant diagonal inertia about joint j of the distal point masses with the
 * chain straight, I_j = sum_{i>=j} m_i (sum_{r=j..i} l_r)^2 (equal to m l^2
 * for one link), joint stiffness k_j and damping b_j:
 *   qdd_j = (u_j - k_j q_j - b_j qd_j - G_j) / I_j,
 * integrated by semi-implicit Euler: qd <- qd + dt qdd, q <- q + dt qd. */
static void chain_constants(const or_problem *P, double *tail_mass, double *inertia) {
    int d = P->m;
    for (int r = 0; r < d; ++r) {
        double s = 0.0;
        for (int i = r; i < d; ++i) s += P->mass[i];
        tail_mass[r] = s;
    }
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int i = j; i < d; ++i) {
            double dist = 0.0;
            for (int r = j; r <= i; ++r) dist += P->len[r];
            s += P->mass[i] * dist * dist;
        }
        inertia[j] = s;
    }
}

static void chain_step(const or_problem *P, const double *tail_mass, const double *inertia,
                       const double *x, const double *u, double *x_next) {
    int d = P->m;
    const double *q = x, *qd = x + d;
    double *sphi = (double *)malloc(sizeof(double) * (size_t)d);
    double phi = 0.0;
    for (int r = 0; r < d; ++r) {
        phi += q[r];
        sphi[r] = sin(phi);
    }
    for (int j = 0; j < d; ++j) {
        double G = 0.0;
        for (int r = j; r < d; ++r) G += P->len[r] * tail_mass[r] * sphi[r];
        G *= P->gravity;
        double f = u[j] - P->stiff[j] * q[j] - P->damp[j] * qd[j] - G;
        double qd_new = qd[j] + P->dt * (f / inertia[j]);
        if (P->fric_c) {
            /* dry friction with stiction: a joint at rest stays at rest while
             * |f| <= fric_s, else it breaks away against fric_c; a moving
             * joint is slowed by fric_c, and if that (or f) turns it round
             * while |f| <= fric_s it sticks */
            double tc = P->fric_c[j], ts = P->fric_s[j], dti = P->dt / inertia[j];
            if (qd[j] == 0.0) {
                qd_new = fabs(f) <= ts ? 0.0 : qd_new - dti * tc * (f > 0.0 ? 1.0 : -1.0);
            } else {
                qd_new -= dti * tc * (qd[j] > 0.0 ? 1.0 : -1.0);
                if (qd_new * qd[j] <= 0.0 && fabs(f) <= ts) qd_new = 0.0;
            }
        }
        double q_new = q[j] + P->dt * qd_new;
        /* joint limits with impacts: an if/else branch inside the
         * simulation of the kind Sec. V-A names (contact, impacts) */
        if (P->q_max && q_new > P->q_max[j]) {
            q_new = P->q_max[j];
            if (qd_new > 0.0) qd_new = -P->restitution * qd_new;
        } else if (P->q_min && q_new < P->q_min[j]) {
            q_new = P->q_min[j];
            if (qd_new < 0.0) qd_new = -P->restitution * qd_new;
        }
        x_next[d + j] = qd_new;
        x_next[j] = q_new;
    }
    free(sphi);
}

static void linear_step(const or_problem *P, const double *x, const double *u, double *x_next) {
    int n = P->n, m = P->m;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += P->Ad[i * n + j] * x[j];
        for (int j = 0; j < m; ++j) s += P->Bd[i * m + j] * u[j];
        if (P->wd) s += P->wd[i];
        x_next[i] = s;
    }
}

void or_step(const or_problem *P, const double *x, const double *u, double *x_next) {
    if (P->model == OR_LINEAR) {
        linear_step(P, x, u, x_next);
    } else {
        double *tm = (double *)malloc(sizeof(double) * (size_t)P->m);
        double *in = (double *)malloc(sizeof(double) * (size_t)P->m);
        chain_constants(P, tm, in);
        chain_step(P, tm, in, x, u, x_next);
        free(tm);
        free(in);
    }
}

void or_plant_step(const or_problem *P, const double *x, const double *u, const double *noise,
                   double *x_next) {
    or_step(P, x, u, x_next);
    if (noise)
        for (int i = 0; i < P->n; ++i) x_next[i] += noise[i];
}

/* ---------------------------------------------------------------------------
 * Cost of eq. 3 on x_1..x_T and u_0..u_{T-1} with diagonal Q, R, plus the
 * terminal term on x_T (Alg. 1 adds the stage cost after each simulated step
 * and a terminal cost after the loop). */
static double x_goal_at(const or_problem *P, int i) { return P->x_goal ? P->x_goal[i] : 0.0; }
static double u_goal_at(const or_problem *P, int i) { return P->u_goal ? P->u_goal[i] : 0.0; }

/* State box as a soft constraint (a variant: the paper names non-smooth
 * costs and constraints as what a sampling method admits, Sec. VII): the
 * squared distance of each state to [x_min, x_max], weighted by qb. */
static double box_penalty(const or_problem *P, const double *x) {
    double J = 0.0;
    if (!P->qb) return 0.0;
    for (int i = 0; i < P->n; ++i) {
        double over = x[i] - P->x_max[i], under = P->x_min[i] - x[i];
        if (over > 0.0) J += P->qb[i] * over * over;
        if (under > 0.0) J += P->qb[i] * under * under;
        /* a constant charge for being outside at all: discontinuous at the
         * bounds (Sec. V-A: costs need not be continuous) */
        if (P->sb && (x[i] > P->x_max[i] || x[i] < P->x_min[i])) J += P->sb[i];
    }
    return J;
}

/* e^T W e for a symmetric n x n row-major W */
static double quad_form(const double *W, const double *e, int n) {
    double J = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) J += e[i] * W[i * n + j] * e[j];
    return J;
}

/* d box_penalty / d x_i */
static double box_penalty_grad(const or_problem *P, const double *x, int i) {
    if (!P->qb) return 0.0;
    double over = x[i] - P->x_max[i], under = P->x_min[i] - x[i];
    if (over > 0.0) return 2.0 * P->qb[i] * over;
    if (under > 0.0) return -2.0 * P->qb[i] * under;
    return 0.0;
}

static double stage_cost(const or_problem *P, const double *x, const double *u) {
    double J = box_penalty(P, x);
    double *e = (double *)malloc(sizeof(double) * (size_t)(P->n > P->m ? P->n : P->m));
    for (int i = 0; i < P->n; ++i) e[i] = x_goal_at(P, i) - x[i];
    if (P->Q) {
        J += quad_form(P->Q, e, P->n);
    } else {
        for (int i = 0; i < P->n; ++i) J += P->q[i] * e[i] * e[i];
    }
    for (int i = 0; i < P->m; ++i) e[i] = u_goal_at(P, i) - u[i];
    if (P->R) {
        J += quad_form(P->R, e, P->m);
    } else {
        for (int i = 0; i < P->m; ++i) J += P->r[i] * e[i] * e[i];
    }
    free(e);
    return J;
}

static double terminal_cost(const or_problem *P, const double *x) {
    double J = 0.0;
    if (P->Qf) {
        double *e = (double *)malloc(sizeof(double) * (size_t)P->n);
        for (int i = 0; i < P->n; ++i) e[i] = x_goal_at(P, i) - x[i];
        J = quad_form(P->Qf, e, P->n);
        free(e);
        return J;
    }
    if (!P->qf) return 0.0;
    for (int i = 0; i < P->n; ++i) {
        double e = x_goal_at(P, i) - x[i];
        J += P->qf[i] * e * e;
    }
    return J;
}

/* Simulate one candidate from x0 over T steps (Alg. 1, simulation loop) and
 * return its cost.  If traj != NULL it receives x_0..x_T, (T+1)*n values. */
double or_rollout_one(const or_problem *P, const double *x0, const double *knots, int64_t ld,
                      int64_t cand, double *traj) {
    int n = P->n, m = P->m;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *xn = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)m);
    double *tm = NULL, *in = NULL;
    if (P->model == OR_PENDULUM_CHAIN) {
        tm = (double *)malloc(sizeof(double) * (size_t)m);
        in = (double *)malloc(sizeof(double) * (size_t)m);
        chain_constants(P, tm, in);
    }
    memcpy(x, x0, sizeof(double) * (size_t)n);
    if (traj) memcpy(traj, x, sizeof(double) * (size_t)n);
    double J = 0.0;
    for (int k = 0; k < P->T; ++k) {
        or_input_at(P, knots, ld, cand, k, u);
        if (P->model == OR_LINEAR)
            linear_step(P, x, u, xn);
        else
            chain_step(P, tm, in, x, u, xn);
        memcpy(x, xn, sizeof(double) * (size_t)n);
        if (traj) memcpy(traj + (size_t)(k + 1) * n, x, sizeof(double) * (size_t)n);
        J += stage_cost(P, x, u);
    }
    J += terminal_cost(P, x);
    free(x); free(xn); free(u); free(tm); free(in);
    return J;
}

void or_rollout_cost(const or_problem *P, const double *x0, const double *knots, int64_t ncand,
                     int64_t ld, double *cost) {
    for (int64_t c = 0; c < ncand; ++c) cost[c] = or_rollout_one(P, x0, knots, ld, c, NULL);
}

/* ---------------------------------------------------------------------------
 * Parent selection (Sec. V): the numParents candidates of lowest cost.
 * Total order (isnan(J), J, index): every NaN ranks after every number,
 * +infinity included, numbers in numeric order (-0 and +0 tie), ties by
 * index.  elite_idx receives the selected indices in ascending index order;
 * *best the first in that order. */
static int cost_cmp(double a, int64_t ia, double b, int64_t ib) {
    int na = isnan(a) != 0, nb = isnan(b) != 0;
    if (na != nb) return na - nb;
    if (!na) {
        if (a < b) return -1;
        if (a > b) return 1;
    }
    return (ia > ib) - (ia < ib);
}
/* comparator context of or_select; one per thread, so that concurrent
 * selections (the all-cores baseline runs one oracle per thread) do not mix */
static _Thread_local const double *g_sort_cost;
static int cmp_cost_idx(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return cost_cmp(g_sort_cost[a], a, g_sort_cost[b], b);
}
static int cmp_i64(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return (a > b) - (a < b);
}

void or_select(const double *cost, int64_t pop, int k, int64_t *elite_idx, int64_t *best) {
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)pop);
    for (int64_t i = 0; i < pop; ++i) order[i] = i;
    g_sort_cost = cost;
    qsort(order, (size_t)pop, sizeof(int64_t), cmp_cost_idx);
    *best = order[0];
    memcpy(elite_idx, order, sizeof(int64_t) * (size_t)k);
    qsort(elite_idx, (size_t)k, sizeof(int64_t), cmp_i64);
    free(order);
}

/* ---------------------------------------------------------------------------
 * Population for the next generation (Sec. V, Alg. 1 cold / warm start).
 * elite_knots: k rows of p*m parameters (row s = elite s in ascending index
 * order).  knots: output, SoA [p*m][ld]. */
void or_next_population(const or_problem *P, const or_ga *G, const double *elite_knots, int cold,
                        uint32_t tick, uint32_t gen, double *knots, int64_t ld) {
    int m = P->m, pm = P->p * P->m, k = G->n_elite;
    int XB = 1 + (m + 127) / 128;
    int NB = XB + (pm + 127) / 128;
    double *child = (double *)malloc(sizeof(double) * (size_t)pm);
    for (int64_t s = 0; s < G->pop; ++s) {
        uint32_t slot = (uint32_t)s;
        if (cold) {
            /* U(i) ~ Uniform(u_min(i), u_max(i)) */
            for (int j = 0; j < pm; ++j) {
                uint32_t blk[4];
                ga_block(G, slot, gen, tick, 1, (uint32_t)(j / 4), blk);
                int i = j % m;
                child[j] = P->u_min[i] + (P->u_max[i] - P->u_min[i]) * uni23(blk[j % 4]);
            }
        } else if (G->elitism && s < k) {
            memcpy(child, elite_knots + (size_t)s * pm, sizeof(double) * (size_t)pm);
        } else {
            uint32_t b0[4];
            ga_block(G, slot, gen, tick, 0, 0, b0);
            int64_t P1 = draw_index(b0[0], k);
            int64_t P2 = draw_index(b0[1], k);
            const double *U1 = elite_knots + (size_t)P1 * pm;
            const double *U2 = elite_knots + (size_t)P2 * pm;
            /* mate: each parameter from either parent with probability 1/2 */
            for (int j = 0; j < pm; ++j) {
                uint32_t bx[4];
                ga_block(G, slot, gen, tick, 0, (uint32_t)(XB + j / 128), bx);
                child[j] = bit_of(bx, j % 128) ? U2[j] : U1[j];
            }
            /* mutate: each input flagged with probability 1/2; a flagged
             * input gets N(0, sigma^2) noise on each of its knots */
            for (int j = 0; j < pm; ++j) {
                int i = j % m;
                uint32_t bf[4];
                ga_block(G, slot, gen, tick, 0, (uint32_t)(1 + i / 128), bf);
                if (!bit_of(bf, i % 128)) continue;
                uint32_t bn[4];
                ga_block(G, slot, gen, tick, 0, (uint32_t)(NB + j / 4), bn);
                int pair = (j % 4) / 2;
                double u1 = uni23(bn[2 * pair]);
                double u2 = uni23(bn[2 * pair + 1]);
                double rad = sqrt(-2.0 * log(u1));
                double ang = 6.283185307179586 * u2; /* 2 pi */
                double z = (j % 2 == 0) ? rad * cos(ang) : rad * sin(ang);
                child[j] += G->sigma * z;
            }
            /* simple bounding of the trajectory: clamp every knot */
            for (int j = 0; j < pm; ++j) {
                int i = j % m;
                if (child[j] < P->u_min[i]) child[j] = P->u_min[i];
                if (child[j] > P->u_max[i]) child[j] = P->u_max[i];
            }
        }
        for (int j = 0; j < pm; ++j) knots[(int64_t)j * ld + s] = child[j];
    }
    free(child);
}

/* ---------------------------------------------------------------------------
 * Adjoint gradient dJ/dknots (not in the paper; the plain definition of the
 * derivative of the rollout cost).  With lambda_k = dJ/dx_k:
 *   lambda_T = 2 (Q + Q_f)(x_T - g)
 *   lambda_k = 2 Q (x_k - g) + f_x(x_k, u_k)^T lambda_{k+1},   k = T-1..1
 *   dJ/du_k  = 2 R (u_k - u_g) + f_u(x_k, u_k)^T lambda_{k+1}, k = T-1..0
 * and dJ/du_k is scattered to knots idx1 (weight 1-c) and idx2 (weight c).
 * Full trajectory storage; no checkpointing. */
static void chain_vjp(const or_problem *P, const double *tail_mass, const double *inertia,
                      const double *x, const double *lam_next, double *lam_x, double *lam_u) {
    /* semi-implicit Euler: v' = v + dt a(q, v, u), q' = q + dt v'.
     * mu = lambda_v' + dt lambda_q' is the total adjoint of v'. */
    int d = P->m;
    double dt = P->dt;
    const double *q = x;
    const double *lq = lam_next, *lv = lam_next + d;
    double *mu = (double *)malloc(sizeof(double) * (size_t)d);
    double *cphi = (double *)malloc(sizeof(double) * (size_t)d);
    double *S = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double phi = 0.0;
    for (int r = 0; r < d; ++r) {
        phi += q[r];
        cphi[r] = cos(phi);
    }
    /* S_t = sum_{r>=t} l_r M_r cos(phi_r); dG_j/dq_s = g S_{max(j,s)} */
    S[d] = 0.0;
    for (int t = d - 1; t >= 0; --t) S[t] = S[t + 1] + P->len[t] * tail_mass[t] * cphi[t];
    for (int j = 0; j < d; ++j) mu[j] = lv[j] + dt * lq[j];
    for (int s = 0; s < d; ++s) {
        /* (d a / d q)^T mu: a_j = (... - k_j q_j - G_j)/I_j */
        double acc = -P->stiff[s] * mu[s] / inertia[s];
        for (int j = 0; j < d; ++j) {
            int t = j > s ? j : s;
            acc -= P->gravity * S[t] * mu[j] / inertia[j];
        }
        lam_x[s] = lq[s] + dt * acc;
        lam_x[d + s] = mu[s] - dt * P->damp[s] / inertia[s] * mu[s];
        lam_u[s] = dt * mu[s] / inertia[s];
    }
    free(mu); free(cphi); free(S);
}

static void linear_vjp(const or_problem *P, const double *lam_next, double *lam_x,
                       double *lam_u) {
    int n = P->n, m = P->m;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += P->Ad[i * n + j] * lam_next[i];
        lam_x[j] = s;
    }
    for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += P->Bd[i * m + j] * lam_next[i];
        lam_u[j] = s;
    }
}

static void grad_one(const or_problem *P, const double *x0, const double *knots, int64_t ld,
                     int64_t cand, double *dJ, int64_t ldg, double *cost) {
    int n = P->n, m = P->m, T = P->T, pm = P->p * P->m;
    double *traj = (double *)malloc(sizeof(double) * (size_t)(T + 1) * n);
    double *lam = (double *)malloc(sizeof(double) * (size_t)n);
    double *lamx = (double *)malloc(sizeof(double) * (size_t)n);
    double *lamu = (double *)malloc(sizeof(double) * (size_t)m);
    double *u = (double *)malloc(sizeof(double) * (size_t)m);
    double *tm = NULL, *in = NULL;
    if (P->model == OR_PENDULUM_CHAIN) {
        tm = (double *)malloc(sizeof(double) * (size_t)m);
        in = (double *)malloc(sizeof(double) * (size_t)m);
        chain_constants(P, tm, in);
    }
    double J = or_rollout_one(P, x0, knots, ld, cand, traj);
    if (cost) cost[cand] = J;
    for (int j = 0; j < pm; ++j) dJ[(int64_t)j * ldg + cand] = 0.0;
    const double *xT = traj + (size_t)T * n;
    for (int i = 0; i < n; ++i) {
        double e = xT[i] - x_goal_at(P, i);
        lam[i] = 2.0 * (P->q[i] + (P->qf ? P->qf[i] : 0.0)) * e + box_penalty_grad(P, xT, i);
    }
    for (int k = T - 1; k >= 0; --k) {
        const double *xk = traj + (size_t)k * n;
        or_input_at(P, knots, ld, cand, k, u);
        if (P->model == OR_LINEAR)
            linear_vjp(P, lam, lamx, lamu);
        else
            chain_vjp(P, tm, in, xk, lam, lamx, lamu);
        int a, b;
        double c;
        or_knot_weights(T, P->p, k, &a, &b, &c);
        for (int i = 0; i < m; ++i) {
            double g = 2.0 * P->r[i] * (u[i] - u_goal_at(P, i)) + lamu[i];
            dJ[(int64_t)(a * m + i) * ldg + cand] += (1.0 - c) * g;
            dJ[(int64_t)(b * m + i) * ldg + cand] += c * g;
        }
        if (k > 0)
            for (int i = 0; i < n; ++i)
                lam[i] = 2.0 * P->q[i] * (xk[i] - x_goal_at(P, i)) + box_penalty_grad(P, xk, i) + lamx[i];
    }
    free(traj); free(lam); free(lamx); free(lamu); free(u); free(tm); free(in);
}

void or_grad(const or_problem *P, const double *x0, const double *knots, int64_t ncand,
             int64_t ld, double *dJ, double *cost) {
    for (int64_t c = 0; c < ncand; ++c) grad_one(P, x0, knots, ld, c, dJ, ld, cost);
}

/* Gradient refinement of candidates by Adam (Kingma & Ba 2015: beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected moments), `steps` updates each
 * followed by a clamp to the input bounds; a refined candidate replaces the
 * original only if its cost is lower.  knots [p*m][ld] and cost [ncand] are
 * updated in place; cost must hold the candidates' current costs. */
void or_refine(const or_problem *P, const double *x0, double *knots, int64_t ncand, int64_t ld,
               double *cost, double lr, int steps) {
    int pm = P->p * P->m, m = P->m;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    double *U = (double *)malloc(sizeof(double) * (size_t)pm);
    double *g = (double *)malloc(sizeof(double) * (size_t)pm);
    double *m1 = (double *)malloc(sizeof(double) * (size_t)pm);
    double *m2 = (double *)malloc(sizeof(double) * (size_t)pm);
    for (int64_t c = 0; c < ncand; ++c) {
        for (int j = 0; j < pm; ++j) {
            U[j] = knots[(int64_t)j * ld + c];
            m1[j] = 0.0;
            m2[j] = 0.0;
        }
        for (int t = 1; t <= steps; ++t) {
            double Jc;
            grad_one(P, x0, U, 1, 0, g, 1, &Jc);
            double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
            for (int j = 0; j < pm; ++j) {
                m1[j] = b1 * m1[j] + (1.0 - b1) * g[j];
                m2[j] = b2 * m2[j] + (1.0 - b2) * g[j] * g[j];
                double mh = m1[j] / c1, vh = m2[j] / c2;
                U[j] -= lr * mh / (sqrt(vh) + eps);
                int i = j % m;
                if (U[j] < P->u_min[i]) U[j] = P->u_min[i];
                if (U[j] > P->u_max[i]) U[j] = P->u_max[i];
            }
        }
        double Jnew = or_rollout_one(P, x0, U, 1, 0, NULL);
        if (Jnew < cost[c]) {
            cost[c] = Jnew;
            for (int j = 0; j < pm; ++j) knots[(int64_t)j * ld + c] = U[j];
        }
    }
    free(U); free(g); free(m1); free(m2);
}

/* ---------------------------------------------------------------------------
 * One EMPC solve (one control tick): `generations` rounds of {population,
 * simulate and cost, select} (Alg. 1, applied once per generation as in
 * Sec. V), then u* = get_u_from_U(U_best, 0).
 * elite_knots [k][p*m] and *has_elites carry the warm start between ticks
 * (has_elites = 0 -> cold start).  Work arrays: knots_ws [p*m][pop],
 * cost_ws [pop], idx_ws [k].  gen_best (optional) receives the best cost of
 * each generation.  refine != 0 applies or_refine to the elites after each
 * selection.  Returns the index of the best candidate in the last
 * generation. */
/* ---------------------------------------------------------------------------
 * Warm start moved one control step later (a variant; the paper keeps the
 * parents as they are).  Knot a sits at step a (T-1)/(p-1); the moved knot a
 * is the carried input one step after that time, which lies between knots a
 * and a+1 at the fraction d = (p-1)/(T-1) of their spacing, so
 * U'_a = (1-d) U_a + d U_{a+1}; the last knot has no successor and is held.
 * rows: k rows of p*m parameters, moved in place. */
void or_shift_knots(const or_problem *P, double *rows, int k) {
    int m = P->m, p = P->p, pm = p * m;
    if (p < 2) return;
    double d = (double)(p - 1) / (double)(P->T - 1);
    for (int s = 0; s < k; ++s) {
        double *U = rows + (size_t)s * pm;
        for (int a = 0; a < p - 1; ++a)
            for (int i = 0; i < m; ++i) U[a * m + i] = (1.0 - d) * U[a * m + i] + d * U[(a + 1) * m + i];
    }
}

/* Mutation noise of a solve from state x0 (Sec. VII: exploration noise as a
 * function of the distance to the goal; the function is not given, so: linear
 * in the Euclidean distance, sigma_min at the goal, sigma from sigma_dist
 * on).  sigma_dist = 0 keeps sigma. */
double or_sigma_at(const or_problem *P, const or_ga *G, const double *x0) {
    if (!(G->sigma_dist > 0.0)) return G->sigma;
    double d2 = 0.0;
    for (int i = 0; i < P->n; ++i) {
        double e = x0[i] - x_goal_at(P, i);
        d2 += e * e;
    }
    double r = sqrt(d2) / G->sigma_dist;
    if (r > 1.0) r = 1.0;
    return G->sigma_min + (G->sigma - G->sigma_min) * r;
}

int or_solve(const or_problem *P, const or_ga *G, double *elite_knots, int *has_elites,
             const double *x0, uint32_t tick, double *u_star, double *best_cost,
             double *gen_best, double *knots_ws, double *cost_ws, int64_t *idx_ws, int refine,
             double lr, int adam_steps) {
    int pm = P->p * P->m, k = G->n_elite;
    int64_t pop = G->pop;
    int64_t best = 0;
    int best_slot = 0;
    double *ek = (double *)malloc(sizeof(double) * (size_t)k * pm);
    double *ec = (double *)malloc(sizeof(double) * (size_t)k);
    or_ga Gt = *G; /* this solve's noise */
    Gt.sigma = or_sigma_at(P, G, x0);
    if (G->shift && *has_elites) or_shift_knots(P, elite_knots, k);
    for (int g = 0; g < G->generations; ++g) {
        or_next_population(P, &Gt, elite_knots, !*has_elites, tick, (uint32_t)g, knots_ws, pop);
        or_rollout_cost(P, x0, knots_ws, pop, pop, cost_ws);
        or_select(cost_ws, pop, k, idx_ws, &best);
        for (int s = 0; s < k; ++s) {
            for (int j = 0; j < pm; ++j) elite_knots[(size_t)s * pm + j] = knots_ws[(int64_t)j * pop + idx_ws[s]];
            ec[s] = cost_ws[idx_ws[s]];
            if (idx_ws[s] == best) best_slot = s;
        }
        if (refine) {
            for (int s = 0; s < k; ++s)
                for (int j = 0; j < pm; ++j) ek[(int64_t)j * k + s] = elite_knots[(size_t)s * pm + j];
            or_refine(P, x0, ek, k, k, ec, lr, adam_steps);
            for (int s = 0; s < k; ++s)
                for (int j = 0; j < pm; ++j) elite_knots[(size_t)s * pm + j] = ek[(int64_t)j * k + s];
            /* best after refinement: first in (isnan(J), J, slot) order among
             * the elites */
            best_slot = 0;
            for (int s = 1; s < k; ++s)
                if (cost_cmp(ec[s], s, ec[best_slot], best_slot) < 0) best_slot = s;
        }
        *has_elites = 1;
        if (gen_best) gen_best[g] = ec[best_slot];
    }
    *best_cost = ec[best_slot];
    /* u*(i) = get_u_from_U(U_best(i), t = 0) */
    int a, b;
    double c;
    or_knot_weights(P->T, P->p, 0, &a, &b, &c);
    for (int i = 0; i < P->m; ++i) {
        const double *Ub = elite_knots + (size_t)best_slot * pm;
        u_star[i] = (1.0 - c) * Ub[a * P->m + i] + c * Ub[b * P->m + i];
    }
    free(ek);
    free(ec);
    return best_slot;
}
