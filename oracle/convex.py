"""Parameterized small-matrix convex MPC, FP64 reference (the paper's
Sec. IV-B small-matrix formulation with the knot parameterization of
Sec. IV-E).

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: the test suite, the
smoke check and the benchmark's CPU-baseline leg are its only callers.

With z the knot vector (z[j m + i] = knot j of input i), the stacked states
[x_1 .. x_T] = S z + v and inputs [u_0 .. u_{T-1}] = Phi z, so the cost of
eq. 3 (stage cost on x_1..x_T, terminal weight Q_f on x_T) is the quadratic
    J(z) = z^T P z + 2 q^T z + c,
    P = S^T Qb S + Phi^T Rb Phi,   q = S^T Qb (v - X_g) - Phi^T Rb U_g,
    c = (v - X_g)^T Qb (v - X_g) + U_g^T Rb U_g,
Qb = blockdiag(Q, .., Q, Q + Q_f), Rb = blockdiag(R, .., R).  The columns of
S are built here as the oracle's own simulations of unit knots from rest
(no matrix powers), v as the simulation of zero knots from x0.  Knot bounds
u_min <= z <= u_max keep every interpolated input in bounds (convexity), so
the parameterized MPC is the box-constrained QP min J(z), solved exactly by
bounded-variable least squares (Stark & Parker 1995, scipy's bvls) on the
factored form J(z) = |L^T z + L^-1 q|^2 + const, P = L L^T.

Parity pins (tests/test_convex_pins.py): P, q, c equal the paper's
construction of S from powers of A_d and J(z) the oracle's simulated cost;
the minimizer meets the optimality conditions (zero projected gradient, no
feasible perturbation lowers the cost), equals -P^-1 q when no bound is
active, and the enumeration of the active sets of two-variable problems;
the evolutionary solve's best cost is bounded below by the minimum.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import knot_weights, rollout_one


def qp_form(prob, x0):
    """(P [pm][pm], q [pm], c) of a linear problem at state x0."""
    n, m, T, p = prob.n, prob.m, prob.T, prob.p
    pm = p * m
    x0 = np.asarray(x0, dtype=np.float64)
    rest = dataclasses.replace(prob, wd=np.zeros(n), qb=None)
    S = np.zeros((T * n, pm))
    for j in range(pm):
        e = np.zeros((pm, 1))
        e[j, 0] = 1.0
        _, traj = rollout_one(rest, np.zeros(n), e)
        S[:, j] = traj[1:].reshape(-1)
    _, traj = rollout_one(dataclasses.replace(prob, qb=None), x0, np.zeros((pm, 1)))
    v = traj[1:].reshape(-1)
    Phi = np.zeros((T * m, pm))
    for k in range(T):
        a, b, cw = knot_weights(T, p, k)
        for i in range(m):
            Phi[k * m + i, a * m + i] += 1.0 - cw
            Phi[k * m + i, b * m + i] += cw
    qdiag = np.tile(prob.q, T)
    if prob.qf is not None:
        qdiag[-n:] += prob.qf
    rdiag = np.tile(prob.r, T)
    Xg = np.tile(prob.x_goal if prob.x_goal is not None else np.zeros(n), T)
    Ug = np.tile(prob.u_goal if prob.u_goal is not None else np.zeros(m), T)
    P = S.T @ (qdiag[:, None] * S) + Phi.T @ (rdiag[:, None] * Phi)
    q = S.T @ (qdiag * (v - Xg)) - Phi.T @ (rdiag * Ug)
    c = float((v - Xg) @ (qdiag * (v - Xg)) + Ug @ (rdiag * Ug))
    return P, q, c


def qp_cost(P, q, c, z):
    z = np.asarray(z, dtype=np.float64)
    return float(z @ P @ z + 2.0 * q @ z + c)


def qp_solve(P, q, lo, hi):
    """Exact minimizer of z^T P z + 2 q^T z over lo <= z <= hi (P positive
    definite), by bounded-variable least squares."""
    import scipy.linalg
    import scipy.optimize

    L = scipy.linalg.cholesky(P, lower=True)
    A = L.T
    b = -scipy.linalg.solve_triangular(L, q, lower=True)
    r = scipy.optimize.lsq_linear(A, b, bounds=(lo, hi), method="bvls", tol=1e-15,
                                  lsmr_tol=None, max_iter=10 * len(q) + 100)
    return np.clip(r.x, lo, hi)


def knot_bounds(prob):
    """Per-knot bounds of z (each input's bounds repeated over the knots)."""
    return np.tile(prob.u_min, prob.p), np.tile(prob.u_max, prob.p)
