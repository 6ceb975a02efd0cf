"""Pins of the parameterized small-matrix convex MPC oracle (oracle/convex.py,
the paper's Sec. IV-B form with the knot parameterization of Sec. IV-E):
the quadratic form against the paper's matrix-power construction of S and
against the oracle's own simulated costs; the box-QP minimizer against the
optimality conditions, the unconstrained closed form, and enumeration of
the active sets on two-variable problems."""
import numpy as np
import pytest

import workloads as W
from test_oracle_pins import box_qp_min, quadratic_form, random_linear


@pytest.fixture(scope="module")
def C(oracle_lib):
    from oracle import convex

    return convex


@pytest.mark.parametrize("n,m,T,p", [(5, 3, 12, 4), (4, 2, 20, 5), (6, 2, 15, 15), (3, 1, 10, 1)])
def test_qp_form_matches_matrix_powers_and_simulation(oracle_lib, C, n, m, T, p):
    # S from unit-knot simulations equals the paper's construction from powers
    # of A_d; J(z) equals the simulated cost of z
    prob = random_linear(n, m, T, p, seed=3 + n + T)
    x0 = np.random.default_rng(1).normal(0, 1, n)
    P, q, c = C.qp_form(prob, x0)
    Pw, qw, cw = quadratic_form(prob, x0)
    np.testing.assert_allclose(P, Pw, rtol=1e-11, atol=1e-12 * np.abs(Pw).max())
    np.testing.assert_allclose(q, qw, rtol=1e-11, atol=1e-12 * np.abs(qw).max())
    np.testing.assert_allclose(c, cw, rtol=1e-12)
    Z = np.random.default_rng(2).uniform(-1, 1, (p * m, 8))
    J = oracle_lib.rollout_cost(prob, x0, Z)
    for k in range(8):
        np.testing.assert_allclose(C.qp_cost(P, q, c, Z[:, k]), J[k], rtol=1e-10)


def kkt_residual(P, q, z, lo, hi):
    """Largest violation of the box-QP optimality conditions: the projected
    gradient step z - clip(z - g) with g = P z + q (zero exactly at the
    minimizer)."""
    g = P @ z + q
    return np.abs(z - np.clip(z - g, lo, hi)).max()


@pytest.mark.parametrize("seed", range(4))
def test_qp_solve_meets_optimality_conditions(C, seed):
    prob = random_linear(6, 3, 20, 5, seed=seed)
    x0 = np.random.default_rng(seed).normal(0, 2, 6)
    P, q, c = C.qp_form(prob, x0)
    lo, hi = C.knot_bounds(prob)
    z = C.qp_solve(P, q, lo, hi)
    assert np.all(z >= lo) and np.all(z <= hi)
    assert kkt_residual(P, q, z, lo, hi) < 1e-9 * max(1.0, np.abs(q).max())
    # no feasible perturbation lowers the cost
    J = C.qp_cost(P, q, c, z)
    rng = np.random.default_rng(seed + 50)
    for _ in range(50):
        y = np.clip(z + rng.normal(0, 1e-3, z.shape), lo, hi)
        assert C.qp_cost(P, q, c, y) >= J - 1e-12 * abs(J)


def test_qp_solve_interior_is_the_unconstrained_minimum(C):
    prob = random_linear(4, 2, 15, 4, seed=11)
    prob.u_min, prob.u_max = np.full(2, -1e6), np.full(2, 1e6)
    x0 = np.array([0.3, -0.2, 0.1, 0.5])
    P, q, c = C.qp_form(prob, x0)
    lo, hi = C.knot_bounds(prob)
    np.testing.assert_allclose(C.qp_solve(P, q, lo, hi), -np.linalg.solve(P, q), rtol=1e-9,
                               atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_qp_solve_two_variables_by_enumeration(C, seed):
    # m = 1, p = 2: the minimum over the 3^2 active-set patterns
    prob = W.linear_chain(1, 10, 2, seed=seed)
    x0 = np.array([0.8, -0.5]) * (1 + 2 * seed)
    P, q, c = C.qp_form(prob, x0)
    lo, hi = C.knot_bounds(prob)
    z = C.qp_solve(P, q, lo, hi)
    np.testing.assert_allclose(C.qp_cost(P, q, c, z), box_qp_min(P, q, c, -1.0, 1.0),
                               rtol=1e-12, atol=1e-14)


def test_empc_never_beats_the_convex_optimum(oracle_lib, C):
    # every in-bounds knot vector costs at least the box-QP minimum, so the
    # evolutionary solve's best cost is bounded below by it (and approaches it)
    prob, ga = W.config_c1(0)
    x0 = W.draw_x0(prob.n, 0)
    P, q, c = C.qp_form(prob, x0)
    lo, hi = C.knot_bounds(prob)
    Jstar = C.qp_cost(P, q, c, C.qp_solve(P, q, lo, hi))
    ga = W.dataclasses.replace(ga, generations=40)
    _, Jbest, _ = oracle_lib.Solver(prob, ga).solve(x0, 0)
    assert Jstar - 1e-12 * abs(Jstar) <= Jbest <= Jstar * 1.05
