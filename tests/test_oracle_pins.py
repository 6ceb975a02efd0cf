"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: the
paper's worked examples (Sec. IV-D/E), its small-matrix closed form
(Sec. IV-B), published Philox known-answer vectors, an independent Philox
implementation, library sorts, brute force over tiny problems, invariants of
the dynamics, and finite differences.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

import workloads as W
from conftest import load_golden

# ---------------------------------------------------------------------------
# helpers that build the paper's small-matrix closed form independently of
# the oracle's step-by-step simulation


def hat_weights(T, p):
    """W[k, j]: weight of knot j at step k, from the hat functions of
    piecewise-linear interpolation with knots at k = j (T-1)/(p-1)."""
    Wt = np.zeros((T, p))
    if p == 1:
        Wt[:, 0] = 1.0
        return Wt
    for k in range(T):
        for j in range(p):
            Wt[k, j] = max(0.0, 1.0 - abs(k * (p - 1) - j * (T - 1)) / (T - 1))
    return Wt


def small_matrix(A, B, w, x0, T, p):
    """S (nT x pm), v (nT), Phi (Tm x pm) with [x_1..x_T] = S z + v and
    [u_0..u_{T-1}] = Phi z, z[j*m + i] = knot j of input i (Sec. IV-B/E)."""
    n, m = B.shape
    Wt = hat_weights(T, p)
    powers = [np.eye(n)]
    for _ in range(T):
        powers.append(A @ powers[-1])
    S = np.zeros((n * T, p * m))
    v = np.zeros(n * T)
    for k in range(1, T + 1):
        blk = np.zeros((n, p * m))
        for j in range(k):
            for kn in range(p):
                blk[:, kn * m:(kn + 1) * m] += Wt[j, kn] * powers[k - 1 - j] @ B
        S[(k - 1) * n:k * n] = blk
        v[(k - 1) * n:k * n] = powers[k] @ x0 + sum(powers[i] @ w for i in range(k))
    Phi = np.zeros((T * m, p * m))
    for k in range(T):
        for kn in range(p):
            Phi[k * m:(k + 1) * m, kn * m:(kn + 1) * m] = Wt[k, kn] * np.eye(m)
    return S, v, Phi


def quadratic_form(prob, x0):
    """P, q, c with J(z) = z'Pz + 2q'z + c (small-matrix form with the
    constant term written out; terminal weight on the last block)."""
    T, n, m = prob.T, prob.n, prob.m
    S, v, Phi = small_matrix(prob.Ad, prob.Bd, prob.wd, x0, T, prob.p)
    qdiag = np.tile(prob.q, T)
    qdiag[-n:] += prob.qf
    Qb = np.diag(qdiag)
    Rb = np.diag(np.tile(prob.r, T))
    Xg = np.tile(prob.x_goal, T)
    Ug = np.tile(prob.u_goal, T)
    P = S.T @ Qb @ S + Phi.T @ Rb @ Phi
    q = S.T @ Qb @ (v - Xg) - Phi.T @ Rb @ Ug
    c = (v - Xg) @ Qb @ (v - Xg) + Ug @ Rb @ Ug
    return P, q, c


def random_linear(n, m, T, p, seed, goal=True):
    rng = np.random.default_rng(seed)
    A = rng.normal(0, 1, (n, n))
    A *= 0.95 / max(abs(np.linalg.eigvals(A)))
    B = rng.normal(0, 1, (n, m))
    prob = W.Problem(model=W.LINEAR, n=n, m=m, T=T, p=p, Ad=A, Bd=B, wd=rng.normal(0, 0.1, n),
                     q=rng.uniform(0.5, 2, n), r=rng.uniform(0.01, 0.1, m),
                     qf=rng.uniform(0, 1, n),
                     x_goal=rng.normal(0, 1, n) if goal else np.zeros(n),
                     u_goal=rng.normal(0, 0.2, m) if goal else np.zeros(m),
                     u_min=-np.ones(m), u_max=np.ones(m))
    return prob


def knots_to_z(knots, cand):
    return knots[:, cand].copy()


# ---------------------------------------------------------------------------
# Philox


def test_philox_known_answers(oracle_lib):
    for row in load_golden("philox4x32_10_kat.txt"):
        vals = [int(x, 16) for x in row]
        assert oracle_lib.philox4x32_10(vals[0:4], vals[4:6]) == vals[6:10]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(oracle_lib, tmp_path):
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_probe.cpp")
    exe = str(tmp_path / "probe")
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", src, "-o", exe],
                   check=True, capture_output=True)
    rng = np.random.default_rng(11)
    cases = rng.integers(0, 2**32, (64, 6), dtype=np.uint64)
    text = "\n".join(" ".join("%08x" % v for v in row) for row in cases) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    for row, ref in zip(cases, got):
        assert oracle_lib.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:]]) == ref


# ---------------------------------------------------------------------------
# knot interpolation and the parameterized matrices (Sec. IV-C/D/E)


def test_knot_weights_worked_example(oracle_lib):
    for row in load_golden("knot_weights_T5_p3.txt"):
        k = int(row[0])
        want = np.array([float(x) for x in row[1:]])
        a, b, c = oracle_lib.knot_weights(5, 3, k)
        got = np.zeros(3)
        got[a] += 1.0 - c
        got[b] += c
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("T,p", [(5, 3), (50, 10), (100, 10), (20, 5), (37, 6), (7, 7), (9, 1),
                                 (1, 1), (2, 2), (100, 3)])
def test_knot_weights_match_hat_functions(oracle_lib, T, p):
    Wt = hat_weights(T, p)
    for k in range(T):
        a, b, c = oracle_lib.knot_weights(T, p, k)
        got = np.zeros(p)
        got[a] += 1.0 - c
        got[b] += c
        np.testing.assert_allclose(got, Wt[k], rtol=0, atol=1e-15)
        assert 0 <= a <= b <= p - 1 and 0.0 <= c < 1.0


def test_knot_count_equal_horizon_is_traditional_mpc(oracle_lib):
    # p = T: every step applies its own knot exactly (Sec. III-C)
    for T in (1, 2, 5, 50):
        for k in range(T):
            a, b, c = oracle_lib.knot_weights(T, T, k)
            assert a == k and c == 0.0


def test_parameterized_S_worked_example(oracle_lib):
    rng = np.random.default_rng(3)
    n, m, T, p = 4, 2, 5, 3
    A = rng.normal(0, 0.5, (n, n))
    B = rng.normal(0, 1, (n, m))
    prob = W.Problem(model=W.LINEAR, n=n, m=m, T=T, p=p, Ad=A, Bd=B, wd=np.zeros(n),
                     q=np.ones(n), r=np.ones(m), qf=np.zeros(n), x_goal=np.zeros(n),
                     u_goal=np.zeros(m), u_min=-np.ones(m) * 10, u_max=np.ones(m) * 10)
    pw = [np.linalg.matrix_power(A, e) for e in range(5)]
    # S columns from unit-knot rollouts from x0 = 0
    S = np.zeros((n * T, p * m))
    for col in range(p * m):
        knots = np.zeros((p * m, 1))
        knots[col, 0] = 1.0
        _, traj = oracle_lib.rollout_one(prob, np.zeros(n), knots)
        S[:, col] = traj[1:].reshape(-1)
    for row in load_golden("param_S_T5_p3.txt"):
        i, j = int(row[0]), int(row[1])
        coef = [float(x) for x in row[2:]]
        blk = sum(c * pw[e] for e, c in enumerate(coef)) @ B
        np.testing.assert_allclose(S[(i - 1) * n:i * n, j * m:(j + 1) * m], blk, rtol=0,
                                   atol=1e-13)


# ---------------------------------------------------------------------------
# linear rollout and cost against the closed forms of Sec. IV-B


@pytest.mark.parametrize("n,m,T,p", [(5, 3, 12, 4), (4, 2, 20, 5), (6, 6, 9, 9), (3, 1, 7, 1),
                                     (8, 3, 30, 30)])
def test_linear_rollout_closed_form(oracle_lib, n, m, T, p):
    prob = random_linear(n, m, T, p, seed=n * 100 + T)
    rng = np.random.default_rng(5)
    x0 = rng.normal(0, 1, n)
    knots = rng.uniform(-1, 1, (p * m, 3))
    S, v, Phi = small_matrix(prob.Ad, prob.Bd, prob.wd, x0, T, p)
    for cand in range(3):
        _, traj = oracle_lib.rollout_one(prob, x0, knots, cand)
        want = S @ knots[:, cand] + v
        np.testing.assert_allclose(traj[1:].reshape(-1), want, rtol=1e-12, atol=1e-12)
        np.testing.assert_array_equal(traj[0], x0)


@pytest.mark.parametrize("n,m,T,p", [(5, 3, 12, 4), (4, 2, 20, 5), (6, 2, 15, 15), (3, 1, 10, 1)])
def test_linear_cost_quadratic_form(oracle_lib, n, m, T, p):
    prob = random_linear(n, m, T, p, seed=7 + n + T)
    rng = np.random.default_rng(9)
    x0 = rng.normal(0, 1, n)
    knots = rng.uniform(-1, 1, (p * m, 16))
    P, q, c = quadratic_form(prob, x0)
    J = oracle_lib.rollout_cost(prob, x0, knots)
    for cand in range(16):
        z = knots[:, cand]
        np.testing.assert_allclose(J[cand], z @ P @ z + 2 * q @ z + c, rtol=1e-10)


def test_linear_trajectory_with_linear_knots(oracle_lib):
    # knots on a line are reproduced exactly at every step by linear
    # interpolation: u_k = alpha + beta * k (p-1)/(T-1)
    n, m, T, p = 3, 2, 17, 5
    prob = random_linear(n, m, T, p, seed=1)
    alpha, beta = np.array([0.2, -0.3]), np.array([0.1, 0.05])
    knots = np.array([[alpha[i] + beta[i] * j] for j in range(p) for i in range(m)])
    x = np.zeros(n)
    _, traj = oracle_lib.rollout_one(prob, x, knots)
    for k in range(T):
        u = alpha + beta * k * (p - 1) / (T - 1)
        x = prob.Ad @ x + prob.Bd @ u + prob.wd
        np.testing.assert_allclose(traj[k + 1], x, rtol=1e-13, atol=1e-14)


def test_equilibrium_stays(oracle_lib):
    lin = W.linear_chain(3, 25, 5, seed=2)
    ch = W.pendulum_chain(5, 40, 6, seed=2)
    for prob in (lin, ch):
        knots = np.zeros((prob.p * prob.m, 2))
        J, traj = oracle_lib.rollout_one(prob, np.zeros(prob.n), knots)
        assert J == 0.0
        assert np.all(traj == 0.0)


# ---------------------------------------------------------------------------
# pendulum chain: reductions and invariants


def chain_positions(prob, q):
    """Planar positions of the point masses, angles from the downward vertical."""
    phi = np.cumsum(q)
    x = np.cumsum(prob.length * np.sin(phi))
    y = -np.cumsum(prob.length * np.cos(phi))
    return x, y


def test_chain_single_link_is_eq5(oracle_lib):
    # one link: m l^2 qdd + b qd + m g l sin q + k q = tau, semi-implicit Euler
    prob = W.pendulum_chain(1, 10, 2, seed=4)
    ml2 = prob.mass[0] * prob.length[0] ** 2
    x = np.array([0.7, -0.3])
    u = np.array([0.4])
    qdd = (u[0] - prob.damping[0] * x[1] - prob.mass[0] * prob.gravity * prob.length[0] *
           np.sin(x[0]) - prob.stiffness[0] * x[0]) / ml2
    qd = x[1] + prob.dt * qdd
    want = np.array([x[0] + prob.dt * qd, qd])
    np.testing.assert_allclose(oracle_lib.step(prob, x, u), want, rtol=1e-14)


def test_chain_gravity_torque_is_potential_gradient(oracle_lib):
    # with k = b = 0 and qd = 0, applying u = dV/dq (central differences of
    # V = g sum m_i y_i) holds the chain still for one step
    prob = W.pendulum_chain(7, 10, 2, seed=5)
    prob.stiffness[:] = 0.0
    prob.damping[:] = 0.0
    rng = np.random.default_rng(1)
    q = rng.normal(0, 0.6, 7)

    def V(qq):
        _, y = chain_positions(prob, qq)
        return prob.gravity * np.sum(prob.mass * y)

    h = 1e-5
    grad = np.array([(V(q + h * e) - V(q - h * e)) / (2 * h) for e in np.eye(7)])
    x = np.concatenate([q, np.zeros(7)])
    xn = oracle_lib.step(prob, x, grad)
    assert np.max(np.abs(xn[7:])) < 1e-6
    # and without the compensating torque the chain does move
    xn0 = oracle_lib.step(prob, x, np.zeros(7))
    assert np.max(np.abs(xn0[7:])) > 1e-3


def test_chain_inertia_is_mass_matrix_diagonal(oracle_lib):
    # g = k = b = 0 and a unit torque at joint j from rest, straight chain:
    # qd_j' = dt / M_jj(0), with M_jj = sum_i m_i |d p_i / d q_j|^2 by
    # finite differences of the forward kinematics
    d = 6
    prob = W.pendulum_chain(d, 10, 2, seed=6)
    prob.stiffness[:] = 0.0
    prob.damping[:] = 0.0
    prob.gravity = 0.0
    h = 1e-6
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        xp, yp = chain_positions(prob, e)
        xm, ym = chain_positions(prob, -e)
        Mjj = np.sum(prob.mass * (((xp - xm) / (2 * h)) ** 2 + ((yp - ym) / (2 * h)) ** 2))
        u = np.zeros(d)
        u[j] = 1.0
        xn = oracle_lib.step(prob, np.zeros(2 * d), u)
        np.testing.assert_allclose(xn[d + j], prob.dt / Mjj, rtol=1e-8)


def test_chain_energy_bounded(oracle_lib):
    # undamped, unforced: semi-implicit Euler keeps the energy
    # 1/2 sum I_j qd_j^2 + V(q) from drifting (it oscillates about its start)
    d = 4
    prob = W.pendulum_chain(d, 10, 2, seed=8)
    prob.damping[:] = 0.0
    inertia = np.array([prob.dt / oracle_lib.step(
        W.dataclasses.replace(prob, gravity=0.0, stiffness=np.zeros(d)), np.zeros(2 * d),
        np.eye(d)[j])[d + j] for j in range(d)])

    def energy(x):
        _, y = chain_positions(prob, x[:d])
        return (0.5 * np.sum(inertia * x[d:] ** 2) + prob.gravity * np.sum(prob.mass * y) +
                0.5 * np.sum(prob.stiffness * x[:d] ** 2))

    x = np.concatenate([np.full(d, 0.3), np.zeros(d)])
    E0 = energy(x)
    Es = []
    for _ in range(4000):
        x = oracle_lib.step(prob, x, np.zeros(d))
        Es.append(energy(x))
    Es = np.array(Es)
    scale = abs(E0 - prob.gravity * np.sum(prob.mass * chain_positions(prob, np.zeros(d))[1]))
    assert np.max(np.abs(Es - E0)) < 0.1 * scale
    # no secular drift: first and last quarter average the same
    assert abs(Es[-1000:].mean() - Es[:1000].mean()) < 0.02 * scale


def test_chain_c3_instance_is_stable(oracle_lib):
    # the configuration's 36-link chain stays finite over the horizon from
    # x0 ~ N(0, 0.5^2) under bounded random inputs
    prob = W.pendulum_chain(36, 100, 10, seed=0)
    x0 = W.draw_x0(prob.n, 0)
    knots = W.draw_knots(prob, 8, seed=1)
    J = oracle_lib.rollout_cost(prob, x0, knots)
    assert np.all(np.isfinite(J))
    _, traj = oracle_lib.rollout_one(prob, x0, knots, 0)
    assert np.max(np.abs(traj)) < 1e3


# ---------------------------------------------------------------------------
# selection


def test_select_matches_library_sort(oracle_lib):
    rng = np.random.default_rng(4)
    for trial in range(20):
        pop = int(rng.integers(1, 400))
        k = int(rng.integers(1, pop + 1))
        cost = np.round(rng.normal(0, 1, pop), 1)  # many exact ties
        cost[rng.random(pop) < 0.05] = np.nan
        cost[rng.random(pop) < 0.02] = np.inf
        # library sort on (isnan, J, index): NaN after every number, +inf
        # included (np.lexsort sorts by its last key first)
        isnan = np.isnan(cost)
        order = np.lexsort((np.arange(pop), np.where(isnan, 0.0, cost), isnan))
        idx, best = oracle_lib.select(cost, k)
        np.testing.assert_array_equal(idx, np.sort(order[:k]))
        assert best == order[0]


def test_select_nan_ranks_after_inf(oracle_lib):
    # a NaN at a lower index than a +inf still ranks after it
    idx, best = oracle_lib.select([np.nan, np.inf], 1)
    assert list(idx) == [1] and best == 1
    idx, best = oracle_lib.select([np.nan, np.inf, 1.0], 2)
    assert list(idx) == [1, 2] and best == 2
    idx, best = oracle_lib.select([np.nan, np.nan, -np.inf], 2)
    assert list(idx) == [0, 2] and best == 2
    # -0 and +0 tie, broken by index
    idx, best = oracle_lib.select([0.0, -0.0, 1.0], 1)
    assert list(idx) == [0] and best == 0


# ---------------------------------------------------------------------------
# evolutionary step: distributions, bounds, elitism


def _ga_problem(m=6, p=5):
    return W.linear_chain(m, 20, p, seed=1)


def test_cold_start_uniform(oracle_lib):
    prob = _ga_problem()
    prob.u_min = np.linspace(-2, -0.5, prob.m)
    prob.u_max = np.linspace(0.5, 3, prob.m)
    ga = W.GA(pop=4000, n_elite=8, generations=1, sigma=0.1, seed=3)
    K = oracle_lib.next_population(prob, ga, None, cold=True, tick=0, gen=0)
    for j in range(prob.p * prob.m):
        i = j % prob.m
        z = (K[j] - prob.u_min[i]) / (prob.u_max[i] - prob.u_min[i])
        assert z.min() > 0 and z.max() < 1
        assert scipy.stats.kstest(z, "uniform").pvalue > 1e-4


def test_elites_kept_and_children_in_bounds(oracle_lib):
    prob = _ga_problem()
    rng = np.random.default_rng(2)
    k = 8
    E = rng.uniform(-1, 1, (k, prob.p * prob.m))
    ga = W.GA(pop=512, n_elite=k, generations=1, sigma=3.0, seed=5)
    K = oracle_lib.next_population(prob, ga, E, cold=False, tick=4, gen=2)
    np.testing.assert_array_equal(K[:, :k].T, E)
    assert K.min() >= -1.0 and K.max() <= 1.0
    assert np.mean(np.abs(K[:, k:]) == 1.0) > 0.2  # heavy noise does clamp
    ga2 = W.dataclasses.replace(ga, elitism=False)
    K2 = oracle_lib.next_population(prob, ga2, E, cold=False, tick=4, gen=2)
    assert not np.array_equal(K2[:, :k].T, E)


def test_crossover_parents_and_mutation_statistics(oracle_lib):
    prob = _ga_problem(m=6, p=5)
    pm = prob.p * prob.m
    k = 16
    # elite s holds the constant value v_s everywhere
    vals = np.linspace(-0.75, 0.75, k)
    E = np.repeat(vals[:, None], pm, axis=1)
    pop = 20000
    ga0 = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.0, seed=9)
    K = oracle_lib.next_population(prob, ga0, E, cold=False, tick=1, gen=0)[:, k:]
    # sigma = 0: every parameter is one of the two parents' values
    ids = np.rint((K + 0.75) / 1.5 * (k - 1)).astype(int)
    np.testing.assert_allclose(K, vals[ids], atol=1e-15)
    # each child draws from at most 2 parents; parents uniform over k
    nuniq = np.array([len(np.unique(ids[:, c])) for c in range(ids.shape[1])])
    assert nuniq.max() <= 2
    first = ids.min(axis=0)
    second = ids.max(axis=0)
    counts = np.bincount(np.concatenate([first, second]), minlength=k)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4
    # crossover: among children with two distinct parents, each parameter
    # comes from either with probability 1/2
    two = nuniq == 2
    frac = np.mean(ids[:, two] == first[two])
    assert abs(frac - 0.5) < 0.01
    # mutation: elites at 0, sigma 0.1, far from the bounds
    E0 = np.zeros((k, pm))
    ga1 = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=10)
    K1 = oracle_lib.next_population(prob, ga1, E0, cold=False, tick=1, gen=3)[:, k:]
    mutated = K1 != 0.0  # (pm, children)
    per_input = mutated.reshape(prob.p, prob.m, -1)
    # a flagged input has all of its knots perturbed, an unflagged one none
    assert np.all(per_input.all(axis=0) == per_input.any(axis=0))
    assert abs(per_input[0].mean() - 0.5) < 0.01
    z = K1[mutated] / 0.1
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4


# ---------------------------------------------------------------------------
# solve: brute force on tiny problems, elitism invariant


def box_qp_min(P, q, c, lo, hi):
    """Exact minimum of z'Pz + 2q'z + c over a 2-D box by active sets."""
    best = np.inf
    for s0 in ("f", "l", "u"):
        for s1 in ("f", "l", "u"):
            z = np.zeros(2)
            free = []
            for i, s in enumerate((s0, s1)):
                if s == "l":
                    z[i] = lo
                elif s == "u":
                    z[i] = hi
                else:
                    free.append(i)
            if free:
                fixed = [i for i in range(2) if i not in free]
                rhs = -q[free] - P[np.ix_(free, fixed)] @ z[fixed]
                z[free] = np.linalg.solve(P[np.ix_(free, free)], rhs)
            if np.all(z >= lo - 1e-12) and np.all(z <= hi + 1e-12):
                best = min(best, z @ P @ z + 2 * q @ z + c)
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_empc_brute_force_tiny(oracle_lib, seed):
    prob = W.linear_chain(1, 10, 2, seed=seed)
    x0 = np.array([0.8, -0.5]) * (1 + seed)
    P, q, c = quadratic_form(prob, x0)
    Jbox = box_qp_min(P, q, c, -1.0, 1.0)
    g = np.linspace(-1, 1, 201)
    Z = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    Jgrid = np.einsum("ki,ij,kj->k", Z, P, Z) + 2 * Z @ q + c
    L = 2 * np.linalg.norm(P, 2) * np.sqrt(2) + 2 * np.linalg.norm(q)
    assert Jbox <= Jgrid.min() + 1e-12
    assert Jgrid.min() <= Jbox + L * 0.01
    # grid values agree with the oracle's simulation
    Kg = Z[::97].T.copy()
    np.testing.assert_allclose(oracle_lib.rollout_cost(prob, x0, Kg), Jgrid[::97], rtol=1e-10)
    ga = W.GA(pop=256, n_elite=16, generations=50, sigma=0.1, seed=seed)
    s = oracle_lib.Solver(prob, ga)
    u, Jbest, gen_best = s.solve(x0, tick=0)
    assert Jbox - 1e-12 <= Jbest <= Jgrid.min() + 1e-9
    assert np.all(np.diff(gen_best) <= 0)
    assert np.all(np.abs(s.elite_knots) <= 1.0)
    # u* is knot 0 of the best candidate
    assert u[0] == s.elite_knots[s.best_slot, 0]


def test_solve_warm_start_and_elitism_over_ticks(oracle_lib):
    prob, ga = W.config_c1(0)
    ga = W.dataclasses.replace(ga, generations=4)
    s = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    for tick in range(3):
        u, J, gb = s.solve(x, tick)
        assert np.all(np.diff(gb) <= 0)
        assert np.all(np.abs(u) <= 1.0)
        x = oracle_lib.step(prob, x, u)
    # a second solver run with the same seed repeats bit for bit
    s2 = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    u1, J1, _ = s2.solve(x, 0)
    s3 = oracle_lib.Solver(prob, ga)
    u2, J2, _ = s3.solve(x, 0)
    assert J1 == J2 and np.array_equal(u1, u2)


# ---------------------------------------------------------------------------
# warm-start variants: parents moved one step later, distance-dependent noise


@pytest.mark.parametrize("T,p", [(9, 5), (13, 4), (21, 11)])
def test_shift_samples_the_carried_input_one_step_later(oracle_lib, T, p):
    # knot a sits at step a (T-1)/(p-1), an integer for these (T, p); the moved
    # knot must be the carried piecewise-linear input at that step plus one,
    # evaluated with the interpolation weights of Sec. IV-C (pinned above by
    # the worked example), and the last knot is held
    m = 3
    prob = W.linear_chain(m, T, p, seed=1)
    rng = np.random.default_rng(5)
    rows = rng.uniform(-1, 1, (4, p * m))
    moved = oracle_lib.shift_knots(prob, rows)
    step = (T - 1) // (p - 1)
    for s in range(rows.shape[0]):
        U = rows[s].reshape(p, m)
        for a in range(p - 1):
            ka, kb, c = oracle_lib.knot_weights(T, p, a * step + 1)
            want = (1 - c) * U[ka] + c * U[kb]
            np.testing.assert_allclose(moved[s].reshape(p, m)[a], want, rtol=0, atol=1e-15)
        np.testing.assert_array_equal(moved[s].reshape(p, m)[p - 1], U[p - 1])


def test_shift_special_cases(oracle_lib):
    rng = np.random.default_rng(6)
    # p = T: every step has its own knot, so the move is exactly "next knot"
    prob = W.linear_chain(2, 7, 7, seed=2)
    rows = rng.uniform(-1, 1, (3, 14))
    moved = oracle_lib.shift_knots(prob, rows)
    np.testing.assert_array_equal(moved[:, :12], rows[:, 2:])
    np.testing.assert_array_equal(moved[:, 12:], rows[:, 12:])
    # p = 1: a constant input has nothing to move
    prob1 = W.linear_chain(2, 7, 1, seed=2)
    rows1 = rng.uniform(-1, 1, (3, 2))
    np.testing.assert_array_equal(oracle_lib.shift_knots(prob1, rows1), rows1)
    # a constant trajectory stays constant
    prob5 = W.linear_chain(2, 10, 4, seed=2)
    const = np.tile(np.array([0.3, -0.7]), (2, 4))
    np.testing.assert_allclose(oracle_lib.shift_knots(prob5, const), const, rtol=0, atol=1e-15)


def test_sigma_schedule(oracle_lib):
    prob = W.linear_chain(2, 10, 4, seed=3)
    ga = W.GA(pop=8, n_elite=2, generations=1, sigma=0.4, seed=1, sigma_min=0.05, sigma_dist=2.0)
    goal = np.zeros(prob.n)
    assert oracle_lib.sigma_at(prob, ga, goal) == 0.05
    e = np.array([0.6, 0.0, 0.8, 0.0])  # distance 1 = half of sigma_dist
    np.testing.assert_allclose(oracle_lib.sigma_at(prob, ga, e), 0.05 + 0.35 * 0.5, rtol=1e-15)
    assert oracle_lib.sigma_at(prob, ga, 3 * e) == 0.4  # beyond sigma_dist
    plain = W.dataclasses.replace(ga, sigma_dist=0.0)
    assert oracle_lib.sigma_at(prob, plain, goal) == 0.4


def test_solve_noise_schedule_limits(oracle_lib):
    # at the goal with sigma_min = 0 the schedule gives no noise, so the solve
    # equals one with sigma = 0; at or beyond sigma_dist it equals the plain
    # solve with sigma
    prob = W.linear_chain(2, 12, 4, seed=4)
    ga = W.GA(pop=64, n_elite=8, generations=3, sigma=0.3, seed=9, sigma_min=0.0, sigma_dist=1.0)
    far = np.full(prob.n, 2.0)
    for x0, twin in ((np.zeros(prob.n), W.dataclasses.replace(ga, sigma=0.0, sigma_dist=0.0)),
                     (far, W.dataclasses.replace(ga, sigma_dist=0.0))):
        a, b = oracle_lib.Solver(prob, ga), oracle_lib.Solver(prob, twin)
        for tick in range(2):
            ua, Ja, _ = a.solve(x0, tick)
            ub, Jb, _ = b.solve(x0, tick)
            assert Ja == Jb and np.array_equal(ua, ub)
            assert np.array_equal(a.elite_knots, b.elite_knots)


def test_solve_shift_moves_carried_parents_once_per_tick(oracle_lib):
    # with the shift, a tick equals the plain tick started from the carried
    # parents moved one step later; the first (cold) tick has nothing to move
    prob = W.linear_chain(2, 17, 5, seed=8)
    ga = W.GA(pop=48, n_elite=6, generations=2, sigma=0.1, seed=4, shift=True)
    a = oracle_lib.Solver(prob, ga)
    b = oracle_lib.Solver(prob, W.dataclasses.replace(ga, shift=False))
    x = W.draw_x0(prob.n, 3)
    for tick in range(3):
        if tick > 0:
            b.elite_knots[:] = oracle_lib.shift_knots(prob, b.elite_knots)
        ua, Ja, _ = a.solve(x, tick)
        ub, Jb, _ = b.solve(x, tick)
        assert Ja == Jb and np.array_equal(ua, ub), tick
        x = oracle_lib.step(prob, x, ua)


# ---------------------------------------------------------------------------
# state box as a soft constraint


def with_box(prob, lo, hi, qb):
    out = W.dataclasses.replace(prob)
    out.x_min = np.full(prob.n, float(lo)) if np.isscalar(lo) else np.asarray(lo, float)
    out.x_max = np.full(prob.n, float(hi)) if np.isscalar(hi) else np.asarray(hi, float)
    out.qb = np.full(prob.n, float(qb)) if np.isscalar(qb) else np.asarray(qb, float)
    return out


def test_box_penalty_inside_is_free(oracle_lib):
    prob = W.linear_chain(3, 20, 4, seed=1)
    x0 = W.draw_x0(prob.n, 1)
    knots = W.draw_knots(prob, 8, seed=1)
    plain = oracle_lib.rollout_cost(prob, x0, knots)
    boxed = oracle_lib.rollout_cost(with_box(prob, -1e6, 1e6, 5.0), x0, knots)
    np.testing.assert_array_equal(plain, boxed)


def test_box_penalty_closed_form(oracle_lib):
    # x_{k+1} = x_k (A = 1, B = 0), q = r = 0: the state sits at x0 outside
    # the box for all T steps, so J = T qb (x0 - x_max)^2, and mirrored below
    for x0, lo, hi in ((2.5, -1.0, 1.0), (-3.0, -1.0, 0.5)):
        T = 17
        prob = W.Problem(model=W.LINEAR, n=1, m=1, T=T, p=3, Ad=np.ones((1, 1)),
                         Bd=np.zeros((1, 1)), q=np.zeros(1), r=np.zeros(1), qf=np.zeros(1),
                         x_goal=np.zeros(1), u_goal=np.zeros(1), u_min=-np.ones(1),
                         u_max=np.ones(1))
        knots = W.draw_knots(prob, 3, seed=2)
        d = x0 - hi if x0 > hi else lo - x0
        J = oracle_lib.rollout_cost(with_box(prob, lo, hi, 0.7), np.array([x0]), knots)
        np.testing.assert_allclose(J, T * 0.7 * d * d, rtol=1e-14)


@pytest.mark.parametrize("mk", [W.linear_chain, W.pendulum_chain])
def test_box_penalty_point_box_is_extra_state_weight(oracle_lib, mk):
    # a zero-width box at the goal makes the penalty qb_i (x_i - g_i)^2 on
    # x_1..x_T: the stage cost with q_i + qb_i and no box (terminal term
    # untouched), with some weights zero
    prob = mk(4, 30, 6, seed=6)
    prob.x_goal = np.linspace(-0.1, 0.1, prob.n)
    prob.qf = np.linspace(0.5, 1.0, prob.n)
    w = np.where(np.arange(prob.n) % 3 == 0, 0.0, 0.7)
    x0 = W.draw_x0(prob.n, 6)
    knots = W.draw_knots(prob, 20, seed=6)
    boxed = oracle_lib.rollout_cost(with_box(prob, prob.x_goal, prob.x_goal, w), x0, knots)
    heavier = oracle_lib.rollout_cost(W.dataclasses.replace(prob, q=prob.q + w), x0, knots)
    np.testing.assert_allclose(boxed, heavier, rtol=1e-13)


@pytest.mark.parametrize("model", ["linear", "chain"])
def test_box_penalty_gradient_central_differences(oracle_lib, model):
    # the penalty is piecewise quadratic: away from the box faces central
    # differences with h = 1e-4 are exact up to rounding for the linear
    # model and O(h^2) for the chain
    if model == "linear":
        prob = with_box(W.linear_chain(3, 25, 5, seed=4), -0.05, 0.05, 4.0)
    else:
        prob = with_box(W.pendulum_chain(4, 25, 5, seed=4), -0.1, 0.1, 3.0)
    x0 = W.draw_x0(prob.n, 4)
    knots = W.draw_knots(prob, 2, seed=4)
    dJ, cost = oracle_lib.grad(prob, x0, knots)
    plain = W.dataclasses.replace(prob, qb=None, x_min=None, x_max=None)
    assert np.all(cost > oracle_lib.rollout_cost(plain, x0, knots))  # the box is active
    h = 1e-4
    for cand in range(2):
        fd = np.zeros(prob.p * prob.m)
        for j in range(prob.p * prob.m):
            kp = knots[:, cand:cand + 1].copy()
            km = kp.copy()
            kp[j] += h
            km[j] -= h
            fd[j] = (oracle_lib.rollout_cost(prob, x0, kp)[0] -
                     oracle_lib.rollout_cost(prob, x0, km)[0]) / (2 * h)
        np.testing.assert_allclose(dJ[:, cand], fd, rtol=1e-4, atol=1e-5 * np.abs(fd).max())


# ---------------------------------------------------------------------------
# adjoint gradient


@pytest.mark.parametrize("n,m,T,p", [(5, 3, 12, 4), (4, 2, 20, 5), (6, 2, 9, 9)])
def test_grad_linear_matches_quadratic_form(oracle_lib, n, m, T, p):
    prob = random_linear(n, m, T, p, seed=21 + n)
    rng = np.random.default_rng(2)
    x0 = rng.normal(0, 1, n)
    knots = rng.uniform(-1, 1, (p * m, 5))
    P, q, c = quadratic_form(prob, x0)
    dJ, cost = oracle_lib.grad(prob, x0, knots)
    for cand in range(5):
        z = knots[:, cand]
        want = 2 * P @ z + 2 * q
        np.testing.assert_allclose(dJ[:, cand], want, rtol=1e-9, atol=1e-10 * np.abs(want).max())
        np.testing.assert_allclose(cost[cand], z @ P @ z + 2 * q @ z + c, rtol=1e-10)


def test_grad_chain_central_differences(oracle_lib):
    prob = W.pendulum_chain(5, 30, 4, seed=3)
    prob.qf = np.full(prob.n, 0.5)
    x0 = W.draw_x0(prob.n, 3)
    knots = W.draw_knots(prob, 2, seed=3)
    dJ, cost = oracle_lib.grad(prob, x0, knots)
    h = 1e-3
    for cand in range(2):
        fd = np.zeros(prob.p * prob.m)
        for j in range(prob.p * prob.m):
            kp = knots[:, cand:cand + 1].copy()
            km = kp.copy()
            kp[j] += h
            km[j] -= h
            fd[j] = (oracle_lib.rollout_cost(prob, x0, kp)[0] -
                     oracle_lib.rollout_cost(prob, x0, km)[0]) / (2 * h)
        np.testing.assert_allclose(dJ[:, cand], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_refine_never_increases_cost(oracle_lib):
    prob = W.linear_chain(3, 20, 4, seed=1)
    x0 = W.draw_x0(prob.n, 1)
    knots = W.draw_knots(prob, 6, seed=2)
    cost = oracle_lib.rollout_cost(prob, x0, knots)
    k2, c2 = oracle_lib.refine(prob, x0, knots, cost, lr=0.01, steps=5)
    assert np.all(c2 <= cost)
    assert np.sum(c2 < cost) >= 4  # convex problem: Adam makes progress
    np.testing.assert_allclose(oracle_lib.rollout_cost(prob, x0, k2), c2, rtol=1e-12)
    assert np.all(np.abs(k2) <= 1.0)


# Adam (Kingma & Ba 2015, Algorithm 1) on a one-parameter quadratic: n = m =
# T = p = 1, A_d = 0, B_d = 1, goal 1, so x_1 = u and J(u) = q (u - 1)^2,
# dJ/du = 2 q (u - 1).


def _scalar_quadratic(q=1.0, lo=-10.0, hi=10.0, goal=1.0):
    one = np.ones(1)
    return W.Problem(model=W.LINEAR, n=1, m=1, T=1, p=1, q=q * one, r=0 * one, qf=0 * one,
                     x_goal=goal * one, u_goal=0 * one, u_min=lo * one, u_max=hi * one,
                     Ad=np.zeros((1, 1)), Bd=np.ones((1, 1)), wd=np.zeros(1))


def _adam_decimal(u0, q, lr, steps, lo, hi, goal=1.0, clamp_each=True):
    """The bias-corrected Adam recursion on q (u - goal)^2, with a clamp after
    every update (or, clamp_each=False, once at the end), evaluated in
    40-digit decimal arithmetic (independent of the oracle's binary64 code
    path)."""
    from decimal import Decimal as D, getcontext

    getcontext().prec = 40
    b1, b2, eps = D("0.9"), D("0.999"), D("1e-8")
    u, m, v = D(repr(u0)), D(0), D(0)
    for t in range(1, steps + 1):
        g = 2 * D(repr(q)) * (u - D(repr(goal)))
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh, vh = m / (1 - b1 ** t), v / (1 - b2 ** t)
        u = u - D(repr(lr)) * mh / (vh.sqrt() + eps)
        if clamp_each:
            u = min(max(u, D(repr(lo))), D(repr(hi)))
    return float(min(max(u, D(repr(lo))), D(repr(hi))))


def _refine1(oracle_lib, prob, u0, lr, steps):
    knots = np.array([[u0]])
    cost = oracle_lib.rollout_cost(prob, np.zeros(1), knots)
    k2, c2 = oracle_lib.refine(prob, np.zeros(1), knots, cost, lr=lr, steps=steps)
    return float(k2[0, 0]), float(c2[0]), float(cost[0])


def test_adam_first_step_is_lr_times_sign(oracle_lib):
    # from zero moments the bias corrections make m_hat = g and v_hat = g^2,
    # whatever beta1 and beta2 are: the first update is exactly
    # -lr g / (|g| + eps).  A missing correction would move by about
    # lr (1 - b1) / sqrt(1 - b2) = 3.16 lr.
    prob = _scalar_quadratic()
    for u0, lr in [(0.0, 0.1), (0.3, 0.01), (2.5, 0.2)]:
        g = 2 * (u0 - 1)
        u1, _, _ = _refine1(oracle_lib, prob, u0, lr, 1)
        assert abs(u1 - (u0 - lr * g / (abs(g) + 1e-8))) < 1e-15


def test_adam_steps_follow_the_recursion(oracle_lib):
    # steps 2 and 3 carry the moments: their values depend on beta1, beta2
    # and the bias corrections separately (swapped betas or a dropped
    # correction change them at the 1e-3 level)
    prob = _scalar_quadratic(q=3.0)
    for u0, lr, steps in [(0.0, 0.1, 2), (0.0, 0.1, 3), (-0.7, 0.05, 5)]:
        got, _, _ = _refine1(oracle_lib, prob, u0, lr, steps)
        assert abs(got - _adam_decimal(u0, 3.0, lr, steps, -10, 10)) < 1e-14
    # the second step from u0 = 0, lr = 0.1 (q = 1) by hand: g1 = -2,
    # u1 = 0.2 / (2 + eps) (= 0.1 up to 5e-10); g2 = 2 (u1 - 1) (about -1.8);
    # m = 0.9 (0.1 g1) + 0.1 g2, v = 0.999 (0.001 g1^2) + 0.001 g2^2;
    # m_hat = m / (1 - 0.81), v_hat = v / (1 - 0.998001)
    u1 = 0.2 / (2 + 1e-8)
    g2 = 2 * (u1 - 1)
    m = 0.9 * 0.1 * -2 + 0.1 * g2
    v = 0.999 * 0.001 * 4 + 0.001 * g2 * g2
    u2 = u1 - 0.1 * (m / 0.19) / (np.sqrt(v / 0.001999) + 1e-8)
    got, _, _ = _refine1(oracle_lib, _scalar_quadratic(), 0.0, 0.1, 2)
    assert abs(got - u2) < 1e-14
    assert abs(got - 0.1995877718) < 1e-9
    # swapped betas (m with 0.999, v with 0.9) would move u2 to about 0.1997
    m_sw = 0.999 * 0.001 * -2 + 0.001 * g2
    v_sw = 0.9 * 0.1 * 4 + 0.1 * g2 * g2
    u2_sw = u1 - 0.1 * (m_sw / 0.001999) / (np.sqrt(v_sw / 0.19) + 1e-8)
    assert abs(got - u2_sw) > 1e-5


def test_adam_clamp_binds_mid_sequence(oracle_lib):
    # the clamp acts on the parameter after every update, not once at the
    # end: goal 0.12, u_max = 0.15, from 0 with lr = 0.1 the momentum carries
    # steps 2..5 past the bound (cut to 0.15 each time, gradients then taken
    # at 0.15) before the iterate turns back; the moments keep their own
    # history
    prob = _scalar_quadratic(hi=0.15, goal=0.12)
    got, c, c0 = _refine1(oracle_lib, prob, 0.0, 0.1, 7)
    want = _adam_decimal(0.0, 1.0, 0.1, 7, -10, 0.15, goal=0.12)
    assert abs(got - want) < 1e-14
    assert abs(want - 0.1278793876) < 1e-9
    end_only = _adam_decimal(0.0, 1.0, 0.1, 7, -10, 0.15, goal=0.12, clamp_each=False)
    assert abs(got - end_only) > 0.03
    assert c < c0  # and the refined candidate is accepted


def test_adam_moments_reset_per_call_and_scale_invariance(oracle_lib):
    # each call starts from zero moments: two one-step calls are two first
    # steps
    prob = _scalar_quadratic()
    u1, _, _ = _refine1(oracle_lib, prob, 0.0, 0.1, 1)
    u2, _, _ = _refine1(oracle_lib, prob, u1, 0.1, 1)
    g1 = 2 * (u1 - 1)
    assert abs(u2 - (u1 - 0.1 * g1 / (abs(g1) + 1e-8))) < 1e-15
    # Adam's update does not depend on the gradient's scale (up to eps)
    a, _, _ = _refine1(oracle_lib, _scalar_quadratic(q=1.0), 0.2, 0.05, 4)
    b, _, _ = _refine1(oracle_lib, _scalar_quadratic(q=1000.0), 0.2, 0.05, 4)
    assert abs(a - b) < 1e-8  # eps = 1e-8 against gradients of order 1


def test_adam_rejects_a_worse_candidate(oracle_lib):
    # an update that raises the cost is not accepted: knots and cost stay
    prob = _scalar_quadratic()
    u, c, c0 = _refine1(oracle_lib, prob, 0.9, 5.0, 1)  # overshoots to 5.9
    assert u == 0.9 and c == c0
    u, c, c0 = _refine1(oracle_lib, prob, 0.0, 0.5, 1)  # 0 -> 0.5: better
    assert abs(u - 0.5) < 1e-8 and c < c0


# ---------------------------------------------------------------------------
# input generator sanity (zero-order hold)


def test_zoh_matches_closed_form_oscillator():
    # 1-DoF mass-spring-damper: A_d = expm(A dt) checked against the closed
    # form of an underdamped oscillator; A_d ~ I + A dt for small dt
    mass, k, c = 1.3, 40.0, 1.2
    A, B = W.chain_continuous(np.array([mass]), np.array([k]), np.array([c]))
    dt = 0.01
    Ad, Bd = W.zoh(A, B, dt)
    wn = np.sqrt(k / mass)
    zeta = c / (2 * np.sqrt(k * mass))
    wd = wn * np.sqrt(1 - zeta ** 2)
    e = np.exp(-zeta * wn * dt)
    x_free = e * (np.cos(wd * dt) + zeta * wn / wd * np.sin(wd * dt))
    v_free = -e * wn ** 2 / wd * np.sin(wd * dt)
    np.testing.assert_allclose(Ad[:, 0], [x_free, v_free], rtol=1e-12)
    # B_d = A^{-1}(A_d - I) B for invertible A
    np.testing.assert_allclose(Bd, np.linalg.solve(A, (Ad - np.eye(2)) @ B), rtol=1e-10)
    Ad2, _ = W.zoh(A, B, 1e-6)
    np.testing.assert_allclose(Ad2, np.eye(2) + A * 1e-6, atol=1e-10)
