"""Pins of the oracle's non-smooth terms and full weights (Sec. V-A: effects
placed in if/else branches of the simulation, costs that need not be
continuous; eq. 3 with full Q and R).

Full weights are pinned against the small-matrix closed form of Sec. IV-B
with block-diagonal full Q and R (matrix powers, no simulation loop) and
against a rotation of the state coordinates that turns a diagonal Q into a
full one (the oracle's diagonal code path on one side, its full-matrix path
on the other).  The step charge sb is pinned by trajectories known in
closed form and by the jump it makes when a bound crosses a state.  Joint
limits are pinned by the bounce of a free joint (closed form, restitution
0, 1/2 and 1) and by invariants of a driven chain.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_pins import small_matrix


def spd(n, rng, cond=20.0):
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Qm * np.geomspace(1.0, 1.0 / cond, n)) @ Qm.T


def full_weights(prob, rng, terminal=True):
    out = W.dataclasses.replace(prob)
    out.Q = spd(prob.n, rng)
    out.R = 0.05 * spd(prob.m, rng)
    out.Qf = 3.0 * spd(prob.n, rng) if terminal else None
    return out


# ---------------------------------------------------------------------------
# full Q, R, Qf


@pytest.mark.parametrize("d,T,p", [(2, 12, 4), (3, 20, 5), (5, 9, 9)])
def test_full_weights_match_small_matrix_closed_form(d, T, p):
    rng = np.random.default_rng([d, T, p])
    prob = full_weights(W.linear_chain(d, T, p, seed=d), rng)
    prob.wd = 0.01 * rng.standard_normal(prob.n)
    prob.x_goal = 0.1 * rng.standard_normal(prob.n)
    prob.u_goal = 0.1 * rng.standard_normal(prob.m)
    x0 = W.draw_x0(prob.n, d)
    knots = W.draw_knots(prob, 6, seed=d)
    S, v, Phi = small_matrix(prob.Ad, prob.Bd, prob.wd, x0, T, p)
    Qb = np.kron(np.eye(T), prob.Q)
    Qb[-prob.n:, -prob.n:] += prob.Qf
    Rb = np.kron(np.eye(T), prob.R)
    Xg, Ug = np.tile(prob.x_goal, T), np.tile(prob.u_goal, T)
    want = []
    for c in range(knots.shape[1]):
        z = knots[:, c]
        ex, eu = S @ z + v - Xg, Phi @ z - Ug
        want.append(ex @ Qb @ ex + eu @ Rb @ eu)
    got = oracle.rollout_cost(prob, x0, knots)
    np.testing.assert_allclose(got, want, rtol=1e-11)


@pytest.mark.parametrize("mixed", [False, True])
def test_full_weights_rotation_of_a_diagonal_problem(mixed):
    # x' = V x with V orthogonal: A' = V A V^T, B' = V B, w' = V w, goal
    # V g, Q' = V diag(q) V^T, Qf' = V diag(qf) V^T; the cost of every
    # candidate is unchanged.  mixed: R stays diagonal (vector r).
    rng = np.random.default_rng(11)
    prob = W.linear_chain(4, 25, 5, seed=11)
    prob.qf = rng.uniform(0.5, 2.0, prob.n)
    prob.x_goal = 0.2 * rng.standard_normal(prob.n)
    prob.wd = 0.01 * rng.standard_normal(prob.n)
    V, _ = np.linalg.qr(rng.standard_normal((prob.n, prob.n)))
    rot = W.dataclasses.replace(prob, Ad=V @ prob.Ad @ V.T, Bd=V @ prob.Bd, wd=V @ prob.wd,
                                x_goal=V @ prob.x_goal, Q=V @ np.diag(prob.q) @ V.T,
                                Qf=V @ np.diag(prob.qf) @ V.T,
                                R=None if mixed else np.diag(prob.r))
    x0 = W.draw_x0(prob.n, 11)
    knots = W.draw_knots(prob, 12, seed=11)
    plain = oracle.rollout_cost(prob, x0, knots)
    rotated = oracle.rollout_cost(rot, V @ x0, knots)
    np.testing.assert_allclose(rotated, plain, rtol=1e-12)


def test_full_weights_coupling_terms_count():
    # Q = [[1, a], [a, 1]] on a 2-state system held at x = (s, t) (A = I,
    # B = 0): every stage costs s^2 + 2 a s t + t^2, so J(a) - J(0) =
    # 2 a s t T, linear in the off-diagonal entry
    T, s_, t_ = 7, 0.3, -1.1
    base = W.Problem(model=W.LINEAR, n=2, m=1, T=T, p=2, Ad=np.eye(2), Bd=np.zeros((2, 1)),
                     q=np.ones(2), r=np.zeros(1), qf=np.zeros(2), x_goal=np.zeros(2),
                     u_goal=np.zeros(1), u_min=-np.ones(1), u_max=np.ones(1))
    knots = W.draw_knots(base, 2, seed=0)
    x0 = np.array([s_, t_])
    for a in (0.0, 0.25, -0.6):
        prob = W.dataclasses.replace(base, Q=np.array([[1.0, a], [a, 1.0]]))
        J = oracle.rollout_cost(prob, x0, knots)
        np.testing.assert_allclose(J, T * (s_ * s_ + 2 * a * s_ * t_ + t_ * t_), rtol=1e-14)


def test_full_weights_refused_by_the_adjoint():
    prob = full_weights(W.linear_chain(2, 10, 3, seed=1), np.random.default_rng(1))
    knots = W.draw_knots(prob, 2, seed=1)
    with pytest.raises(ValueError):
        oracle.grad(prob, W.draw_x0(prob.n, 1), knots)


# ---------------------------------------------------------------------------
# step charge outside the state box (discontinuous cost)


def held_problem(n, T):
    """x_{k+1} = x_k + u_k (A = I, B = I), zero weights, p = T (one knot per
    step): the trajectory is the running sum of the knots."""
    return W.Problem(model=W.LINEAR, n=n, m=n, T=T, p=T, Ad=np.eye(n), Bd=np.eye(n),
                     q=np.zeros(n), r=np.zeros(n), qf=np.zeros(n), x_goal=np.zeros(n),
                     u_goal=np.zeros(n), u_min=-np.ones(n), u_max=np.ones(n))


def test_step_charge_counts_states_outside_the_box():
    rng = np.random.default_rng(5)
    n, T = 3, 16
    prob = held_problem(n, T)
    lo, hi = np.array([-0.5, -0.2, -1.0]), np.array([0.4, 0.3, 0.1])
    sb = np.array([1.0, 2.5, 0.125])
    prob = W.dataclasses.replace(prob, x_min=lo, x_max=hi, qb=np.zeros(n), sb=sb)
    x0 = rng.uniform(-0.3, 0.3, n)
    knots = rng.uniform(-0.3, 0.3, (T * n, 5))
    got = oracle.rollout_cost(prob, x0, knots)
    for c in range(5):
        u = knots[:, c].reshape(T, n)
        xs = x0 + np.cumsum(u, axis=0)  # x_1..x_T
        outside = (xs > hi) | (xs < lo)
        assert got[c] == pytest.approx(float((outside * sb).sum()), rel=1e-15, abs=0)


def test_step_charge_jumps_when_a_bound_crosses_a_state():
    # the state sits at x0 for T steps: moving x_max from just above to just
    # below x0 adds exactly T sb (no continuity), while the squared-distance
    # term changes by only T qb eps^2
    T, x0, sb, qb, eps = 9, 0.75, 4.0, 2.0, 1e-6
    prob = held_problem(1, T)
    knots = np.zeros((T, 1))
    J = []
    for hi in (x0 + eps, x0 - eps):
        P = W.dataclasses.replace(prob, x_min=np.array([-1.0]), x_max=np.array([hi]),
                                  qb=np.array([qb]), sb=np.array([sb]))
        J.append(oracle.rollout_cost(P, np.array([x0]), knots)[0])
    assert J[0] == 0.0
    assert J[1] == pytest.approx(T * sb + T * qb * eps * eps, rel=1e-12)


def test_step_charge_with_infinite_bounds_is_free():
    prob = W.pendulum_chain(3, 20, 4, seed=2)
    x0 = W.draw_x0(prob.n, 2)
    knots = W.draw_knots(prob, 6, seed=2)
    free = W.dataclasses.replace(prob, x_min=np.full(prob.n, -np.inf),
                                 x_max=np.full(prob.n, np.inf), qb=np.ones(prob.n),
                                 sb=np.full(prob.n, 7.0))
    np.testing.assert_array_equal(oracle.rollout_cost(free, x0, knots),
                                  oracle.rollout_cost(prob, x0, knots))


# ---------------------------------------------------------------------------
# joint limits with impacts (pendulum chain)


def free_joint(restitution, q_max=0.5, T=40):
    """One link, no stiffness, damping or gravity: the joint turns at a
    constant rate until it meets the limit."""
    prob = W.pendulum_chain(1, T, 2, seed=0)
    return W.dataclasses.replace(prob, stiffness=np.zeros(1), damping=np.zeros(1), gravity=0.0,
                                 q_min=np.array([-10.0]), q_max=np.array([q_max]),
                                 restitution=restitution)


@pytest.mark.parametrize("e", [0.0, 0.5, 1.0])
def test_free_joint_bounces_off_its_limit(e):
    # semi-implicit Euler at zero torque: q_k = q0 + k dt w until the first
    # step past q_max, which lands on q_max with rate -e w; from there the
    # joint moves back at that rate (e = 0: it stays on the limit)
    prob = free_joint(e)
    dt, w, q0 = prob.dt, 3.0, 0.21
    x = np.array([q0, w])
    k_hit = int(np.floor((0.5 - q0) / (dt * w))) + 1
    for k in range(1, 25):
        x = oracle.step(prob, x, np.zeros(1))
        if k < k_hit:
            want = (q0 + k * dt * w, w)
        else:
            want = (0.5 - (k - k_hit) * dt * e * w, -e * w)
        np.testing.assert_allclose(x, want, rtol=1e-13, atol=1e-15)


def test_elastic_bounce_keeps_kinetic_energy_and_plastic_stops():
    for e, ratio in ((1.0, 1.0), (0.5, 0.25), (0.0, 0.0)):
        prob = free_joint(e)
        x = np.array([0.45, 4.0])
        for _ in range(3):
            x = oracle.step(prob, x, np.zeros(1))
        assert x[1] ** 2 == pytest.approx(ratio * 16.0, rel=1e-14, abs=1e-30)


def test_limits_hold_on_a_driven_chain_and_wide_limits_change_nothing():
    prob = W.pendulum_chain(6, 60, 6, seed=3)
    rng = np.random.default_rng(3)
    x0 = W.draw_x0(prob.n, 3)
    knots = W.draw_knots(prob, 4, seed=3)
    lim = W.dataclasses.replace(prob, q_min=np.full(6, -0.2), q_max=np.full(6, 0.25),
                                restitution=0.3)
    x0c = x0.copy()
    x0c[:6] = np.clip(x0c[:6], -0.2, 0.25)
    for c in range(4):
        _, traj = oracle.rollout_one(lim, x0c, knots, c)
        q = traj[1:, :6]
        assert np.all(q <= 0.25) and np.all(q >= -0.2)
        assert np.any(q == 0.25) or np.any(q == -0.2)  # the limits were met
    wide = W.dataclasses.replace(prob, q_min=np.full(6, -1e6), q_max=np.full(6, 1e6),
                                 restitution=float(rng.uniform()))
    np.testing.assert_array_equal(oracle.rollout_cost(wide, x0, knots),
                                  oracle.rollout_cost(prob, x0, knots))


def test_impacts_refused_by_the_adjoint():
    prob = free_joint(0.5)
    with pytest.raises(ValueError):
        oracle.grad(prob, np.array([0.0, 1.0]), W.draw_knots(prob, 2, seed=0))


# ---------------------------------------------------------------------------
# dry friction with stiction (pendulum chain)


def frictional_joint(tc, ts, T=40):
    """One link, no stiffness, damping or gravity, dry friction."""
    prob = W.pendulum_chain(1, T, 2, seed=0)
    return W.dataclasses.replace(prob, stiffness=np.zeros(1), damping=np.zeros(1), gravity=0.0,
                                 fric_c=np.array([tc]), fric_s=np.array([ts]))


def inertia(prob):
    return prob.mass[0] * prob.length[0] ** 2


def test_friction_holds_a_joint_at_rest_below_breakaway():
    prob = frictional_joint(0.2, 0.5)
    x = np.array([0.3, 0.0])
    for u in (0.49, -0.5, 0.0, 0.3):
        y = x.copy()
        for _ in range(10):
            y = oracle.step(prob, y, np.array([u]))
        np.testing.assert_array_equal(y, x)  # exactly at rest


def test_friction_breakaway_and_sliding_closed_form():
    # from rest under u > fric_s the joint accelerates at (u - fric_c) / I
    prob = frictional_joint(0.2, 0.5)
    dt, I = prob.dt, inertia(prob)
    x = np.array([0.0, 0.0])
    q = v = 0.0
    for k in range(1, 15):
        x = oracle.step(prob, x, np.array([0.8]))
        v += dt * 0.8 / I - dt / I * 0.2
        q += dt * v
        np.testing.assert_allclose(x, (q, v), rtol=1e-12, atol=1e-15)


def test_friction_slides_to_a_stop_and_sticks():
    # no torque: the rate falls by dt fric_c / I per step, then stops and stays
    prob = frictional_joint(0.3, 0.3)
    dt, I = prob.dt, inertia(prob)
    dv = dt * 0.3 / I
    v0 = 7.5 * dv
    x = np.array([0.0, v0])
    q, v = 0.0, v0
    for k in range(1, 20):
        x = oracle.step(prob, x, np.zeros(1))
        v = max(v - dv, 0.0)
        q += dt * v
        np.testing.assert_allclose(x, (q, v), rtol=1e-12, atol=1e-15)
    assert x[1] == 0.0


def test_friction_hysteresis_of_a_torque_cycle():
    # the torque needed to start the joint (fric_s) exceeds the one that
    # keeps it moving (fric_c): ramping the torque up, the joint first moves
    # once u > fric_s; ramping back down it keeps moving below fric_s
    prob = frictional_joint(0.2, 0.5)
    x = np.array([0.0, 0.0])
    up = np.linspace(0.0, 0.6, 61)
    started = None
    for i, u in enumerate(up):
        x = oracle.step(prob, x, np.array([u]))
        if started is None and x[1] != 0.0:
            started = u
    assert started is not None and started > 0.5
    for u in np.linspace(0.6, 0.3, 31):
        x = oracle.step(prob, x, np.array([u]))
        assert x[1] > 0.0  # still moving at torques below the breakaway


def test_zero_friction_changes_nothing():
    prob = W.pendulum_chain(5, 40, 5, seed=5)
    x0 = W.draw_x0(prob.n, 5)
    knots = W.draw_knots(prob, 6, seed=5)
    zero = W.dataclasses.replace(prob, fric_c=np.zeros(5), fric_s=np.zeros(5))
    np.testing.assert_array_equal(oracle.rollout_cost(zero, x0, knots),
                                  oracle.rollout_cost(prob, x0, knots))


def test_oracle_struct_matches_its_header(tmp_path):
    """Every field of the oracle's ctypes mirror sits where the C compiler
    puts it."""
    import ctypes
    import os
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    py = oracle._OrProblem
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "empc_oracle.h"',
             "int main(void) {", '  printf("size %zu\\n", sizeof(or_problem));']
    for f, _ in py._fields_:
        lines.append('  printf("%s %%zu\\n", offsetof(or_problem, %s));' % (f, f))
    lines.append("  return 0;\n}\n")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "oracle"), str(src), "-o",
                    str(exe)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(py)
    for f, _ in py._fields_:
        assert int(out[f]) == getattr(py, f).offset, f
