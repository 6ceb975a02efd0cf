"""Pins of the N-link planar robot oracle (the robot of the paper's Sec. IV-F
setup and Sec. VI-A EMPC experiments): closed forms, invariants of
Lagrangian mechanics and finite differences, none of which shares the
oracle's formulation (mass matrix from the mass points' Jacobians, Coriolis
terms from Christoffel symbols, Jacobians by the complex step)."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def robot(N, seed=0, uniform=False):
    rng = np.random.default_rng(seed)
    if uniform:
        return np.ones(N), np.full(N, 0.25)
    return rng.uniform(0.5, 2.0, N), rng.uniform(0.1, 0.4, N)


def test_two_link_closed_form(O):
    # the textbook two-link arm with point masses at the link ends:
    # M11 = m1 l1^2 + m2 (l1^2 + l2^2 + 2 l1 l2 cos q2), M12 = m2 (l2^2 + l1 l2 cos q2),
    # M22 = m2 l2^2; with h = -m2 l1 l2 sin q2: C1 = h qd2^2 + 2 h qd1 qd2, C2 = -h qd1^2
    rng = np.random.default_rng(3)
    for _ in range(5):
        (m1, m2), (l1, l2) = rng.uniform(0.5, 2, 2), rng.uniform(0.1, 0.5, 2)
        q, qd = rng.uniform(-3, 3, 2), rng.uniform(-2, 2, 2)
        M, C = O.nlink_mass_matrix([m1, m2], [l1, l2], q, qd)
        c2 = np.cos(q[1])
        Mw = np.array([[m1 * l1**2 + m2 * (l1**2 + l2**2 + 2 * l1 * l2 * c2),
                        m2 * (l2**2 + l1 * l2 * c2)],
                       [m2 * (l2**2 + l1 * l2 * c2), m2 * l2**2]])
        h = -m2 * l1 * l2 * np.sin(q[1])
        Cw = np.array([h * qd[1]**2 + 2 * h * qd[0] * qd[1], -h * qd[0]**2])
        np.testing.assert_allclose(M, Mw, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(C, Cw, rtol=1e-13, atol=1e-15)


def test_one_link_is_eq5_without_gravity(O):
    # m l^2 qdd + b qd = tau (eq. 5 with g = 0, the plane is horizontal)
    m, l, b = 1.3, 0.25, 0.01
    for q, qd, tau in ((0.4, -1.2, 0.7), (-2.0, 3.0, -1.5)):
        f = O.nlink_deriv([m], [l], b, [q, qd], [tau])
        np.testing.assert_allclose(f, [qd, (tau - b * qd) / (m * l * l)], rtol=1e-15)
        # its ZOH model is the closed form of qdd = -(b / I) qd + tau / I
        Ad, Bd, wd = O.nlink_linearize([m], [l], b, [q, qd], [tau], 0.01)
        a = b / (m * l * l)
        e = np.exp(-a * 0.01)
        np.testing.assert_allclose(Ad, [[1, (1 - e) / a], [0, e]], rtol=1e-13)
        np.testing.assert_allclose(
            Bd[:, 0], [(0.01 - (1 - e) / a) / (m * l * l * a), (1 - e) / (m * l * l * a)],
            rtol=1e-10)
        # the one-link model is linear: no offset
        np.testing.assert_allclose(wd, 0, atol=1e-16)


@pytest.mark.parametrize("N", [1, 3, 7, 13])
def test_kinetic_energy_matches_mass_matrix(O, N):
    # 1/2 qd^T M qd equals the kinetic energy summed from the mass points'
    # velocities (no mass matrix involved); M is symmetric positive definite
    mass, length = robot(N, N)
    rng = np.random.default_rng(N + 10)
    for _ in range(4):
        q, qd = rng.uniform(-np.pi, np.pi, N), rng.uniform(-2, 2, N)
        M, _ = O.nlink_mass_matrix(mass, length, q)
        np.testing.assert_allclose(0.5 * qd @ M @ qd, O.nlink_kinetic(mass, length, q, qd),
                                   rtol=1e-13)
        np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-14 * np.abs(M).max())
        assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("N", [2, 5, 13])
def test_undamped_robot_conserves_energy(O, N):
    # no gravity, no damping, no torque: the kinetic energy is constant
    mass, length = robot(N, 1, uniform=True)
    rng = np.random.default_rng(N)
    x = np.concatenate([rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)])
    e0 = O.nlink_kinetic(mass, length, x[:N], x[N:])
    for _ in range(20):
        x = O.nlink_rk4(mass, length, 0.0, x, np.zeros(N), 0.01, 10)
    e1 = O.nlink_kinetic(mass, length, x[:N], x[N:])
    assert abs(e1 - e0) <= 1e-9 * e0


@pytest.mark.parametrize("N", [2, 6, 13])
def test_power_balance_and_lagrange_equation(O, N):
    # dE/dt = qd^T (tau - b qd) (the Coriolis terms do no work), and
    # d/dt (M qd) - 1/2 d(qd^T M qd)/dq = tau - b qd (Lagrange's equation),
    # both by central differences along the exact flow of the oracle's
    # dynamics (a dropped or mis-signed Coriolis term fails both)
    mass, length = robot(N, 2)
    b = 0.05
    rng = np.random.default_rng(N + 1)
    x = np.concatenate([rng.uniform(-2, 2, N), rng.uniform(-1.5, 1.5, N)])
    tau = rng.uniform(-1, 1, N)
    h = 1e-5
    xp = O.nlink_rk4(mass, length, b, x, tau, h, 4)
    xm = O.nlink_rk4(mass, length, b, x, tau, -h, 4)
    q, qd = x[:N], x[N:]
    E = lambda y: O.nlink_kinetic(mass, length, y[:N], y[N:])  # noqa: E731
    dE = (E(xp) - E(xm)) / (2 * h)
    np.testing.assert_allclose(dE, qd @ (tau - b * qd), rtol=1e-5)
    Mp, _ = O.nlink_mass_matrix(mass, length, xp[:N])
    Mm, _ = O.nlink_mass_matrix(mass, length, xm[:N])
    dp = (Mp @ xp[N:] - Mm @ xm[N:]) / (2 * h)
    g = np.zeros(N)
    for s in range(N):
        e = np.zeros(N)
        e[s] = 1e-6
        Ma, _ = O.nlink_mass_matrix(mass, length, q + e)
        Mb, _ = O.nlink_mass_matrix(mass, length, q - e)
        g[s] = 0.5 * qd @ (Ma - Mb) @ qd / 2e-6
    np.testing.assert_allclose(dp - g, tau - b * qd, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("N", [1, 4, 13])
def test_complex_step_jacobian_matches_central_differences(O, N):
    mass, length = robot(N, 4)
    rng = np.random.default_rng(N + 2)
    x = np.concatenate([rng.uniform(-2, 2, N), rng.uniform(-1, 1, N)])
    tau = rng.uniform(-2, 2, N)
    A, B, f0 = O.nlink_jacobian(mass, length, 0.01, x, tau)
    np.testing.assert_allclose(f0, O.nlink_deriv(mass, length, 0.01, x, tau), rtol=0, atol=0)
    h = 1e-4
    scale = max(1.0, np.abs(A).max(), np.abs(B).max())
    for s in range(2 * N + N):
        xp, xm, tp, tm = x.copy(), x.copy(), tau.copy(), tau.copy()
        if s < 2 * N:
            xp[s] += h
            xm[s] -= h
            col = A[:, s]
        else:
            tp[s - 2 * N] += h
            tm[s - 2 * N] -= h
            col = B[:, s - 2 * N]
        fd = (O.nlink_deriv(mass, length, 0.01, xp, tp) -
              O.nlink_deriv(mass, length, 0.01, xm, tm)) / (2 * h)
        # truncation O(h^2) relative; rounding of f (amplified by the
        # conditioning of M, about 1e4 at 13 links) over 2h absolute
        np.testing.assert_allclose(col, fd, rtol=1e-5, atol=1e-7 * scale)
    # the position rows are [0 I]
    np.testing.assert_array_equal(A[:N, :N], 0)
    np.testing.assert_array_equal(A[:N, N:], np.eye(N))
    np.testing.assert_array_equal(B[:N], 0)


@pytest.mark.parametrize("N", [2, 9])
def test_linearized_model_zoh(O, N):
    # (A_d, B_d, w_d) is the zero-order hold of the affine expansion
    # y' = A y + B tau + w: it equals a fine RK4 integration of that linear
    # ODE; and the affine flow agrees with the robot's own flow in value,
    # slope (f) and curvature (A f) at the linearization point, so its step
    # error is third order in dt (halving dt divides it by 8): a wrong offset
    # w leaves a first-order error, a wrong Jacobian a second-order one
    mass, length = robot(N, 5)
    rng = np.random.default_rng(N + 3)
    x = np.concatenate([rng.uniform(-1, 1, N), rng.uniform(-0.5, 0.5, N)])
    tau = rng.uniform(-1, 1, N)
    A, B, f0 = O.nlink_jacobian(mass, length, 0.01, x, tau)
    w = f0 - A @ x - B @ tau
    Ad, Bd, wd = O.nlink_linearize(mass, length, 0.01, x, tau, 0.01)
    y, h = x.copy(), 0.01 / 2000
    g = lambda v: A @ v + B @ tau + w  # noqa: E731
    for _ in range(2000):
        k1 = g(y)
        k2 = g(y + 0.5 * h * k1)
        k3 = g(y + 0.5 * h * k2)
        k4 = g(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    np.testing.assert_allclose(Ad @ x + Bd @ tau + wd, y, rtol=1e-12, atol=1e-13)
    errs = []
    for dt in (0.02, 0.01):
        Ad, Bd, wd = O.nlink_linearize(mass, length, 0.01, x, tau, dt)
        errs.append(np.abs(Ad @ x + Bd @ tau + wd -
                           O.nlink_rk4(mass, length, 0.01, x, tau, dt, 256)).max())
    assert 6.0 < errs[0] / errs[1] < 10.0


def test_rk4_converges_at_fourth_order(O):
    # the plant integrator: the error against a very fine solution drops by
    # 2^4 when the substep halves
    mass, length = robot(5, 6)
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.uniform(-1, 1, 5), rng.uniform(-3, 3, 5)])
    tau = rng.uniform(-2, 2, 5)
    ref = O.nlink_rk4(mass, length, 0.01, x, tau, 0.2, 4096)
    e1 = np.abs(O.nlink_rk4(mass, length, 0.01, x, tau, 0.2, 16) - ref).max()
    e2 = np.abs(O.nlink_rk4(mass, length, 0.01, x, tau, 0.2, 32) - ref).max()
    assert 12.0 < e1 / e2 < 20.0
