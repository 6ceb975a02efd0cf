"""GPU parity of the N-link planar robot (the robot of the paper's Sec. IV-F
setup and Sec. VI-A experiments) against the FP64 oracle, through the C
ABI: the relinearized discrete model (A_d, B_d, w_d), the RK4 plant, and the
whole relinearize / solve / step closed loop.

The two sides share no formulation: the kernels use a recursive
Newton-Euler pass with dual numbers and a Taylor exponential, the oracle
the Lagrangian mass matrix with Christoffel symbols, complex-step
derivatives and scipy's Pade exponential.  Tolerances: 1e-11 relative (FP64
model and plant; rounding of two different formulations, amplified by the
conditioning of M), 1e-6 (the same model rounded to FP32), 1e-9 for the
closed loop's u* and best cost (the method's FP64 bar)."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    E.lib()
    return E


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def robot_params(N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 2.0, N), rng.uniform(0.1, 0.4, N), 0.05


def gpu_linearize(E, mass, length, b, x, u, dt, dtype):
    N = len(mass)
    R = E.NLinkRobot(mass, length, b, dtype)
    Ad = torch.full((2 * N, 2 * N), float("nan"), dtype=dtype, device="cuda")
    Bd = torch.full((2 * N, N), float("nan"), dtype=dtype, device="cuda")
    wd = torch.full((2 * N,), float("nan"), dtype=dtype, device="cuda")
    E.empc_nlink_linearize(R, dt, dev(x, dtype), dev(u, dtype), Ad, Bd, wd)
    torch.cuda.synchronize()
    return (Ad.cpu().numpy().astype(np.float64), Bd.cpu().numpy().astype(np.float64),
            wd.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("N", [1, 2, 5, 13, 16])
def test_linearize_matches_oracle_fp64(oracle_lib, E, N):
    mass, length, b = robot_params(N, N)
    rng = np.random.default_rng(100 + N)
    for trial in range(3):
        x = np.concatenate([rng.uniform(-2, 2, N), rng.uniform(-1.5, 1.5, N)])
        u = rng.uniform(-2, 2, N)
        got = gpu_linearize(E, mass, length, b, x, u, 0.01, F64)
        want = oracle_lib.nlink_linearize(mass, length, b, x, u, 0.01)
        for g, w, name in zip(got, want, ("Ad", "Bd", "wd")):
            scale = max(1.0, np.abs(w).max())
            if name == "wd":
                # the offset is a difference of terms of size |A_d x| + |B_d u|
                scale = max(scale, np.abs(want[0]).max() * np.abs(x).max() +
                            np.abs(want[1]).max() * np.abs(u).max())
            np.testing.assert_allclose(g, w, rtol=1e-11, atol=1e-12 * scale, err_msg=name)


def test_linearize_large_step_needs_squaring(oracle_lib, E):
    # dt large enough that the hold matrix is scaled down and squared back
    mass, length, b = robot_params(4, 7)
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.uniform(-2, 2, 4), rng.uniform(-3, 3, 4)])
    u = rng.uniform(-2, 2, 4)
    got = gpu_linearize(E, mass, length, b, x, u, 0.5, F64)
    want = oracle_lib.nlink_linearize(mass, length, b, x, u, 0.5)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=1e-10, atol=1e-11 * max(1.0, np.abs(w).max()))


def test_linearize_fp32_outputs(oracle_lib, E):
    # FP32 robot: inputs rounded to float32, FP64 arithmetic, outputs rounded
    N = 6
    mass, length, b = robot_params(N, 3)
    mass, length = mass.astype(np.float32).astype(np.float64), length.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)]).astype(np.float32)
    u = rng.uniform(-2, 2, N).astype(np.float32)
    got = gpu_linearize(E, mass, length, b, x, u, 0.01, F32)
    want = oracle_lib.nlink_linearize(mass, length, b, x.astype(np.float64), u.astype(np.float64),
                                      0.01)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(w).max()))


def test_linearize_at_rest_is_linear_in_torque(oracle_lib, E):
    # at rest with zero torque the robot has no acceleration: w_d = 0 and
    # A_d's position-velocity block is the integrator of the damped joints
    N = 5
    mass, length, b = robot_params(N, 11)
    x = np.concatenate([np.linspace(-1, 1, N), np.zeros(N)])
    Ad, Bd, wd = gpu_linearize(E, mass, length, b, x, np.zeros(N), 0.01, F64)
    np.testing.assert_allclose(wd, 0, atol=1e-15)
    np.testing.assert_allclose(Ad[:N, :N], np.eye(N), atol=1e-15)


@pytest.mark.parametrize("N,sub", [(1, 1), (3, 4), (13, 4), (16, 2)])
def test_step_matches_oracle_fp64(oracle_lib, E, N, sub):
    mass, length, b = robot_params(N, 20 + N)
    rng = np.random.default_rng(200 + N)
    x = np.concatenate([rng.uniform(-2, 2, N), rng.uniform(-2, 2, N)])
    u = rng.uniform(-2, 2, N)
    R = E.NLinkRobot(mass, length, b, F64)
    xd = dev(x, F64)
    out = torch.empty_like(xd)
    E.empc_nlink_step(R, 0.01, sub, xd, dev(u, F64), out)
    want = oracle_lib.nlink_rk4(mass, length, b, x, u, 0.01, sub)
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-11, atol=1e-12)
    # in place (x_next = x) gives the same state
    E.empc_nlink_step(R, 0.01, sub, xd, dev(u, F64), xd)
    np.testing.assert_allclose(xd.cpu().numpy(), want, rtol=1e-11, atol=1e-12)


def test_nlink_argument_errors(E):
    R = E.NLinkRobot(np.ones(17), np.full(17, 0.25), 0.01, F64)
    x = torch.zeros(34, dtype=F64, device="cuda")
    u = torch.zeros(17, dtype=F64, device="cuda")
    with pytest.raises(E.EmpcError) as ei:
        E.empc_nlink_step(R, 0.01, 1, x, u, x)
    assert ei.value.status == E.binding.EMPC_EUNSUPPORTED
    R = E.NLinkRobot(np.ones(2), np.full(2, 0.25), 0.01, F64)
    x, u = x[:4].contiguous(), u[:2].contiguous()
    with pytest.raises(E.EmpcError):
        E.empc_nlink_step(R, 0.0, 1, x, u, x)
    with pytest.raises(E.EmpcError):
        E.empc_nlink_step(R, 0.01, 0, x, u, x)
    with pytest.raises(ValueError):
        E.empc_nlink_step(R, 0.01, 1, x.float(), u, x)


@pytest.mark.parametrize("N", [2, 4])
def test_relinearized_closed_loop_matches_oracle_fp64(oracle_lib, E, N):
    # each tick: relinearize the robot at its state and the last applied
    # torque, one EMPC solve on that model (warm-started across ticks), RK4
    # step of the robot under u*; the GPU loop follows the oracle's loop
    robot = W.nlink_robot(N)
    x0, xg = W.nlink_start_goal(N, 5)
    prob = W.nlink_problem(N, 20, 3, xg)
    ga = W.GA(pop=96, n_elite=8, generations=2, sigma=0.2, seed=3)
    R = E.NLinkRobot(robot.mass, robot.length, robot.damping, F64)
    dp = E.DeviceProblem(prob, F64, keep=("wd",))
    solver = E.Solver(dp, ga)
    osolver = oracle_lib.Solver(prob, ga)
    x, xo = dev(x0, F64), x0.copy()
    u, uo = torch.zeros(N, dtype=F64, device="cuda"), np.zeros(N)
    for tick in range(5):
        E.empc_nlink_linearize(R, 0.01, x, u, dp.tensors["Ad"], dp.tensors["Bd"],
                               dp.tensors["wd"])
        us, J = solver.solve(x, tick)
        u = us.clone()
        E.empc_nlink_step(R, 0.01, 4, x, u, x)
        Ad, Bd, wd = oracle_lib.nlink_linearize(robot.mass, robot.length, robot.damping, xo,
                                                 uo, 0.01)
        osolver.P = oracle_lib.OracleProblem(dataclasses.replace(prob, Ad=Ad, Bd=Bd, wd=wd))
        uo, Jo, _ = osolver.solve(xo, tick)
        xo = oracle_lib.nlink_rk4(robot.mass, robot.length, robot.damping, xo, uo, 0.01, 4)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        np.testing.assert_allclose(x.cpu().numpy(), xo, rtol=1e-9, atol=1e-12)
