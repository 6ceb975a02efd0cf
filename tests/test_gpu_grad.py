"""GPU adjoint (empc_grad), Adam refinement (empc_refine) and the autograd
wrapper, against the FP64 oracle's adjoint and Adam, and against central
finite differences of the GPU's own FP64 rollout cost (h = 1e-3)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    assert torch.cuda.is_available()
    E.lib()
    return E


def npdt(dtype):
    return np.float32 if dtype == F32 else np.float64


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def setup(prob, ncand, dtype, seed=0, ld=None):
    prob = prob.cast(npdt(dtype))
    x0 = W.draw_x0(prob.n, seed).astype(npdt(dtype)).astype(np.float64)
    knots = W.draw_knots(prob, ncand, seed + 3, ld=ld).astype(npdt(dtype)).astype(np.float64)
    return prob, x0, knots


def gpu_grad(E, prob, x0, knots, ncand, dtype):
    dp = E.DeviceProblem(prob, dtype)
    K = dev(knots, dtype)
    dJ = torch.full_like(K, float("nan"))
    cost = torch.zeros(ncand, dtype=dtype, device="cuda")
    E.empc_grad(dp, dev(x0, dtype), K, ncand, knots.shape[1], dJ, cost)
    torch.cuda.synchronize()
    return dJ.cpu().numpy().astype(np.float64), cost.cpu().numpy().astype(np.float64)


def rel_err_cols(got, want):
    scale = np.maximum(np.abs(want).max(axis=0), 1e-30)
    return (np.abs(got - want).max(axis=0) / scale).max()


CASES = [
    ("linear", 2, 20, 5), ("linear", 14, 50, 10), ("linear", 7, 33, 33), ("linear", 5, 17, 1),
    ("linear", 21, 40, 6), ("chain", 3, 30, 4), ("chain", 36, 100, 10), ("chain", 9, 50, 50),
]


def make(kind, d, T, p, seed=0):
    prob = (W.linear_chain if kind == "linear" else W.pendulum_chain)(d, T, p, seed=seed)
    prob.qf = np.linspace(0.2, 1.0, prob.n)
    prob.x_goal = np.linspace(-0.1, 0.2, prob.n)
    return prob


@pytest.mark.parametrize("kind,d,T,p", CASES)
def test_grad_fp64_matches_oracle(oracle_lib, E, kind, d, T, p):
    prob, x0, knots = setup(make(kind, d, T, p), 9, F64, ld=12)
    dJ, cost = gpu_grad(E, prob, x0, knots, 9, F64)
    want, wcost = oracle_lib.grad(prob, x0, knots, 9)
    assert rel_err_cols(dJ[:, :9], want[:, :9]) < 1e-9
    np.testing.assert_allclose(cost, wcost, rtol=1e-10)


@pytest.mark.parametrize("kind,d,T,p", CASES)
def test_grad_fp32_matches_oracle(oracle_lib, E, kind, d, T, p):
    prob, x0, knots = setup(make(kind, d, T, p), 64, F32)
    dJ, cost = gpu_grad(E, prob, x0, knots, 64, F32)
    want, wcost = oracle_lib.grad(prob, x0, knots, 64)
    assert rel_err_cols(dJ, want) < 2e-3
    np.testing.assert_allclose(cost, wcost, rtol=1e-4)


@pytest.mark.parametrize("kind,d,T,p", [("linear", 14, 50, 10), ("linear", 2, 20, 5),
                                         ("chain", 6, 40, 5), ("chain", 20, 30, 4)])
def test_grad_fp64_box_penalty_matches_oracle(oracle_lib, E, kind, d, T, p):
    # the state box penalty enters the cost and every adjoint step
    prob = make(kind, d, T, p)
    rng = np.random.default_rng(d)
    hw = 0.05 * rng.uniform(0.5, 1.5, prob.n)
    prob.x_min, prob.x_max = prob.x_goal - hw, prob.x_goal + hw
    prob.qb = 3.0 * rng.uniform(0.5, 2.0, prob.n)
    prob, x0, knots = setup(prob, 9, F64, ld=12)
    dJ, cost = gpu_grad(E, prob, x0, knots, 9, F64)
    want, wcost = oracle_lib.grad(prob, x0, knots, 9)
    assert rel_err_cols(dJ[:, :9], want[:, :9]) < 1e-9
    np.testing.assert_allclose(cost, wcost, rtol=1e-10)


@pytest.mark.parametrize("kind,d,T,p", [("linear", 14, 50, 10), ("chain", 6, 40, 5)])
def test_grad_fp64_central_differences(E, kind, d, T, p):
    prob, x0, knots = setup(make(kind, d, T, p), 2, F64)
    dJ, _ = gpu_grad(E, prob, x0, knots, 2, F64)
    pm = prob.p * prob.m
    h = 1e-3
    # all perturbed candidates in one rollout launch
    plus = np.repeat(knots[:, :1], pm, axis=1) + h * np.eye(pm)
    minus = np.repeat(knots[:, :1], pm, axis=1) - h * np.eye(pm)
    dp = E.DeviceProblem(prob, F64)
    cost = torch.zeros(2 * pm, dtype=F64, device="cuda")
    E.empc_rollout_cost(dp, dev(x0, F64), dev(np.hstack([plus, minus]), F64), 2 * pm, 2 * pm,
                        cost)
    c = cost.cpu().numpy()
    fd = (c[:pm] - c[pm:]) / (2 * h)
    tol = 1e-8 if kind == "linear" else 1e-5  # linear J is quadratic: FD is exact
    np.testing.assert_allclose(dJ[:, 0], fd, rtol=tol, atol=tol * np.abs(fd).max())


@pytest.mark.parametrize("kind,d,T,p", [("linear", 14, 50, 10), ("chain", 5, 30, 4)])
def test_refine_fp64_matches_oracle(oracle_lib, E, kind, d, T, p):
    prob, x0, knots = setup(make(kind, d, T, p), 16, F64)
    cost = oracle_lib.rollout_cost(prob, x0, knots)
    wk, wc = oracle_lib.refine(prob, x0, knots, cost, lr=0.01, steps=5)
    dp = E.DeviceProblem(prob, F64)
    K, C = dev(knots, F64), dev(cost, F64)
    E.empc_refine(dp, dev(x0, F64), K, 16, 16, C, 0.01, 5)
    torch.cuda.synchronize()
    np.testing.assert_allclose(C.cpu().numpy(), wc, rtol=1e-9)
    np.testing.assert_allclose(K.cpu().numpy(), wk, rtol=0, atol=1e-10)
    assert np.all(wc <= cost) and np.any(wc < cost)


def test_refine_fp32_c2_elites(oracle_lib, E):
    prob, _ = W.config_c2(0)
    prob, x0, knots = setup(prob, 64, F32)
    dp = E.DeviceProblem(prob, F32)
    K = dev(knots, F32)
    C = torch.zeros(64, dtype=F32, device="cuda")
    E.empc_rollout_cost(dp, dev(x0, F32), K, 64, 64, C)
    c0 = C.clone()
    E.empc_refine(dp, dev(x0, F32), K, 64, 64, C, 0.01, 5)
    C2 = torch.zeros_like(C)
    E.empc_rollout_cost(dp, dev(x0, F32), K, 64, 64, C2)
    torch.cuda.synchronize()
    assert torch.all(C <= c0) and torch.sum(C < c0) > 32
    np.testing.assert_allclose(C2.cpu().numpy(), C.cpu().numpy(), rtol=1e-5)
    assert float(K.abs().max()) <= 1.0
    cost64 = oracle_lib.rollout_cost(prob, x0, knots)
    _, wc = oracle_lib.refine(prob, x0, knots, cost64, lr=0.01, steps=5)
    np.testing.assert_allclose(C.cpu().numpy(), wc, rtol=1e-3)


def test_autograd_function(E):
    prob, x0, knots = setup(make("linear", 4, 20, 5), 8, F64)
    dp = E.DeviceProblem(prob, F64)
    K = dev(knots, F64).requires_grad_(True)
    w = torch.linspace(0.5, 2.0, 8, dtype=F64, device="cuda")
    cost = E.EmpcCost.apply(K, dev(x0, F64), dp)
    (cost * w).sum().backward()
    dJ, c = gpu_grad(E, prob, x0, knots, 8, F64)
    np.testing.assert_allclose(cost.detach().cpu().numpy(), c, rtol=1e-12)
    np.testing.assert_allclose(K.grad.cpu().numpy(), dJ * w.cpu().numpy()[None, :], rtol=1e-12)


@pytest.mark.parametrize("shift", [False, True])
def test_refined_solve_fp64_matches_oracle(oracle_lib, E, shift):
    # gradient-refined ticks (Adam on the parents after every selection):
    # FP64 keeps the parent sets identical, so whole ticks agree (also with
    # the carried parents moved one step later per tick)
    prob = W.linear_chain(3, 20, 5, seed=2)
    ga = W.GA(pop=256, n_elite=16, generations=3, sigma=0.1, seed=4, shift=shift)
    dp = E.DeviceProblem(prob, F64)
    s = E.Solver(dp, ga)
    o = oracle_lib.Solver(prob, ga, refine=True, lr=0.01, adam_steps=5)
    x = W.draw_x0(prob.n, 3)
    for tick in range(3):
        u, J = s.solve(dev(x, F64), tick, refine_steps=5, lr=0.01)
        uo, Jo, _ = o.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


@pytest.mark.parametrize("case", ["chain5", "chain16_rows"])
def test_refined_solve_fp64_chain_matches_oracle(oracle_lib, E, case):
    # the pendulum chain through the refined tick: lane-form rollout (5
    # joints) and row-form rollout (16 joints), the chain adjoint and Adam on
    # the parents; FP64 keeps every parent set identical over ticks
    d, T, p = (5, 20, 4) if case == "chain5" else (16, 25, 5)
    prob = W.pendulum_chain(d, T, p, seed=d)
    ga = W.GA(pop=128, n_elite=8, generations=2, sigma=0.1, seed=17)
    dp = E.DeviceProblem(prob, F64)
    s = E.Solver(dp, ga)
    o = oracle_lib.Solver(prob, ga, refine=True, lr=0.01, adam_steps=3)
    x = W.draw_x0(prob.n, 5) * 0.5
    for tick in range(3):
        u, J = s.solve(dev(x, F64), tick, refine_steps=3, lr=0.01)
        uo, Jo, _ = o.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


def test_refined_solve_fp32_c2_not_worse(E):
    prob, ga = W.config_c2(0)
    ga = W.dataclasses.replace(ga, generations=5)
    dp = E.DeviceProblem(prob, F32)
    x0 = dev(W.draw_x0(prob.n, 0), F32)
    plain = E.Solver(dp, ga)
    refined = E.Solver(dp, ga)
    _, Jp = plain.solve(x0, 0)
    _, Jr = refined.solve(x0, 0, refine_steps=5, lr=0.01)
    assert float(Jr.item()) <= float(Jp.item()) * (1 + 1e-4)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_refined_solve_quadratic_form_equals_adjoint_path(E, dtype):
    # a linear problem without the state box refines its parents on the
    # quadratic form 2 (P z + q); the same problem with a box of infinite
    # bounds (no penalty, but not quadratic to the library) refines through
    # the adjoint kernel: both give the same ticks (FP64 1e-9; FP32 through
    # a few ticks within the FP32 tolerance of the cost)
    prob = W.linear_chain(4, 25, 5, seed=8)
    boxed = W.dataclasses.replace(prob, x_min=np.full(prob.n, -np.inf),
                                  x_max=np.full(prob.n, np.inf), qb=np.ones(prob.n))
    ga = W.GA(pop=256, n_elite=16, generations=4 if dtype == F64 else 1, sigma=0.1, seed=6)
    sq = E.Solver(E.DeviceProblem(prob, dtype), ga)
    sa = E.Solver(E.DeviceProblem(boxed, dtype), ga)
    x = dev(W.draw_x0(prob.n, 8), dtype)
    rtol = 1e-9 if dtype == F64 else 2e-4
    for tick in range(3 if dtype == F64 else 1):
        uq, Jq = sq.solve(x, tick, refine_steps=5, lr=0.01)
        ua, Ja = sa.solve(x, tick, refine_steps=5, lr=0.01)
        np.testing.assert_allclose(float(Jq.item()), float(Ja.item()), rtol=rtol)
        if dtype == F64:
            np.testing.assert_allclose(uq.cpu().numpy(), ua.cpu().numpy(), rtol=1e-9,
                                       atol=1e-12)


def test_refined_solve_fp64_beyond_the_adjoint_limit(oracle_lib, E):
    # 36-DoF linear chain (72 states, above the adjoint's 64): its parents
    # refine on the quadratic form; FP64 ticks follow the oracle's adjoint
    prob = W.linear_chain(36, 20, 5, seed=36)
    ga = W.GA(pop=128, n_elite=8, generations=2, sigma=0.1, seed=8)
    s = E.Solver(E.DeviceProblem(prob, F64), ga)
    o = oracle_lib.Solver(prob, ga, refine=True, lr=0.01, adam_steps=5)
    x = W.draw_x0(prob.n, 36)
    for tick in range(2):
        u, J = s.solve(dev(x, F64), tick, refine_steps=5, lr=0.01)
        uo, Jo, _ = o.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)
