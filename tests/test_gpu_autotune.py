"""The single-problem autotuner and its tuning table (through the C ABI):
the matrix-core launch shapes and the population's parameter groups keep
every bit of the fixed rules; the vector-ALU linear rollout (one lane per
candidate, n, m <= 16) follows the FP64 oracle at 1e-9 and the FP32 one at
1e-4 over the shapes and optional terms of the method; a tuned solve stays
on the oracle's trajectory."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
RTOL = {F32: 1e-4, F64: 1e-9}


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    E.lib()
    yield E
    E.empc_autotune_reset()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def ticks(E, prob, ga, dtype, n_ticks, x_seed=3):
    s = E.Solver(E.DeviceProblem(prob, dtype), ga)
    out = []
    for t in range(n_ticks):
        u, J = s.solve(dev(W.draw_x0(prob.n, x_seed + t), dtype), t)
        out.append((u.clone(), J.clone()))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("which", ["c2_linear", "chain"])
def test_matrix_core_shapes_keep_the_bits(E, which):
    if which == "c2_linear":
        prob, ga = W.config_c2(0)
        ga = W.dataclasses.replace(ga, generations=3)
    else:
        prob = W.pendulum_chain(20, 30, 5, 2)
        ga = W.GA(pop=3000, n_elite=32, generations=3, sigma=0.1, seed=4)
    prob = prob.cast(np.float32)
    E.empc_autotune_reset()
    ref = ticks(E, prob, ga, F32, 2)
    info = E.empc_autotune(E.DeviceProblem(prob, F32), E.make_ga(ga), reps=3, allow_valu=False)
    assert info["rollout_form"] != E.binding.RF_VALU256 and info["rollout_form"] != E.binding.RF_VALU64
    assert info["pop_groups"] in (1, 2, 4)
    assert 0 < info["rollout_us"] <= info["rule_rollout_us"]
    got = ticks(E, prob, ga, F32, 2)
    for (u, J), (ur, Jr) in zip(got, ref):
        assert torch.equal(u, ur) and torch.equal(J, Jr)
    # every shape by hand, too
    forms = ([E.binding.RF_ONE1, E.binding.RF_ONE2, E.binding.RF_ONE4, E.binding.RF_SPLIT]
             if which == "c2_linear" else [E.binding.RF_CH64, E.binding.RF_CH128])
    for f, g in zip(forms, (1, 2, 4, 1)):
        E.empc_autotune_set(E.DeviceProblem(prob, F32), E.make_ga(ga), f, g)
        got = ticks(E, prob, ga, F32, 1)
        assert torch.equal(got[0][0], ref[0][0]) and torch.equal(got[0][1], ref[0][1]), f
    E.empc_autotune_reset()


VALU_SHAPES = [(2, 20, 5), (4, 33, 7), (7, 50, 10), (8, 25, 25), (3, 12, 1)]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d,T,p", VALU_SHAPES)
@pytest.mark.parametrize("form", ["VALU256", "VALU64"])
def test_valu_rollout_matches_oracle(oracle_lib, E, dtype, d, T, p, form):
    # linear chains of d masses (n = 2d <= 16), several workgroups and a
    # ragged last one, goal and input-goal offsets, a terminal weight
    prob = W.linear_chain(d, T, p, seed=d + T)
    rng = np.random.default_rng(d)
    prob.x_goal = rng.normal(0, 0.3, prob.n)
    prob.u_goal = rng.normal(0, 0.1, prob.m)
    prob.qf = rng.uniform(0, 2, prob.n)
    prob = prob.cast(np.float32 if dtype == F32 else np.float64)
    ncand = 517
    x0 = W.draw_x0(prob.n, 5).astype(np.float32 if dtype == F32 else np.float64).astype(np.float64)
    knots = W.draw_knots(prob, ncand, 6).astype(np.float32 if dtype == F32 else np.float64)
    knots = knots.astype(np.float64)
    dp = E.DeviceProblem(prob, dtype)
    ga = W.GA(pop=ncand, n_elite=8, generations=1, sigma=0.1, seed=0)
    E.empc_autotune_set(dp, E.make_ga(ga), getattr(E.binding, "RF_" + form), 0)
    cost = torch.full((ncand,), float("nan"), dtype=dtype, device="cuda")
    E.empc_rollout_cost(dp, dev(x0, dtype), dev(knots, dtype), ncand, ncand, cost)
    torch.cuda.synchronize()
    want = oracle_lib.rollout_cost(prob, x0, knots, ncand)
    np.testing.assert_allclose(cost.cpu().numpy().astype(np.float64), want, rtol=RTOL[dtype])
    E.empc_autotune_reset()


def test_valu_rollout_box_penalty(oracle_lib, E):
    prob = W.linear_chain(5, 30, 6, seed=1)
    prob = W.dataclasses.replace(prob, x_min=np.full(prob.n, -0.2), x_max=np.full(prob.n, 0.3),
                                 qb=np.full(prob.n, 4.0))
    ncand = 300
    x0 = W.draw_x0(prob.n, 2)
    knots = W.draw_knots(prob, ncand, 3)
    dp = E.DeviceProblem(prob, F64)
    E.empc_autotune_set(dp, E.make_ga(W.GA(pop=ncand, n_elite=4, generations=1, sigma=0.1,
                                           seed=0)), E.binding.RF_VALU256, 0)
    cost = torch.empty(ncand, dtype=F64, device="cuda")
    E.empc_rollout_cost(dp, dev(x0, F64), dev(knots, F64), ncand, ncand, cost)
    want = oracle_lib.rollout_cost(prob, x0, knots, ncand)
    np.testing.assert_allclose(cost.cpu().numpy(), want, rtol=1e-9)
    E.empc_autotune_reset()


def test_tuned_fp64_solve_follows_the_oracle(oracle_lib, E):
    # C1 (FP64, 2-DoF): whatever the tuner picks (the vector-ALU form
    # included), the solve keeps the oracle's elite sets over ticks
    prob, ga = W.config_c1(0)
    dp = E.DeviceProblem(prob, F64)
    info = E.empc_autotune(dp, E.make_ga(ga), reps=5, allow_valu=True)
    s = E.Solver(dp, ga)
    o = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    for t in range(3):
        u, J = s.solve(dev(x, F64), t)
        uo, Jo, _ = o.solve(x, t)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)
    assert info["rollout_us"] > 0
    E.empc_autotune_reset()


def test_autotune_set_rejects_bad_choices(E):
    prob, ga = W.config_c2(0)
    dp = E.DeviceProblem(prob.cast(np.float32), F32)
    g = E.make_ga(ga)
    with pytest.raises(E.EmpcError) as ei:
        E.empc_autotune_set(dp, g, E.binding.RF_VALU256, 0)  # n = 28
    assert ei.value.status == E.binding.EMPC_EUNSUPPORTED
    with pytest.raises(E.EmpcError):
        E.empc_autotune_set(dp, g, E.binding.RF_CH64, 0)  # a chain form
    with pytest.raises(E.EmpcError):
        E.empc_autotune_set(dp, g, E.binding.RF_ONE1, 3)
    with pytest.raises(E.EmpcError):
        E.empc_autotune(dp, g, reps=0)
