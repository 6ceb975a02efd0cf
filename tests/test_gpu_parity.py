"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Inputs are seeded synthetic instances from workloads/; for FP32 runs every
input is rounded to float32 first and the same rounded values go to the
oracle.  Tolerances: costs 1e-4 relative in FP32 and 1e-9 relative in FP64
(the bar the method's configuration states); integer decisions (elite sets,
parent picks, crossover bits, mutation flags) bit-exact.
"""
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
    return E


def npdt(dtype):
    return np.float32 if dtype == F32 else np.float64


def as_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rounded(prob, dtype):
    return prob.cast(npdt(dtype))


def gpu_costs(E, prob, x0, knots, ncand, dtype):
    dp = E.DeviceProblem(prob, dtype)
    K = as_dev(knots, dtype)
    cost = torch.full((ncand,), float("nan"), dtype=dtype, device="cuda")
    E.empc_rollout_cost(dp, as_dev(x0, dtype), K, ncand, knots.shape[1], cost)
    torch.cuda.synchronize()
    return cost.cpu().numpy().astype(np.float64)


def check_costs(oracle_lib, E, prob, ncand, ld, dtype, seed=0, spread=1.0):
    prob = rounded(prob, dtype)
    x0 = W.draw_x0(prob.n, seed).astype(npdt(dtype)).astype(np.float64)
    knots = W.draw_knots(prob, ncand, seed + 1, ld=ld, spread=spread)
    knots = knots.astype(npdt(dtype)).astype(np.float64)
    got = gpu_costs(E, prob, x0, knots, ncand, dtype)
    want = oracle_lib.rollout_cost(prob, x0, knots, ncand)
    np.testing.assert_allclose(got, want, rtol=RTOL[dtype], atol=0)
    return got, want


# ---------------------------------------------------------------------------
# rollout + cost


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [2, 7, 14, 21, 36])
def test_rollout_linear_chain_shapes(oracle_lib, E, dtype, d):
    # several 16-candidate tiles plus a ragged tail, ld > ncand
    prob = W.linear_chain(d, 37, 6, seed=d)
    check_costs(oracle_lib, E, prob, ncand=16 * 5 + 7, ld=100, dtype=dtype, seed=d)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [14, 21, 36])
def test_rollout_linear_forms_round_identically(oracle_lib, E, dtype, d):
    # a launch of fewer than 1024 tiles runs the M-split form, a larger one
    # the one-wavefront form: the same candidates must get the same bits
    prob = W.linear_chain(d, 23, 4, seed=d).cast(npdt(dtype))
    big = 16 * 1024 + 5
    x0 = W.draw_x0(prob.n, d)
    knots = W.draw_knots(prob, big, d + 1)
    dp = E.DeviceProblem(prob, dtype)
    K = torch.as_tensor(knots, dtype=dtype).cuda()
    X0 = torch.as_tensor(x0, dtype=dtype).cuda()
    small = torch.zeros(300, dtype=dtype, device="cuda")
    full = torch.zeros(big, dtype=dtype, device="cuda")
    E.empc_rollout_cost(dp, X0, K, 300, big, small)
    E.empc_rollout_cost(dp, X0, K, big, big, full)
    torch.cuda.synchronize()
    assert torch.equal(small, full[:300])
    # and both against the oracle on a sample
    idx = np.arange(0, big, 997)
    want = oracle_lib.rollout_cost(prob, x0.astype(npdt(dtype)).astype(np.float64),
                                   np.ascontiguousarray(knots[:, idx].astype(npdt(dtype))
                                                        .astype(np.float64)), len(idx))
    np.testing.assert_allclose(full.cpu().numpy()[idx], want, rtol=RTOL[dtype])


def test_rollout_linear_c2_shape(oracle_lib, E):
    prob, _ = W.config_c2(0)
    check_costs(oracle_lib, E, prob, ncand=131, ld=131, dtype=F32)


def test_rollout_linear_c1_shape_fp64(oracle_lib, E):
    prob, _ = W.config_c1(0)
    check_costs(oracle_lib, E, prob, ncand=300, ld=301, dtype=F64)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [2, 7, 14, 21, 36])
def test_rollout_pendulum_chain_shapes(oracle_lib, E, dtype, d):
    prob = W.pendulum_chain(d, 60, 7, seed=d)
    check_costs(oracle_lib, E, prob, ncand=300, ld=301, dtype=dtype, seed=d)


@pytest.mark.parametrize("d", [4, 20])
def test_rollout_pendulum_winding_angles(oracle_lib, E, d):
    # cumulative angles of tens of revolutions (low stiffness, wide inputs):
    # the FP32 rollout's hardware sine inside its documented domain
    prob = W.pendulum_chain(d, 30, 5, seed=d)
    prob.stiffness = np.full(d, 0.5)
    prob.u_min, prob.u_max = np.full(d, -20.0), np.full(d, 20.0)
    prob = rounded(prob, F32)
    x0 = np.r_[np.random.default_rng(d).uniform(20, 40, d), np.zeros(d)]
    x0 = x0.astype(np.float32).astype(np.float64)
    knots = W.draw_knots(prob, 80, d).astype(np.float32).astype(np.float64)
    _, traj = oracle_lib.rollout_one(prob, x0, knots, 0)
    phi = np.abs(np.cumsum(traj[:, :d], axis=1))
    assert phi.max() > 2 * np.pi * 10 and phi.max() < 1608  # within +-256 revolutions
    got = gpu_costs(E, prob, x0, knots, 80, F32)
    want = oracle_lib.rollout_cost(prob, x0, knots)
    np.testing.assert_allclose(got, want, rtol=1e-4)


def test_rollout_pendulum_c3_shape(oracle_lib, E):
    prob, _ = W.config_c3(0)
    check_costs(oracle_lib, E, prob, ncand=70, ld=70, dtype=F32)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_rollout_pendulum_c3_full_launch_sampled(oracle_lib, E, dtype):
    # the 36-link chain at its full population (16384 candidates, 1024
    # workgroups of the row form), every 257th candidate and the last one
    # against the oracle
    prob, ga = W.config_c3(0)
    prob = prob.cast(npdt(dtype))
    x0 = W.draw_x0(prob.n, 7).astype(npdt(dtype)).astype(np.float64)
    knots = W.draw_knots(prob, ga.pop, 8).astype(npdt(dtype)).astype(np.float64)
    full = gpu_costs(E, prob, x0, knots, ga.pop, dtype)
    idx = np.append(np.arange(0, ga.pop, 257), ga.pop - 1)
    want = oracle_lib.rollout_cost(prob, x0, np.ascontiguousarray(knots[:, idx]), len(idx))
    np.testing.assert_allclose(full[idx], want, rtol=RTOL[dtype], atol=0)
    assert np.all(np.isfinite(full))


def with_box(prob, half_width, weight, seed=0):
    """The problem with a state box around the goal, tight enough that many
    states leave it: x_goal -/+ half_width (per state, jittered), weights
    qb."""
    rng = np.random.default_rng(seed)
    out = W.dataclasses.replace(prob)
    g = prob.x_goal if prob.x_goal is not None else np.zeros(prob.n)
    hw = half_width * rng.uniform(0.5, 1.5, prob.n)
    out.x_min, out.x_max = g - hw, g + hw
    out.qb = weight * rng.uniform(0.5, 2.0, prob.n)
    return out


# (model maker, d, T, p, candidates): the linear one-wavefront form (4
# states), the M-split form (28 and 42 states), the chain's lane form (5
# joints) and row form (20 joints)
BOX_CASES = [(W.linear_chain, 2, 20, 5, 70), (W.linear_chain, 14, 50, 10, 300),
             (W.linear_chain, 21, 30, 6, 100), (W.pendulum_chain, 5, 40, 5, 200),
             (W.pendulum_chain, 20, 40, 5, 64)]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("case", range(len(BOX_CASES)))
def test_rollout_box_penalty_matches_oracle(oracle_lib, E, dtype, case):
    mk, d, T, p, ncand = BOX_CASES[case]
    prob = with_box(mk(d, T, p, seed=d), 0.05, 3.0, seed=d)
    got, want = check_costs(oracle_lib, E, prob, ncand=ncand, ld=ncand + 3, dtype=dtype, seed=d)
    # the bounds are tight enough that the penalty is active for every candidate
    plain = rounded(W.dataclasses.replace(prob, x_min=None, x_max=None, qb=None), dtype)
    x0 = W.draw_x0(prob.n, d).astype(npdt(dtype)).astype(np.float64)
    knots = W.draw_knots(plain, ncand, d + 1, ld=ncand + 3).astype(npdt(dtype)).astype(np.float64)
    assert np.all(want > oracle_lib.rollout_cost(plain, x0, knots, ncand))


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("mk,d", [(W.linear_chain, 2), (W.linear_chain, 14),
                                  (W.pendulum_chain, 5), (W.pendulum_chain, 20)])
def test_rollout_box_degenerate_cases(E, dtype, mk, d):
    prob = mk(d, 30, 6, seed=d)
    prob.x_goal = np.linspace(-0.1, 0.1, prob.n)
    prob = prob.cast(npdt(dtype))
    x0 = W.draw_x0(prob.n, d)
    knots = W.draw_knots(prob, 100, d + 1)
    plain = gpu_costs(E, prob, x0, knots, 100, dtype)
    # infinite bounds: the penalty is exactly zero, the cost bit for bit the plain one
    inf = W.dataclasses.replace(prob, x_min=np.full(prob.n, -np.inf), x_max=np.full(prob.n, np.inf),
                                qb=np.full(prob.n, 3.0))
    np.testing.assert_array_equal(gpu_costs(E, inf, x0, knots, 100, dtype), plain)
    # a zero-width box at the goal with weight w is w added to the diagonal
    # of Q (stage terms only); some weights zero
    w = np.where(np.arange(prob.n) % 3 == 0, 0.0, 0.7).astype(npdt(dtype))
    point = W.dataclasses.replace(prob, x_min=prob.x_goal.copy(), x_max=prob.x_goal.copy(), qb=w)
    heavier = W.dataclasses.replace(prob, q=(prob.q + w).astype(npdt(dtype)))
    np.testing.assert_allclose(gpu_costs(E, point, x0, knots, 100, dtype),
                               gpu_costs(E, heavier, x0, knots, 100, dtype), rtol=RTOL[dtype] / 10)


def test_box_penalty_needs_bounds(E):
    prob = W.linear_chain(2, 10, 3, seed=0)
    prob.qb = np.ones(prob.n)  # no x_min / x_max
    cost = torch.empty(4, device="cuda")
    with pytest.raises(E.EmpcError):
        E.empc_rollout_cost(E.DeviceProblem(prob, F32), torch.zeros(prob.n, device="cuda"),
                            torch.zeros((prob.p * prob.m, 4), device="cuda"), 4, 4, cost)


def test_solve_fp64_box_matches_oracle(oracle_lib, E):
    prob = with_box(W.linear_chain(3, 20, 5, seed=2), 0.1, 5.0, seed=3)
    ga = W.GA(pop=200, n_elite=10, generations=3, sigma=0.1, seed=8)
    solver = E.Solver(E.DeviceProblem(prob, F64), ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 5)
    for tick in range(3):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


@pytest.mark.parametrize("model", ["linear", "chain"])
@pytest.mark.parametrize("T,p", [(1, 1), (9, 1), (12, 12), (50, 2), (2, 2)])
def test_rollout_knot_edge_cases(oracle_lib, E, model, T, p):
    mk = W.linear_chain if model == "linear" else W.pendulum_chain
    prob = mk(3, T, p, seed=1)
    prob.qf = np.linspace(0.1, 1.0, prob.n)
    prob.x_goal = np.linspace(-0.2, 0.3, prob.n)
    prob.u_goal = np.linspace(0.1, -0.1, prob.m)
    check_costs(oracle_lib, E, prob, ncand=33, ld=40, dtype=F64, seed=T)


def test_rollout_out_of_bounds_knots_used_as_given(oracle_lib, E):
    prob = W.linear_chain(4, 20, 5, seed=3)
    check_costs(oracle_lib, E, prob, ncand=50, ld=50, dtype=F64, spread=3.0)


def test_rollout_zero_and_single_candidate(oracle_lib, E):
    prob = W.linear_chain(2, 10, 3, seed=0)
    dp = E.DeviceProblem(prob, F64)
    cost = torch.full((4,), -7.0, dtype=F64, device="cuda")
    x0 = as_dev(np.zeros(prob.n), F64)
    K = as_dev(np.zeros((prob.p * prob.m, 4)), F64)
    E.empc_rollout_cost(dp, x0, K, 0, 4, cost)
    torch.cuda.synchronize()
    assert torch.all(cost == -7.0)  # ncand = 0 writes nothing
    check_costs(oracle_lib, E, prob, ncand=1, ld=1, dtype=F64)


def test_rollout_full_c2_population_sampled(oracle_lib, E):
    # the benchmark's launch: 4096 candidates in one call; sampled check
    prob, ga = W.config_c2(0)
    prob = rounded(prob, F32)
    x0 = W.draw_x0(prob.n, 0).astype(np.float32).astype(np.float64)
    knots = W.draw_knots(prob, ga.pop, 2).astype(np.float32).astype(np.float64)
    got = gpu_costs(E, prob, x0, knots, ga.pop, F32)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(ga.pop, 40, replace=False), [0, ga.pop - 1]])
    want = oracle_lib.rollout_cost(prob, x0, np.ascontiguousarray(knots[:, idx]))
    np.testing.assert_allclose(got[idx], want, rtol=1e-4)
    assert np.all(np.isfinite(got)) and np.all(got > 0)


def test_rollout_equilibrium_is_zero(E):
    for mk in (W.linear_chain, W.pendulum_chain):
        prob = mk(5, 30, 5, seed=0)
        got = gpu_costs(E, prob, np.zeros(prob.n), np.zeros((prob.p * prob.m, 20)), 20, F32)
        assert np.all(got == 0.0)


def test_rollout_deterministic(E):
    prob, ga = W.config_c2(0)
    knots = W.draw_knots(prob, 1000, 4)
    a = gpu_costs(E, prob, W.draw_x0(prob.n, 0), knots, 1000, F32)
    b = gpu_costs(E, prob, W.draw_x0(prob.n, 0), knots, 1000, F32)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# selection and next population


def gpu_generation(E, prob, ga, knots_in, cost_in, tick, gen, dtype):
    dp = E.DeviceProblem(prob, dtype)
    g = E.make_ga(ga)
    pm = prob.p * prob.m
    out = torch.full((pm, ga.pop), float("nan"), dtype=dtype, device="cuda")
    eidx = torch.full((ga.n_elite,), -1, dtype=torch.int64, device="cuda")
    best = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    if knots_in is None:
        E.empc_generation(dp, g, None, 0, None, out, ga.pop, None, None, tick, gen)
    else:
        E.empc_generation(dp, g, as_dev(knots_in, dtype), knots_in.shape[1],
                          as_dev(cost_in, dtype), out, ga.pop, eidx, best, tick, gen)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), eidx.cpu().numpy(), int(best.item())


@pytest.mark.parametrize("dtype", [F32, F64])
def test_cold_start_population(oracle_lib, E, dtype):
    prob, ga = W.config_c2(0)
    prob = rounded(prob, dtype)
    ga = W.dataclasses.replace(ga, pop=1000)
    got, _, _ = gpu_generation(E, prob, ga, None, None, tick=3, gen=1, dtype=dtype)
    want = oracle_lib.next_population(prob, ga, None, cold=True, tick=3, gen=1)
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-7 if dtype == F32 else 1e-15)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("elitism", [True, False])
def test_warm_generation_matches_oracle(oracle_lib, E, dtype, elitism):
    prob, ga = W.config_c2(0)
    prob = rounded(prob, dtype)
    ga = W.dataclasses.replace(ga, pop=777, n_elite=40, elitism=elitism, seed=12345678901)
    rng = np.random.default_rng(1)
    knots = W.draw_knots(prob, ga.pop, 5).astype(npdt(dtype)).astype(np.float64)
    cost = rng.uniform(0, 10, ga.pop).astype(npdt(dtype)).astype(np.float64)
    got, eidx, best = gpu_generation(E, prob, ga, knots, cost, tick=7, gen=2, dtype=dtype)
    want_idx, want_best = oracle_lib.select(cost, ga.n_elite)
    np.testing.assert_array_equal(eidx, want_idx)
    assert best == want_best
    elite_rows = knots[:, want_idx].T.copy()
    want = oracle_lib.next_population(prob, ga, elite_rows, cold=False, tick=7, gen=2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-6 if dtype == F32 else 1e-14)
    # integer decisions are exact: un-mutated, unclamped children equal a parent
    assert np.mean(got == want) > 0.4


@pytest.mark.parametrize("dtype", [F32, F64])
def test_selection_ties_nan_inf(oracle_lib, E, dtype):
    prob = W.linear_chain(2, 10, 3, seed=0)
    rng = np.random.default_rng(7)
    for pop, k in [(1, 1), (5, 5), (300, 17), (4096, 64), (5000, 256), (1025, 1)]:
        ga = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=1)
        cost = np.round(rng.normal(0, 1, pop), 1)
        cost[rng.random(pop) < 0.05] = np.nan
        cost[rng.random(pop) < 0.03] = np.inf
        cost[rng.random(pop) < 0.03] = -np.inf
        cost[rng.random(pop) < 0.02] = 0.0
        cost[rng.random(pop) < 0.02] = -0.0
        knots = W.draw_knots(prob, pop, 1)
        _, eidx, best = gpu_generation(E, prob, ga, knots, cost, 0, 0, dtype)
        want_idx, want_best = oracle_lib.select(cost, k)
        np.testing.assert_array_equal(eidx, want_idx)
        assert best == want_best


@pytest.mark.parametrize("pop", [600, 6000, 12000])
@pytest.mark.parametrize("cold", [True, False])
def test_population_grouping_matches_oracle(oracle_lib, E, pop, cold):
    # 360 parameters: a single launch takes 16 parameters per workgroup at
    # pop 600, 32 at 6000 and 64 at 12000; every grouping must give the
    # oracle's children (sampled slots, parents and elitism included)
    prob = W.pendulum_chain(36, 100, 10, seed=4).cast(np.float32)
    ga = W.GA(pop=pop, n_elite=64, generations=1, sigma=0.1, seed=0xC0FFEE)
    rng = np.random.default_rng(pop)
    knots = W.draw_knots(prob, pop, 9).astype(np.float32).astype(np.float64)
    cost = rng.uniform(0, 10, pop).astype(np.float32).astype(np.float64)
    if cold:
        got, _, _ = gpu_generation(E, prob, ga, None, None, tick=0, gen=0, dtype=F32)
        want = oracle_lib.next_population(prob, ga, None, cold=True, tick=0, gen=0)
    else:
        got, eidx, _ = gpu_generation(E, prob, ga, knots, cost, tick=4, gen=2, dtype=F32)
        want_idx, _ = oracle_lib.select(cost, ga.n_elite)
        np.testing.assert_array_equal(eidx, want_idx)
        want = oracle_lib.next_population(prob, ga, knots[:, want_idx].T.copy(), cold=False,
                                          tick=4, gen=2)
    slots = np.r_[np.arange(70), rng.choice(pop, 300, replace=False), pop - 1]
    np.testing.assert_allclose(got[:, slots], want[:, slots], rtol=0, atol=1e-6)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_selection_nan_after_inf(oracle_lib, E, dtype):
    # the k boundary between a NaN and a later +inf: NaN ranks last
    prob = W.linear_chain(2, 10, 3, seed=0)
    cases = [([np.nan, np.inf, 1.0], 2, [1, 2], 2), ([np.nan, np.inf], 1, [1], 1),
             ([np.nan, np.nan, -np.inf], 2, [0, 2], 2), ([np.inf, np.nan, np.inf], 2, [0, 2], 0)]
    for cost, k, want_idx, want_best in cases:
        cost = np.array(cost)
        ga = W.GA(pop=len(cost), n_elite=k, generations=1, sigma=0.1, seed=1)
        knots = W.draw_knots(prob, len(cost), 1)
        _, eidx, best = gpu_generation(E, prob, ga, knots, cost, 0, 0, dtype)
        assert list(eidx) == want_idx and best == want_best, (cost, k)
        oidx, obest = oracle_lib.select(cost, k)
        assert list(oidx) == want_idx and obest == want_best


@pytest.mark.parametrize("dtype", [F32, F64])
def test_selection_small_populations(oracle_lib, E, dtype):
    # populations of at most 256 run the one-wavefront bitonic sort (pads
    # past the population, partners across lanes and within a lane): heavy
    # ties, NaN / inf / signed zeros, every k from 1 to pop on a few sizes,
    # exact equality with the oracle
    prob = W.linear_chain(2, 10, 3, seed=0)
    rng = np.random.default_rng(11)
    cases = [(pop, k) for pop in (2, 16, 63, 64, 65, 200, 256) for k in sorted({1, 2, pop // 3 or 1, pop})]
    for pop, k in cases:
        ga = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=1)
        cost = np.round(rng.normal(0, 1, pop), 0)  # many exact ties
        cost[rng.random(pop) < 0.05] = np.nan
        cost[rng.random(pop) < 0.05] = np.inf
        cost[rng.random(pop) < 0.05] = -0.0
        knots = W.draw_knots(prob, pop, 1)
        _, eidx, best = gpu_generation(E, prob, ga, knots, cost, 0, 0, dtype)
        want_idx, want_best = oracle_lib.select(cost, k)
        np.testing.assert_array_equal(eidx, want_idx, err_msg="pop %d k %d" % (pop, k))
        assert best == want_best, (pop, k)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_selection_degenerate_and_large(oracle_lib, E, dtype):
    # all keys equal; ties at the threshold spread over every quarter of the
    # index range; all NaN; a population above the register-cached sizes
    prob = W.linear_chain(2, 10, 3, seed=0)
    rng = np.random.default_rng(3)
    cases = [
        (np.full(4096, 2.5), 64),
        (np.r_[np.zeros(10), np.ones(4086)], 64),
        (np.where(np.arange(4096) % 97 == 0, 0.5, 1.0), 200),
        (np.full(300, np.nan), 17),
        (np.round(rng.normal(0, 1, 20000), 2), 100),
        (rng.permutation(np.arange(70001, dtype=np.float64)), 256),
    ]
    for cost, k in cases:
        pop = len(cost)
        cost = cost.astype(npdt(dtype)).astype(np.float64)
        ga = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=1)
        knots = W.draw_knots(prob, pop, 1)
        _, eidx, best = gpu_generation(E, prob, ga, knots, cost, 0, 0, dtype)
        want_idx, want_best = oracle_lib.select(cost, k)
        np.testing.assert_array_equal(eidx, want_idx)
        assert best == want_best


@pytest.mark.parametrize("dtype", [F32, F64])
def test_selection_random_bands(oracle_lib, E, dtype):
    # costs of a real population sit in a narrow band, so the radix passes
    # start below the bytes every key shares: random pops, k and bands
    prob = W.linear_chain(2, 10, 3, seed=0)
    rng = np.random.default_rng(11)
    for trial in range(40):
        pop = int(rng.integers(1, 5000)) if trial % 5 else 4096
        k = int(rng.integers(1, min(pop, 256) + 1))
        lo = float(rng.choice([0.5, 40.0, 403.0, 1e4]))
        width = lo * float(rng.choice([1e-6, 1e-3, 0.1, 0.25, 3.0]))
        cost = (lo + width * rng.random(pop)).astype(npdt(dtype)).astype(np.float64)
        ga = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=1)
        knots = W.draw_knots(prob, pop, 1)
        _, eidx, best = gpu_generation(E, prob, ga, knots, cost, 0, 0, dtype)
        want_idx, want_best = oracle_lib.select(cost, k)
        np.testing.assert_array_equal(eidx, want_idx, err_msg="trial %d" % trial)
        assert best == want_best, trial


# ---------------------------------------------------------------------------
# FP32 selection on real rollout costs against the FP64 oracle's selection


def check_fp32_elites(oracle_lib, E, prob, knots, x0, k, rtol=1e-4):
    """The GPU selects from its own FP32 costs; the oracle from FP64 costs of
    the same (rounded) knots.  The two elite sets may differ only by swaps
    whose oracle costs lie within rtol of the k-th smallest oracle cost (a
    tie group at the boundary); every other index must agree."""
    pop = knots.shape[1]
    dp = E.DeviceProblem(prob, F32)
    K = as_dev(knots, F32)
    cost = torch.empty(pop, dtype=F32, device="cuda")
    E.empc_rollout_cost(dp, as_dev(x0, F32), K, pop, pop, cost)
    ga = W.GA(pop=pop, n_elite=k, generations=1, sigma=0.1, seed=1)
    g = E.make_ga(ga)
    out = torch.empty((prob.p * prob.m, pop), dtype=F32, device="cuda")
    eidx = torch.empty(k, dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    E.empc_generation(dp, g, K, pop, cost, out, pop, eidx, best, 0, 1)
    torch.cuda.synchronize()
    got = set(eidx.cpu().numpy().tolist())
    J = oracle_lib.rollout_cost(prob, x0, knots)
    np.testing.assert_allclose(cost.cpu().numpy(), J, rtol=rtol)
    want_idx, want_best = oracle_lib.select(J, k)
    want = set(want_idx.tolist())
    thr = np.sort(J)[k - 1]
    tol = rtol * abs(thr)
    for i in got - want:
        assert J[i] <= thr + tol, (i, J[i], thr)
    for i in want - got:
        assert J[i] >= thr - tol, (i, J[i], thr)
    b = int(best.item())
    assert J[b] <= J[want_best] * (1 + rtol)
    return len(got ^ want) // 2


def warm_population(oracle_lib, prob, pop, seed):
    """A population bred from 64 random parents (crossover and mutation with
    sigma 0.1): costs in the narrow band of a real generation."""
    rng = np.random.default_rng(seed)
    parents = rng.uniform(-1, 1, (64, prob.p * prob.m))
    ga = W.GA(pop=pop, n_elite=64, generations=1, sigma=0.1, seed=seed)
    return oracle_lib.next_population(prob, ga, parents, cold=False, tick=1, gen=0)


@pytest.mark.parametrize("warm", [False, True])
def test_fp32_elites_c2(oracle_lib, E, warm):
    prob, ga = W.config_c2(0)
    prob = rounded(prob, F32)
    x0 = W.draw_x0(prob.n, 0).astype(np.float32).astype(np.float64)
    knots = (warm_population(oracle_lib, prob, ga.pop, 3) if warm
             else W.draw_knots(prob, ga.pop, 3))
    knots = knots.astype(np.float32).astype(np.float64)
    check_fp32_elites(oracle_lib, E, prob, knots, x0, ga.n_elite)


@pytest.mark.parametrize("warm", [False, True])
def test_fp32_elites_c3(oracle_lib, E, warm):
    prob, ga = W.config_c3(0)
    prob = rounded(prob, F32)
    x0 = W.draw_x0(prob.n, 0).astype(np.float32).astype(np.float64)
    pop = 4096  # a quarter of the configured population keeps the oracle fast
    knots = (warm_population(oracle_lib, prob, pop, 5) if warm
             else W.draw_knots(prob, pop, 5))
    knots = knots.astype(np.float32).astype(np.float64)
    check_fp32_elites(oracle_lib, E, prob, knots, x0, ga.n_elite)


# ---------------------------------------------------------------------------
# solve


# warm-start variants: carried parents moved one step later per tick, and the
# mutation noise growing with the distance to the goal (0.02 at the goal, the
# configured sigma from distance 1 on)
VARIANTS = {"plain": {}, "shift+noise_schedule": dict(shift=True, sigma_min=0.02, sigma_dist=1.0)}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_solve_fp64_matches_oracle_over_ticks(oracle_lib, E, variant):
    # FP64 keeps every elite set identical to the oracle's, so whole
    # multi-generation, multi-tick trajectories agree
    prob, ga = W.config_c1(0)
    ga = W.dataclasses.replace(ga, **VARIANTS[variant])
    dp = E.DeviceProblem(prob, F64)
    solver = E.Solver(dp, ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    noise = W.process_noise(prob.n, 5, 0)
    for tick in range(5):
        u, J = solver.solve(as_dev(x, F64), tick)
        u = u.cpu().numpy()
        J = float(J.item())
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u, uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(J, Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo, noise[tick])


EDGE_SOLVES = {
    # name: (model maker, d, T, p, GA fields)
    "all_parents": (W.linear_chain, 2, 10, 3, dict(pop=8, n_elite=8, generations=2)),
    "one_parent": (W.linear_chain, 3, 12, 4, dict(pop=50, n_elite=1, generations=3)),
    "ragged_population_chain": (W.pendulum_chain, 5, 15, 5, dict(pop=70, n_elite=5, generations=2)),
    "knot_per_step": (W.linear_chain, 2, 6, 6, dict(pop=40, n_elite=4, generations=2)),
    "single_knot_chain": (W.pendulum_chain, 3, 9, 1, dict(pop=33, n_elite=3, generations=2)),
    "no_elitism": (W.linear_chain, 4, 15, 4, dict(pop=100, n_elite=10, generations=3, elitism=False)),
    "one_step_horizon": (W.linear_chain, 2, 1, 1, dict(pop=20, n_elite=2, generations=2)),
}


@pytest.mark.parametrize("case", sorted(EDGE_SOLVES))
def test_solve_fp64_edge_shapes(oracle_lib, E, case):
    # degenerate and ragged shapes of the method: every slot a parent, a
    # single parent, a population that is not a multiple of any tile, one
    # knot per step, a single knot, no elitism, a one-step horizon; FP64
    # keeps every selection identical, so whole ticks follow the oracle
    mk, d, T, p, g = EDGE_SOLVES[case]
    prob = mk(d, T, p, seed=d + T)
    ga = W.GA(sigma=0.1, seed=31, **g)
    solver = E.Solver(E.DeviceProblem(prob, F64), ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 2)
    for tick in range(2):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9, atol=1e-300)
        x = oracle_lib.step(prob, x, uo)


@pytest.mark.parametrize("d,T,p", [(9, 30, 6), (20, 25, 5)])
def test_solve_fp64_split_rollout_matches_oracle(oracle_lib, E, d, T, p):
    # linear chains of more than 16 states at a population of fewer than
    # 1024 tiles run the M-split rollout (one wavefront per 16-state tile,
    # rows exchanged through LDS every step): whole FP64 ticks must still
    # follow the oracle (ragged last tile: pop is not a multiple of 16)
    prob = W.linear_chain(d, T, p, seed=d)
    ga = W.GA(pop=600, n_elite=24, generations=3, sigma=0.1, seed=11)
    solver = E.Solver(E.DeviceProblem(prob, F64), ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 1)
    for tick in range(3):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


def test_solve_fp32_one_generation_matches_oracle(oracle_lib, E):
    prob, ga = W.config_c2(0)
    prob = rounded(prob, F32)
    ga = W.dataclasses.replace(ga, generations=1)
    x0 = W.draw_x0(prob.n, 0).astype(np.float32).astype(np.float64)
    solver = E.Solver(E.DeviceProblem(prob, F32), ga)
    u, J = solver.solve(as_dev(x0, F32), 0)
    uo, Jo, _ = oracle_lib.Solver(prob, ga).solve(x0, 0)
    np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-4)
    np.testing.assert_allclose(u.cpu().numpy(), uo, atol=1e-6)


def test_solve_fp32_c2_tick_quality(oracle_lib, E):
    # full C2 tick: the best cost is the cost of the returned knots, it is
    # non-increasing over generations, and it is close to the FP64 oracle's
    prob, ga = W.config_c2(0)
    prob = rounded(prob, F32)
    x0 = W.draw_x0(prob.n, 0).astype(np.float32).astype(np.float64)
    dp = E.DeviceProblem(prob, F32)
    bests = []
    for G in (1, 5, 20):
        s = E.Solver(dp, W.dataclasses.replace(ga, generations=G))
        _, J = s.solve(as_dev(x0, F32), 0)
        bests.append(float(J.item()))
    assert bests[0] >= bests[1] >= bests[2]
    _, Jo, gb = oracle_lib.Solver(prob, W.dataclasses.replace(ga, generations=5)).solve(x0, 0)
    np.testing.assert_allclose(bests[1], Jo, rtol=1e-3)


def test_solve_workspace_errors(E):
    prob, ga = W.config_c1(0)
    dp = E.DeviceProblem(prob, F64)
    g = E.make_ga(ga)
    ws = torch.zeros(16, dtype=torch.uint8, device="cuda")
    u = torch.zeros(prob.m, dtype=F64, device="cuda")
    b = torch.zeros(1, dtype=F64, device="cuda")
    with pytest.raises(E.EmpcError) as ei:
        E.empc_solve(dp, g, ws, as_dev(np.zeros(prob.n), F64), 0, u, b)
    assert ei.value.status == 4


# ---------------------------------------------------------------------------
# plant step


@pytest.mark.parametrize("mk", [W.linear_chain, W.pendulum_chain])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_plant_step(oracle_lib, E, mk, dtype):
    prob = rounded(mk(6, 10, 3, seed=2), dtype)
    dp = E.DeviceProblem(prob, dtype)
    x = W.draw_x0(prob.n, 1).astype(npdt(dtype)).astype(np.float64)
    u = np.linspace(-0.5, 0.7, prob.m).astype(npdt(dtype)).astype(np.float64)
    nz = W.process_noise(prob.n, 1, 0)[0].astype(npdt(dtype)).astype(np.float64)
    out = torch.zeros(prob.n, dtype=dtype, device="cuda")
    E.empc_plant_step(dp, as_dev(x, dtype), as_dev(u, dtype), as_dev(nz, dtype), out)
    want = oracle_lib.step(prob, x, u, nz)
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-5 if dtype == F32 else 1e-12,
                               atol=1e-6 if dtype == F32 else 1e-14)
