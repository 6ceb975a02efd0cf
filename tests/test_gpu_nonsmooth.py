"""GPU parity of the non-smooth terms and full weights (Sec. V-A: branches
in the simulation, costs that need not be continuous; eq. 3 with full Q,
R) against the FP64 oracle, through the C ABI.

FP64 costs agree to 1e-9 relative: the two sides take the same branch
decisions (a state within 1e-9 of a bound is vanishingly rare with these
seeds).  In FP32 a branch may go the other way for a state within rounding
of a bound or limit, so the FP32 checks use bounds every state violates
(the step charge then counts every step exactly) or require most
candidates to agree (impacts).
"""
import numpy as np
import pytest
import torch

import workloads as W
from test_gpu_parity import F32, F64, RTOL, as_dev, gpu_costs, npdt, rounded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    E.lib()
    return E


def spd(n, rng, cond=20.0):
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Qm * np.geomspace(1.0, 1.0 / cond, n)) @ Qm.T


def full(prob, seed, which="QRQf"):
    rng = np.random.default_rng(seed)
    out = W.dataclasses.replace(prob)
    if "Q" in which.replace("Qf", ""):
        out.Q = spd(prob.n, rng)
    if "R" in which:
        out.R = 0.05 * spd(prob.m, rng)
    if "Qf" in which:
        out.Qf = 2.0 * spd(prob.n, rng)
    out.x_goal = 0.1 * rng.standard_normal(prob.n)
    return out


def boxed(prob, seed, half_width, qb=1.0, sb=0.5):
    rng = np.random.default_rng(seed)
    out = W.dataclasses.replace(prob)
    g = prob.x_goal if prob.x_goal is not None else np.zeros(prob.n)
    hw = half_width * rng.uniform(0.5, 1.5, prob.n)
    out.x_min, out.x_max = g - hw, g + hw
    out.qb = qb * rng.uniform(0.5, 2.0, prob.n)
    out.sb = sb * rng.uniform(0.5, 2.0, prob.n)
    return out


def compare(oracle_lib, E, prob, ncand, ld, dtype, seed, rtol=None):
    prob = rounded(prob, dtype)
    x0 = W.draw_x0(prob.n, seed).astype(npdt(dtype)).astype(np.float64)
    knots = W.draw_knots(prob, ncand, seed + 1, ld=ld).astype(npdt(dtype)).astype(np.float64)
    got = gpu_costs(E, prob, x0, knots, ncand, dtype)
    want = oracle_lib.rollout_cost(prob, x0, knots, ncand)
    if rtol is not None:
        np.testing.assert_allclose(got, want, rtol=rtol, atol=0)
    return got, want


# ---------------------------------------------------------------------------
# full Q, R, Qf (vector-ALU rollout)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [1, 2, 4, 7, 8])
@pytest.mark.parametrize("which", ["QRQf", "Q", "R", "Qf"])
def test_full_weights_rollout(oracle_lib, E, dtype, d, which):
    prob = full(W.linear_chain(d, 33, 6, seed=d), d, which)
    compare(oracle_lib, E, prob, ncand=16 * 20 + 9, ld=400, dtype=dtype, seed=d,
            rtol=RTOL[dtype])


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [10, 14, 21, 32])
def test_full_weights_row_form_large(oracle_lib, E, dtype, d):
    # 16 lanes per candidate: 20 to 64 states (1 to 4 rows per lane), 10 to
    # 32 inputs (1 or 2 per lane), ragged candidate count, ld > ncand
    prob = full(W.linear_chain(d, 30, 5, seed=d), d)
    compare(oracle_lib, E, prob, ncand=16 * 6 + 5, ld=120, dtype=dtype, seed=d,
            rtol=RTOL[dtype])


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("d", [3, 14])
def test_full_weights_with_box_and_step_charge(oracle_lib, E, dtype, d):
    prob = boxed(full(W.linear_chain(d, 40, 5, seed=9), 9), 9, 0.15)
    if dtype == F32:  # every state outside: the charge counts every step
        prob.x_min, prob.x_max = prob.x_min + 50.0, prob.x_max + 50.0
    compare(oracle_lib, E, prob, ncand=300, ld=300, dtype=dtype, seed=9, rtol=RTOL[dtype])


def test_full_weights_both_launch_shapes_and_the_tuner(oracle_lib, E):
    prob = full(W.linear_chain(5, 30, 5, seed=3), 3)
    x0 = W.draw_x0(prob.n, 3)
    knots = W.draw_knots(prob, 1000, 4)
    dp = E.DeviceProblem(prob, F64)
    ga = E.make_ga(W.GA(pop=1000, n_elite=10, generations=1, sigma=0.1, seed=1))
    want = oracle_lib.rollout_cost(prob, x0, knots)
    outs = []
    try:
        for form in (E.RF_VALU256, E.RF_VALU64):
            E.empc_autotune_set(dp, ga, form, 0)
            cost = torch.empty(1000, dtype=F64, device="cuda")
            E.empc_rollout_cost(dp, as_dev(x0, F64), as_dev(knots, F64), 1000, 1000, cost)
            outs.append(cost.cpu().numpy())
        info = E.empc_autotune(dp, ga, reps=2, allow_valu=True)
        assert info["rollout_form"] in (E.RF_RULE, E.RF_VALU256, E.RF_VALU64)
        with pytest.raises(E.EmpcError):
            E.empc_autotune_set(dp, ga, E.RF_SPLIT, 0)
    finally:
        E.empc_autotune_reset()
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_allclose(outs[0], want, rtol=1e-9)
    # the rule (16-lane row form) against the same oracle costs
    rows = torch.empty(1000, dtype=F64, device="cuda")
    E.empc_rollout_cost(dp, as_dev(x0, F64), as_dev(knots, F64), 1000, 1000, rows)
    np.testing.assert_allclose(rows.cpu().numpy(), want, rtol=1e-9)


def test_full_weights_solve_fp64_over_ticks(oracle_lib, E):
    prob = full(W.linear_chain(2, 20, 5, seed=0), 0)
    ga = W.GA(pop=256, n_elite=16, generations=6, sigma=0.1, seed=5)
    solver = E.Solver(E.DeviceProblem(prob, F64), ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 0)
    for tick in range(4):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


def test_full_weights_limits(E):
    rng = np.random.default_rng(0)
    big = W.linear_chain(33, 20, 4, seed=1)  # n = 66 > 64
    big.Q = spd(big.n, rng)
    dp = E.DeviceProblem(big, F32)
    x0 = torch.zeros(big.n, device="cuda")
    K = torch.zeros(big.p * big.m, 16, device="cuda")
    cost = torch.empty(16, device="cuda")
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(dp, x0, K, 16, 16, cost)
    assert ex.value.status == E.EMPC_EUNSUPPORTED
    prob = full(W.linear_chain(2, 20, 4, seed=1), 1)
    dp = E.DeviceProblem(prob, F32)
    x0 = torch.zeros(prob.n, device="cuda")
    K = torch.zeros(prob.p * prob.m, 16, device="cuda")
    with pytest.raises(E.EmpcError) as ex:
        E.empc_grad(dp, x0, K, 16, 16, torch.empty_like(K), torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EUNSUPPORTED
    with pytest.raises(E.EmpcError):
        E.BatchSolver([dp], W.GA(pop=64, n_elite=4, generations=1, sigma=0.1, seed=0))
    chain = W.pendulum_chain(2, 20, 4, seed=1)
    chain.R = np.eye(2)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(E.DeviceProblem(chain, F32), torch.zeros(4, device="cuda"),
                            torch.zeros(8, 16, device="cuda"), 16, 16,
                            torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL


# ---------------------------------------------------------------------------
# step charge outside the state box (every rollout form)

# (model maker, d, T, p, candidates, half width): linear one-wavefront form
# (4 states), M-split form (28 states), chain lane form (5 joints) and row
# form (20 joints)
SB_CASES = [(W.linear_chain, 2, 20, 5, 70, 0.3), (W.linear_chain, 14, 50, 10, 300, 0.2),
            (W.pendulum_chain, 5, 40, 5, 200, 0.3), (W.pendulum_chain, 20, 40, 5, 64, 0.3)]


@pytest.mark.parametrize("case", range(len(SB_CASES)))
def test_step_charge_fp64(oracle_lib, E, case):
    mk, d, T, p, nc, hw = SB_CASES[case]
    prob = boxed(mk(d, T, p, seed=d), d, hw)
    got, want = compare(oracle_lib, E, prob, ncand=nc, ld=nc + 3, dtype=F64, seed=d,
                        rtol=1e-9)
    plain = oracle_lib.rollout_cost(W.dataclasses.replace(rounded(prob, F64), sb=None),
                                    W.draw_x0(prob.n, d),
                                    W.draw_knots(prob, nc, d + 1, ld=nc + 3), nc)
    assert np.all(want > plain)  # the charge was paid


@pytest.mark.parametrize("case", range(len(SB_CASES)))
def test_step_charge_fp32_every_state_outside(oracle_lib, E, case):
    mk, d, T, p, nc, hw = SB_CASES[case]
    prob = boxed(mk(d, T, p, seed=d), d, hw)
    prob.x_min, prob.x_max = prob.x_min + 100.0, prob.x_max + 100.0
    compare(oracle_lib, E, prob, ncand=nc, ld=nc, dtype=F32, seed=d, rtol=RTOL[F32])


@pytest.mark.parametrize("dtype", [F32, F64])
def test_step_charge_absent_or_zero_keeps_the_bits(E, dtype):
    for mk, d in ((W.linear_chain, 14), (W.pendulum_chain, 20), (W.linear_chain, 2)):
        prob = boxed(mk(d, 30, 5, seed=d), d, 0.2).cast(npdt(dtype))
        x0 = W.draw_x0(prob.n, 1)
        knots = W.draw_knots(prob, 100, 2)
        a = gpu_costs(E, W.dataclasses.replace(prob, sb=None), x0, knots, 100, dtype)
        b = gpu_costs(E, W.dataclasses.replace(prob, sb=np.zeros(prob.n)), x0, knots, 100,
                      dtype)
        np.testing.assert_array_equal(a, b)


def test_step_charge_needs_the_box(E):
    prob = W.linear_chain(2, 10, 3, seed=0)
    prob.sb = np.ones(prob.n)
    dp = E.DeviceProblem(prob, F32)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(dp, torch.zeros(4, device="cuda"), torch.zeros(6, 16, device="cuda"),
                            16, 16, torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL


def test_step_charge_batched_equals_single(E):
    probs = []
    for i, (mk, d) in enumerate(((W.linear_chain, 2), (W.linear_chain, 14),
                                 (W.pendulum_chain, 5), (W.pendulum_chain, 20))):
        probs.append(boxed(mk(d, 30, 5, seed=40 + i), i, 0.2).cast(np.float32))
    ga = W.GA(pop=128, n_elite=8, generations=2, sigma=0.1, seed=12)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga)
    singles = [E.Solver(dp, W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
               for i, dp in enumerate(dps)]
    x0s = [W.draw_x0(p.n, 3 + i).astype(np.float32) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    for tick in range(2):
        bs.solve()
        torch.cuda.synchronize()
        for i, s in enumerate(singles):
            u, J = s.solve(torch.tensor(x0s[i], device="cuda"), tick)
            torch.cuda.synchronize()
            assert torch.equal(bs.u_of(i), u), (tick, i)
            assert torch.equal(bs.best_cost[i:i + 1], J), (tick, i)
    bs.close()


def test_step_charge_refined_solve_fp64(oracle_lib, E):
    # the adjoint's own cost includes the charge (its derivative is zero off
    # the faces), so refinement accepts the same candidates as the oracle
    prob = boxed(W.linear_chain(2, 20, 5, seed=2), 2, 0.3)
    ga = W.GA(pop=128, n_elite=8, generations=3, sigma=0.1, seed=9)
    solver = E.Solver(E.DeviceProblem(prob, F64), ga)
    osolver = oracle_lib.Solver(prob, ga, refine=True)
    x = W.draw_x0(prob.n, 2)
    for tick in range(3):
        u, J = solver.solve(as_dev(x, F64), tick, refine_steps=5)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        x = oracle_lib.step(prob, x, uo)


# ---------------------------------------------------------------------------
# joint limits with impacts (pendulum chain: lane and row forms, plant)


def limited(prob, seed, lo=-0.15, hi=0.2, e=0.4):
    rng = np.random.default_rng(seed)
    d = prob.m
    return W.dataclasses.replace(prob, q_min=lo * rng.uniform(0.5, 1.5, d),
                                 q_max=hi * rng.uniform(0.5, 1.5, d), restitution=e)


def start_inside(prob, seed):
    x0 = W.draw_x0(prob.n, seed)
    d = prob.m
    x0[:d] = np.clip(x0[:d], prob.q_min, prob.q_max)
    return x0


@pytest.mark.parametrize("d", [1, 3, 5, 8, 12, 20, 36])
@pytest.mark.parametrize("box", [False, True])
def test_joint_limits_fp64(oracle_lib, E, d, box):
    lo, hi = (-0.05, 0.05) if d == 1 else (-0.15, 0.2)  # one joint swings less
    prob = limited(W.pendulum_chain(d, 40, 5, seed=d), d, lo, hi)
    if box:
        prob = boxed(prob, d, 0.3)
    x0 = start_inside(prob, d)
    knots = W.draw_knots(prob, 150, d + 1, ld=151)
    got = gpu_costs(E, prob, x0, knots, 150, F64)
    want = oracle_lib.rollout_cost(prob, x0, knots, 150)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=0)
    free = oracle_lib.rollout_cost(W.dataclasses.replace(prob, q_min=None, q_max=None), x0,
                                   knots, 150)
    assert np.any(np.abs(want - free) > 1e-6 * np.abs(free))  # the limits acted


@pytest.mark.parametrize("d", [5, 20])
def test_joint_limits_fp32_mostly_agree(oracle_lib, E, d):
    # each impact is decided in FP32; a joint within rounding of its limit
    # may take the other branch, so most (not all) candidates must agree
    prob = limited(W.pendulum_chain(d, 40, 5, seed=d), d).cast(np.float32)
    x0 = start_inside(prob, d).astype(np.float32).astype(np.float64)
    knots = W.draw_knots(prob, 400, d + 1).astype(np.float32).astype(np.float64)
    got = gpu_costs(E, prob, x0, knots, 400, F32)
    want = oracle_lib.rollout_cost(prob, x0, knots, 400)
    rel = np.abs(got - want) / np.abs(want)
    assert np.mean(rel < 1e-4) >= 0.9, np.sort(rel)[-10:]
    assert np.median(rel) < 1e-5


def test_joint_limits_wide_keep_the_bits(E):
    for d in (5, 20):
        prob = W.pendulum_chain(d, 30, 5, seed=d).cast(np.float32)
        x0 = W.draw_x0(prob.n, 1)
        knots = W.draw_knots(prob, 64, 2)
        a = gpu_costs(E, prob, x0, knots, 64, F32)
        wide = W.dataclasses.replace(prob, q_min=np.full(d, -1e6), q_max=np.full(d, 1e6),
                                     restitution=0.5)
        np.testing.assert_array_equal(gpu_costs(E, wide, x0, knots, 64, F32), a)


def test_joint_limits_plant_and_solve_fp64(oracle_lib, E):
    prob = limited(W.pendulum_chain(4, 30, 5, seed=4), 4, e=0.6)
    ga = W.GA(pop=200, n_elite=10, generations=4, sigma=0.2, seed=3)
    dp = E.DeviceProblem(prob, F64)
    solver = E.Solver(dp, ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = start_inside(prob, 4)
    for tick in range(4):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        # the plant: a large torque drives the joints onto their limits
        push = 3.0 * np.sign(uo + 1e-3)
        xg = torch.empty(prob.n, dtype=F64, device="cuda")
        E.empc_plant_step(dp, as_dev(x, F64), as_dev(push, F64), None, xg)
        xo = oracle_lib.step(prob, x, push)
        np.testing.assert_allclose(xg.cpu().numpy(), xo, rtol=1e-12, atol=1e-14)
        x = oracle_lib.step(prob, x, uo)


def test_joint_limits_refused_where_unsupported(E):
    prob = limited(W.pendulum_chain(3, 20, 4, seed=1), 1)
    dp = E.DeviceProblem(prob, F32)
    K = torch.zeros(prob.p * prob.m, 16, device="cuda")
    with pytest.raises(E.EmpcError) as ex:
        E.empc_grad(dp, torch.zeros(prob.n, device="cuda"), K, 16, 16, torch.empty_like(K),
                    torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EUNSUPPORTED
    with pytest.raises(E.EmpcError):
        E.BatchSolver([dp], W.GA(pop=64, n_elite=4, generations=1, sigma=0.1, seed=0))
    bad = W.dataclasses.replace(prob, restitution=1.5)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(E.DeviceProblem(bad, F32), torch.zeros(prob.n, device="cuda"), K,
                            16, 16, torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL
    lin = W.linear_chain(2, 20, 4, seed=1)
    lin.q_min, lin.q_max = -np.ones(2), np.ones(2)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(E.DeviceProblem(lin, F32), torch.zeros(4, device="cuda"),
                            torch.zeros(8, 16, device="cuda"), 16, 16,
                            torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL


# ---------------------------------------------------------------------------
# dry friction with stiction (pendulum chain: lane and row forms, plant)


def frictional(prob, seed, tc=0.05, ts=0.12):
    rng = np.random.default_rng(seed)
    d = prob.m
    c = tc * rng.uniform(0.5, 1.5, d)
    return W.dataclasses.replace(prob, fric_c=c, fric_s=c + ts * rng.uniform(0.5, 1.5, d))


@pytest.mark.parametrize("d", [1, 3, 5, 8, 12, 20, 36])
@pytest.mark.parametrize("extra", ["", "box", "limits"])
def test_dry_friction_fp64(oracle_lib, E, d, extra):
    prob = frictional(W.pendulum_chain(d, 40, 5, seed=d), d)
    if extra == "box":
        prob = boxed(prob, d, 0.3)
    elif extra == "limits":
        prob = limited(prob, d)
    x0 = start_inside(prob, d) if extra == "limits" else W.draw_x0(prob.n, d)
    x0[prob.m:prob.m + (d + 1) // 2] = 0.0  # some joints start at rest
    knots = W.draw_knots(prob, 150, d + 1, ld=151)
    got = gpu_costs(E, prob, x0, knots, 150, F64)
    want = oracle_lib.rollout_cost(prob, x0, knots, 150)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=0)
    free = oracle_lib.rollout_cost(W.dataclasses.replace(prob, fric_c=None, fric_s=None), x0,
                                   knots, 150)
    assert np.any(np.abs(want - free) > 1e-6 * np.abs(free))  # the friction acted


@pytest.mark.parametrize("d", [5, 20])
def test_dry_friction_fp32_mostly_agree(oracle_lib, E, d):
    # every stick / slip decision is taken in FP32: a torque within rounding
    # of the breakaway torque may go the other way, so most (not all)
    # candidates must agree
    prob = frictional(W.pendulum_chain(d, 40, 5, seed=d), d).cast(np.float32)
    x0 = W.draw_x0(prob.n, d).astype(np.float32).astype(np.float64)
    knots = W.draw_knots(prob, 400, d + 1).astype(np.float32).astype(np.float64)
    got = gpu_costs(E, prob, x0, knots, 400, F32)
    want = oracle_lib.rollout_cost(prob, x0, knots, 400)
    rel = np.abs(got - want) / np.abs(want)
    assert np.mean(rel < 1e-4) >= 0.9, np.sort(rel)[-10:]
    assert np.median(rel) < 1e-5


def test_zero_friction_keeps_the_bits(E):
    for d in (5, 20):
        prob = W.pendulum_chain(d, 30, 5, seed=d).cast(np.float32)
        x0 = W.draw_x0(prob.n, 1)
        knots = W.draw_knots(prob, 64, 2)
        a = gpu_costs(E, prob, x0, knots, 64, F32)
        zero = W.dataclasses.replace(prob, fric_c=np.zeros(d), fric_s=np.zeros(d))
        np.testing.assert_array_equal(gpu_costs(E, zero, x0, knots, 64, F32), a)


def test_dry_friction_plant_and_solve_fp64(oracle_lib, E):
    prob = frictional(W.pendulum_chain(4, 30, 5, seed=4), 4, tc=0.1, ts=0.2)
    ga = W.GA(pop=200, n_elite=10, generations=4, sigma=0.2, seed=3)
    dp = E.DeviceProblem(prob, F64)
    solver = E.Solver(dp, ga)
    osolver = oracle_lib.Solver(prob, ga)
    x = W.draw_x0(prob.n, 4)
    x[4:6] = 0.0
    for tick in range(4):
        u, J = solver.solve(as_dev(x, F64), tick)
        uo, Jo, _ = osolver.solve(x, tick)
        np.testing.assert_allclose(u.cpu().numpy(), uo, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(float(J.item()), Jo, rtol=1e-9)
        for push in (0.05 * np.sign(uo + 1e-3), 3.0 * np.sign(uo + 1e-3)):
            xr = x.copy()
            xr[4:] = 0.0  # at rest: held below breakaway, breaking away above
            xg = torch.empty(prob.n, dtype=F64, device="cuda")
            E.empc_plant_step(dp, as_dev(xr, F64), as_dev(push, F64), None, xg)
            xo = oracle_lib.step(prob, xr, push)
            np.testing.assert_allclose(xg.cpu().numpy(), xo, rtol=1e-12, atol=1e-14)
        x = oracle_lib.step(prob, x, uo)


def test_dry_friction_refused_where_unsupported(E):
    prob = frictional(W.pendulum_chain(3, 20, 4, seed=1), 1)
    dp = E.DeviceProblem(prob, F32)
    K = torch.zeros(prob.p * prob.m, 16, device="cuda")
    with pytest.raises(E.EmpcError) as ex:
        E.empc_grad(dp, torch.zeros(prob.n, device="cuda"), K, 16, 16, torch.empty_like(K),
                    torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EUNSUPPORTED
    with pytest.raises(E.EmpcError):
        E.BatchSolver([dp], W.GA(pop=64, n_elite=4, generations=1, sigma=0.1, seed=0))
    half = W.dataclasses.replace(prob, fric_s=None)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(E.DeviceProblem(half, F32), torch.zeros(prob.n, device="cuda"), K,
                            16, 16, torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL
    lin = W.linear_chain(2, 20, 4, seed=1)
    lin.fric_c, lin.fric_s = np.ones(2), np.ones(2)
    with pytest.raises(E.EmpcError) as ex:
        E.empc_rollout_cost(E.DeviceProblem(lin, F32), torch.zeros(4, device="cuda"),
                            torch.zeros(8, 16, device="cuda"), 16, 16,
                            torch.empty(16, device="cuda"))
    assert ex.value.status == E.EMPC_EINVAL
