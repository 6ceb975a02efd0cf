"""Problem-batched EMPC (empc_solve_batched) on the GPU.

Problem i of a batch draws from the Philox key (seed_lo, seed_hi ^ i), so it
must evolve exactly like a single-problem solve (empc_solve) with seed
seed ^ (i << 32): the two are compared bit for bit over several generations
and ticks.  The first generation is also compared with the FP64 oracle, and
a HIP-graph-captured tick is replayed against eager ticks."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

F32 = torch.float32


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    assert torch.cuda.is_available()
    E.lib()
    return E


def mixed_problems(seed=0):
    """Every kernel shape class of the batching configuration, plus ragged
    horizons and knot counts."""
    rng = np.random.default_rng(seed)
    probs = []
    for i, d in enumerate(W.C5_DOFS):
        for kind in (W.LINEAR, W.PENDULUM_CHAIN):
            T = int(rng.integers(20, 101))
            p = int(rng.integers(5, 11))
            mk = W.linear_chain if kind == W.LINEAR else W.pendulum_chain
            probs.append(mk(d, T, p, seed=100 * i + kind).cast(np.float32))
    return probs


@pytest.mark.parametrize("variant", [{}, dict(shift=True, sigma_min=0.01, sigma_dist=0.8)])
def test_batched_equals_single_solves(E, variant):
    probs = mixed_problems()
    ga = W.GA(pop=256, n_elite=16, generations=2, sigma=0.1, seed=0xABCDEF0123, **variant)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga)
    singles = [E.Solver(dp, W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
               for i, dp in enumerate(dps)]
    x0s = [W.draw_x0(p.n, 7 + i).astype(np.float32) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    for tick in range(3):
        bs.solve()
        torch.cuda.synchronize()
        for i, (s, dp) in enumerate(zip(singles, dps)):
            u, J = s.solve(torch.tensor(x0s[i], device="cuda"), tick)
            torch.cuda.synchronize()
            assert torch.equal(bs.u_of(i), u), (tick, i)
            assert torch.equal(bs.best_cost[i:i + 1], J), (tick, i)
    bs.close()


def test_batched_first_generation_matches_oracle(oracle_lib, E):
    probs = mixed_problems(1)
    ga = W.GA(pop=256, n_elite=16, generations=1, sigma=0.1, seed=5)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga)
    x0s = [W.draw_x0(p.n, i).astype(np.float32).astype(np.float64) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    bs.solve()
    torch.cuda.synchronize()
    best = bs.best_cost.cpu().numpy()
    for i, p in enumerate(probs):
        o = oracle_lib.Solver(p, W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
        u, J, _ = o.solve(x0s[i], 0)
        np.testing.assert_allclose(best[i], J, rtol=1e-4, err_msg="problem %d" % i)
    bs.close()


def test_batched_graph_replay_matches_eager(E):
    probs = mixed_problems(2)[:6]
    ga = W.GA(pop=256, n_elite=16, generations=1, sigma=0.1, seed=9)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    eager = E.BatchSolver(dps, ga)
    graphed = E.BatchSolver(dps, ga)
    for i, p in enumerate(probs):
        x = W.draw_x0(p.n, i)
        eager.set_x0(i, x)
        graphed.set_x0(i, x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.solve()
    # capture recorded the launches without running them: tick 0 is the
    # first replay
    for tick in range(4):
        eager.solve()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eager.u_star, graphed.u_star), tick
        assert torch.equal(eager.best_cost, graphed.best_cost), tick
        # eager host work between replays
        _ = eager.u_star.cpu()
    eager.close()
    graphed.close()


def _run_ticks(bs, x0s, ticks):
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    out = []
    for _ in range(ticks):
        bs.solve()
        torch.cuda.synchronize()
        out.append((bs.u_star.clone(), bs.best_cost.clone()))
    return out


def test_batch_launch_shapes_round_identically(E):
    """Every launch shape of every kernel class gives the same bits: the
    shape only changes how candidates are packed into workgroups."""
    probs = mixed_problems(2)
    ga = W.GA(pop=200, n_elite=8, generations=2, sigma=0.1, seed=77)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    x0s = [W.draw_x0(p.n, 30 + i).astype(np.float32) for i, p in enumerate(probs)]
    base = E.BatchSolver(dps, ga, autotune=False)
    classes = base.classes()
    assert {c["model"] for c in classes} == {"linear", "pendulum_chain"}
    assert any(c["variants"] == 4 for c in classes)  # a linear class with the M-split form
    ref = _run_ticks(base, x0s, 2)
    base.close()
    for v in range(4):
        bs = E.BatchSolver(dps, ga, autotune=False)
        for ci, c in enumerate(bs.classes()):
            bs.set_variant(ci, min(v, c["variants"] - 1))
        assert all(c["variant"] == min(v, c["variants"] - 1) for c in bs.classes())
        got = _run_ticks(bs, x0s, 2)
        for t, ((u0, j0), (u1, j1)) in enumerate(zip(ref, got)):
            assert torch.equal(u0, u1), (v, t)
            assert torch.equal(j0, j1), (v, t)
        with pytest.raises(E.EmpcError):
            bs.set_variant(0, classes[0]["variants"])
        bs.close()


def test_batch_valu_form_equals_single_valu_solves(E):
    """The vector-ALU shape of the small linear classes, offered only when
    the plan allows it, gives each problem the bits of its single solve with
    the VALU form pinned (64 threads); withdrawing it puts the classes back
    on a matrix-core shape.  A class whose problems pad to different state
    counts is not offered the form."""
    probs = [p for p in mixed_problems(3) if p.model == W.LINEAR and p.n <= 16]
    assert sorted(p.n for p in probs) == [4, 14]
    ga = W.GA(pop=200, n_elite=8, generations=2, sigma=0.1, seed=0x5151)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga, autotune=False)
    assert all(c["variants"] == 3 for c in bs.classes())
    bs.allow_valu(True)
    for ci, c in enumerate(bs.classes()):
        assert c["variants"] == 4
        bs.set_variant(ci, 3)
    x0s = [W.draw_x0(p.n, 50 + i).astype(np.float32) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    singles = []
    try:
        for i, dp in enumerate(dps):
            g = W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32))
            E.empc_autotune_set(dp, E.make_ga(g), E.RF_VALU64, 0)
            singles.append(E.Solver(dp, g))
        for tick in range(3):
            bs.solve()
            torch.cuda.synchronize()
            for i, s in enumerate(singles):
                u, J = s.solve(torch.tensor(x0s[i], device="cuda"), tick)
                torch.cuda.synchronize()
                assert torch.equal(bs.u_of(i), u), (tick, i)
                assert torch.equal(bs.best_cost[i:i + 1], J), (tick, i)
    finally:
        E.empc_autotune_reset()
    bs.allow_valu(False)
    assert all(c["variant"] == 0 and c["variants"] == 3 for c in bs.classes())
    with pytest.raises(E.EmpcError):
        bs.set_variant(0, 3)
    bs.close()
    # n = 4 and n = 6 share a class (one state tile, one input slice) but pad
    # to 4 and 8 states in the VALU form
    mixed = [W.linear_chain(2, 30, 5, seed=1).cast(np.float32),
             W.linear_chain(3, 30, 5, seed=2).cast(np.float32)]
    bm = E.BatchSolver([E.DeviceProblem(p, F32) for p in mixed], ga, autotune=False)
    bm.allow_valu(True)
    assert [c["variants"] for c in bm.classes()] == [3]
    bm.close()


def test_batch_autotune_keeps_state_and_results(E):
    """Autotuning between two ticks leaves the warm-start state alone: the
    second tick equals that of an untuned plan."""
    probs = mixed_problems(3)
    ga = W.GA(pop=256, n_elite=16, generations=2, sigma=0.1, seed=91)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    x0s = [W.draw_x0(p.n, 50 + i).astype(np.float32) for i, p in enumerate(probs)]
    plain = E.BatchSolver(dps, ga, autotune=False)
    ref = _run_ticks(plain, x0s, 2)
    plain.close()
    tuned = E.BatchSolver(dps, ga, autotune=True, tune_reps=2)
    got = _run_ticks(tuned, x0s, 1)
    tuned.autotune(2)
    for c in tuned.classes():
        assert 0 <= c["variant"] < c["variants"] and 0 <= c["stream"] < 4
    got += _run_ticks(tuned, x0s, 1)
    for t, ((u0, j0), (u1, j1)) in enumerate(zip(ref, got)):
        assert torch.equal(u0, u1), t
        assert torch.equal(j0, j1), t
    tuned.close()


@pytest.mark.parametrize("pop", [6000, 12000])
def test_large_population_single_matches_batched(E, pop):
    """A C3-sized chain (360 parameters) with a large population: the
    single-problem solve (1024-thread selection, parents read in place after
    the first generation) equals the batched one bit for bit.  Both sides
    size their population grid the same way here (32 parameters per
    workgroup at 6000, 64 at 12000), so this checks the two launch paths,
    not the grouping; test_population_grouping_matches_oracle in the parity
    tests checks the grouped populations against the oracle."""
    prob = W.pendulum_chain(36, 100, 10, seed=4).cast(np.float32)
    ga = W.GA(pop=pop, n_elite=64, generations=3, sigma=0.1, seed=0x5EED)
    dp = E.DeviceProblem(prob, F32)
    bs = E.BatchSolver([dp], ga, autotune=False)
    single = E.Solver(dp, ga)  # problem 0 of a batch uses the seed unchanged
    x0 = W.draw_x0(prob.n, 11).astype(np.float32)
    bs.set_x0(0, x0)
    for tick in range(2):
        bs.solve()
        u, J = single.solve(torch.tensor(x0, device="cuda"), tick)
        torch.cuda.synchronize()
        assert torch.equal(bs.u_of(0), u), tick
        assert torch.equal(bs.best_cost[0:1], J), tick
    bs.close()


def test_batched_box_penalty_equals_single(E):
    """Problems of both models carry a state box penalty (their own kernel
    classes, beside box-free problems of the same shapes): batch and single
    solves agree bit for bit."""
    boxed, probs = mixed_problems(5), mixed_problems(6)
    rng = np.random.default_rng(5)
    for i, p in enumerate(boxed):
        if i % 4 < 2:  # both models at 2, 14 and 36 degrees of freedom
            hw = 0.1 * rng.uniform(0.5, 1.5, p.n)
            p.x_min, p.x_max = -hw, hw
            p.qb = rng.uniform(1.0, 4.0, p.n)
    probs = [p.cast(np.float32) for p in boxed + probs]
    ga = W.GA(pop=128, n_elite=8, generations=2, sigma=0.1, seed=77)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga)
    assert len(bs.classes()) == 16  # 10 shape classes, 6 of them also with a box
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


def test_population_grouping_keeps_the_bits(E):
    """Six 36-link chains at population 2048: alone, each population launch
    has 736 workgroups of 16 parameters; the batch has 4416 and takes 64
    parameters per workgroup.  Every draw keeps its counter, so the batched
    and the single solves agree bit for bit."""
    probs = [W.pendulum_chain(36, 100, 10, seed=20 + i).cast(np.float32) for i in range(6)]
    ga = W.GA(pop=2048, n_elite=32, generations=2, sigma=0.1, seed=0xC0FFEE)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga, autotune=False)
    singles = [E.Solver(dp, W.dataclasses.replace(ga, seed=ga.seed ^ (i << 32)))
               for i, dp in enumerate(dps)]
    x0s = [W.draw_x0(p.n, 40 + i).astype(np.float32) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    for tick in range(2):
        bs.solve()
        torch.cuda.synchronize()
        for i, sv in enumerate(singles):
            u, J = sv.solve(torch.tensor(x0s[i], device="cuda"), tick)
            torch.cuda.synchronize()
            assert torch.equal(bs.u_of(i), u), (tick, i)
            assert torch.equal(bs.best_cost[i:i + 1], J), (tick, i)
    bs.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_c5_plan_sampled_against_single_solves(E, mode):
    """The full batching configuration (512 problems, population 1024,
    autotuned launch shapes or the persistent form, one HIP-graph replay per
    tick): 16 sampled problems equal their single-problem solves bit for bit
    over two ticks."""
    probs, ga = W.config_c5(512, 0)
    probs = [p.cast(np.float32) for p in probs]
    dps = [E.DeviceProblem(p, F32) for p in probs]
    bs = E.BatchSolver(dps, ga, autotune=mode == 0)
    bs.set_mode(mode)
    x0s = [W.draw_x0(p.n, i).astype(np.float32) for i, p in enumerate(probs)]
    for i, x in enumerate(x0s):
        bs.set_x0(i, x)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bs.solve()
    sample = np.random.default_rng(0).choice(len(probs), 16, replace=False)
    singles = {int(i): E.Solver(dps[i], W.dataclasses.replace(ga, seed=ga.seed ^ (int(i) << 32)))
               for i in sample}
    for tick in range(2):
        graph.replay()
        torch.cuda.synchronize()
        for i, s in singles.items():
            u, J = s.solve(torch.tensor(x0s[i], device="cuda"), tick)
            torch.cuda.synchronize()
            assert torch.equal(bs.u_of(i), u), (tick, i)
            assert torch.equal(bs.best_cost[i:i + 1], J), (tick, i)
    bs.close()


def test_persistent_form_equals_class_launches(E):
    """The persistent work-queue form (one kernel per register tier, the last
    tile of a problem selecting for it) gives the bits of the per-class
    launches, tick after tick, for every kernel class, ragged populations
    (units of 16 and 64 candidates with tails) and two generations per
    tick."""
    probs = mixed_problems(3)
    for pop in (256, 200):
        ga = W.GA(pop=pop, n_elite=16, generations=2, sigma=0.1, seed=77)
        dps = [E.DeviceProblem(p, F32) for p in probs]
        a = E.BatchSolver(dps, ga)
        b = E.BatchSolver(dps, ga, autotune=False)
        b.set_mode(1)
        x0s = [W.draw_x0(p.n, 40 + i).astype(np.float32) for i, p in enumerate(probs)]
        ra = _run_ticks(a, x0s, 3)
        rb = _run_ticks(b, x0s, 3)
        for t, ((ua, ja), (ub, jb)) in enumerate(zip(ra, rb)):
            assert torch.equal(ua, ub), (pop, t)
            assert torch.equal(ja, jb), (pop, t)
        a.close()
        b.close()


def test_persistent_form_graph_replay(E):
    """A HIP graph of the persistent form's tick (its counters are cleared by
    the population kernel, the tick advanced by the last selection) replays
    tick after tick like eager ticks of the per-class form."""
    probs = mixed_problems(4)
    ga = W.GA(pop=128, n_elite=8, generations=1, sigma=0.1, seed=21)
    dps = [E.DeviceProblem(p, F32) for p in probs]
    eager = E.BatchSolver(dps, ga, autotune=False)
    graphed = E.BatchSolver(dps, ga, autotune=False)
    graphed.set_mode(1)
    for i, p in enumerate(probs):
        x = W.draw_x0(p.n, i)
        eager.set_x0(i, x)
        graphed.set_x0(i, x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.solve()
    for tick in range(4):
        eager.solve()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eager.u_star, graphed.u_star), tick
        assert torch.equal(eager.best_cost, graphed.best_cost), tick
        _ = eager.u_star.cpu()
    eager.close()
    graphed.close()


def test_persistent_form_limits(E):
    # the box penalty and populations above 1024 stay on the per-class form
    probs = mixed_problems(5)[:3]
    ga = W.GA(pop=64, n_elite=8, generations=1, sigma=0.1, seed=1)
    boxed = probs[0]
    boxed = W.dataclasses.replace(boxed, x_min=np.full(boxed.n, -1.0), x_max=np.full(boxed.n, 1.0),
                                  qb=np.ones(boxed.n))
    bs = E.BatchSolver([E.DeviceProblem(p, F32) for p in [boxed] + probs[1:]], ga,
                       autotune=False)
    with pytest.raises(E.EmpcError) as ei:
        bs.set_mode(1)
    assert ei.value.status == E.binding.EMPC_EUNSUPPORTED
    bs.close()
    big = W.dataclasses.replace(ga, pop=2048)
    bs = E.BatchSolver([E.DeviceProblem(p, F32) for p in probs], big, autotune=False)
    with pytest.raises(E.EmpcError):
        bs.set_mode(1)
    with pytest.raises(E.EmpcError):
        bs.set_mode(2)
    bs.close()
