"""empc_solve_static (the solve whose workspace is the library's static
device array, for callers that cannot allocate) against empc_solve on a
caller-allocated, zero-filled workspace: the same kernels run on the same
inputs, so u* and the best cost agree bit for bit, tick after tick, and a
second problem of a smaller size solved afterwards in the same array gives
again what empc_solve gives."""
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


def run_both(E, prob, ga, dtype, ticks, x_seed):
    """(static, allocated) lists of (u*, best cost) over `ticks` ticks, the
    first tick cold, the next ones warm, on the same states."""
    dp = E.DeviceProblem(prob.cast(np.float32) if dtype == F32 else prob, dtype)
    ref = E.Solver(dp, ga)
    u = torch.zeros(prob.m, dtype=dtype, device="cuda")
    J = torch.zeros(1, dtype=dtype, device="cuda")
    xs = [W.draw_x0(prob.n, x_seed + t) for t in range(ticks)]
    got, want = [], []
    for t in range(ticks):
        x = dev(xs[t], dtype)
        E.empc_solve_static(dp, ref.ga, x, t, 1 if t == 0 else 0, u, J)
        got.append((u.clone(), J.clone()))
        ur, Jr = ref.solve(x, t)
        want.append((ur.clone(), Jr.clone()))
    torch.cuda.synchronize()
    return got, want


def test_static_solve_equals_allocated_solve(E):
    # first a 14-DoF FP32 problem (population 4096, 28 states), then a
    # smaller 2-DoF FP64 one in the same static array: each equals the
    # allocated-workspace solve bit for bit on every tick
    prob, ga = W.config_c2(0)
    ga = W.dataclasses.replace(ga, generations=4)
    got, want = run_both(E, prob, ga, F32, 3, 10)
    for (u, J), (ur, Jr) in zip(got, want):
        assert torch.equal(u, ur) and torch.equal(J, Jr)
    assert np.isfinite(got[-1][1].item())

    prob, ga = W.config_c1(0)
    got, want = run_both(E, prob, ga, F64, 3, 20)
    for (u, J), (ur, Jr) in zip(got, want):
        assert torch.equal(u, ur) and torch.equal(J, Jr)


def test_static_solve_cold_restarts(E):
    # cold = 1 after other solves in the array gives the first-tick result
    # again (the warm-start state is cleared, nothing else is read)
    prob, ga = W.config_c1(0)
    dp = E.DeviceProblem(prob, F64)
    x = dev(W.draw_x0(prob.n, 3), F64)
    u = torch.zeros(prob.m, dtype=F64, device="cuda")
    J = torch.zeros(1, dtype=F64, device="cuda")
    E.empc_solve_static(dp, E.make_ga(ga), x, 0, 1, u, J)
    first = (u.clone(), J.clone())
    E.empc_solve_static(dp, E.make_ga(ga), x, 1, 0, u, J)
    E.empc_solve_static(dp, E.make_ga(ga), x, 0, 1, u, J)
    torch.cuda.synchronize()
    assert torch.equal(u, first[0]) and torch.equal(J, first[1])


def test_static_solve_limits(E):
    # a workspace above the static array is refused before any launch, and
    # so is a cold flag other than 0 / 1
    prob, ga = W.config_c3(0)
    big = W.dataclasses.replace(ga, pop=65536)
    dp = E.DeviceProblem(prob.cast(np.float32), F32)
    x = torch.zeros(prob.n, dtype=F32, device="cuda")
    u = torch.zeros(prob.m, dtype=F32, device="cuda")
    J = torch.zeros(1, dtype=F32, device="cuda")
    assert E.empc_workspace_bytes(dp, E.make_ga(big)) > (64 << 20)
    with pytest.raises(E.EmpcError) as ei:
        E.empc_solve_static(dp, E.make_ga(big), x, 0, 1, u, J)
    assert ei.value.status == E.binding.EMPC_EUNSUPPORTED
    with pytest.raises(E.EmpcError) as ei:
        E.empc_solve_static(dp, E.make_ga(ga), x, 0, 2, u, J)
    assert ei.value.status == E.binding.EMPC_EINVAL
