"""Host-side checks of libempc.so that need no GPU: every symbol declared in
include/empc.h is exported, and argument validation rejects bad calls before
anything reaches the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "empc.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(empc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def E():
    import paper_2001_04931_amd as E

    if not os.path.exists(E.binding.LIB_PATH):
        pytest.skip("libempc.so not built")
    E.lib()
    return E


def test_header_symbols_exported(E):
    names = header_functions()
    assert len(names) >= 10
    L = ctypes.CDLL(E.binding.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert sorted(E.binding.exported_symbols()) == names


def _problem(E, **over):
    c = E.EmpcProblem()
    c.n, c.m, c.T, c.p, c.dtype, c.model = 4, 2, 10, 3, 0, 0
    fake = ctypes.c_void_p(0x1000)
    for f in ("Ad", "Bd", "q", "r", "u_min", "u_max"):
        setattr(c, f, fake)
    for k, v in over.items():
        setattr(c, k, v)
    return c


def _call_rollout(E, c, ncand=8, ld=8):
    fake = ctypes.c_void_p(0x2000)
    return E.lib().empc_rollout_cost(ctypes.byref(c), fake, fake, ncand, ld, fake, None)


@pytest.mark.parametrize("over,status", [
    (dict(p=11), 1), (dict(p=0), 1), (dict(T=0), 1), (dict(n=0), 1), (dict(dtype=7), 1),
    (dict(model=5), 1), (dict(Ad=None), 1), (dict(u_max=None), 1),
    (dict(n=81), 3), (dict(m=41), 3),
    (dict(model=1, n=6, m=3), 1),                       # chain without its parameters
])
def test_rollout_validation(E, over, status):
    st = _call_rollout(E, _problem(E, **over))
    assert st == status
    assert E.lib().empc_last_error().decode() != ""


def test_rollout_bad_sizes(E):
    assert _call_rollout(E, _problem(E), ncand=9, ld=8) == 1
    assert _call_rollout(E, _problem(E), ncand=-1, ld=8) == 1
    assert E.lib().empc_rollout_cost(None, None, None, 1, 1, None, None) == 1


def test_chain_validation(E):
    fake = ctypes.c_void_p(0x1000)
    c = _problem(E, model=1, n=6, m=3, stiffness=fake, damping=fake, mass=fake, length=fake)
    c.dt = 0.0
    assert _call_rollout(E, c) == 1
    c.dt = 0.005
    c.n = 7
    assert _call_rollout(E, c) == 1
    c.n, c.m = 82, 41
    assert _call_rollout(E, c) == 3


def test_ga_validation_and_workspace_size(E):
    c = _problem(E)
    g = E.EmpcGA()
    g.pop, g.n_elite, g.generations, g.elitism, g.sigma, g.seed = 100, 10, 2, 1, 0.1, 0
    nb = E.lib().empc_workspace_bytes(ctypes.byref(c), ctypes.byref(g))
    assert nb >= 4 * (c.p * c.m * 100 + 100 + 10 * c.p * c.m)
    for field, val in (("n_elite", 101), ("n_elite", 0), ("pop", 0), ("generations", 0),
                       ("n_elite", 300), ("sigma", -1.0)):
        g2 = E.EmpcGA.from_buffer_copy(g)
        setattr(g2, field, val)
        if field == "n_elite" and val == 300:
            g2.pop = 1000
        assert E.lib().empc_workspace_bytes(ctypes.byref(c), ctypes.byref(g2)) == 0
    fake = ctypes.c_void_p(0x3000)
    st = E.lib().empc_solve(ctypes.byref(c), ctypes.byref(g), fake, nb - 1, fake, 0, fake, fake,
                            None)
    assert st == 4
    st = E.lib().empc_solve(ctypes.byref(c), ctypes.byref(g), None, nb, fake, 0, fake, fake, None)
    assert st == 4


def test_static_solve_validation(E):
    # the no-allocation solve refuses bad arguments and workspaces above its
    # static array on the host, before it looks up the array or launches
    c = _problem(E)
    g = E.EmpcGA()
    g.pop, g.n_elite, g.generations, g.elitism, g.sigma, g.seed = 100, 10, 2, 1, 0.1, 0
    L = E.lib()
    fake = ctypes.c_void_p(0x3000)
    assert L.empc_solve_static(ctypes.byref(c), ctypes.byref(g), fake, 0, 2, fake, fake, None) == 1
    assert L.empc_solve_static(ctypes.byref(c), ctypes.byref(g), None, 0, 1, fake, fake, None) == 1
    assert L.empc_solve_static(None, ctypes.byref(g), fake, 0, 1, fake, fake, None) == 1
    big = E.EmpcGA.from_buffer_copy(g)
    big.pop = 1 << 22  # 30 parameters x 2^22 candidates x 2 buffers x 4 B > 64 MiB
    assert L.empc_workspace_bytes(ctypes.byref(c), ctypes.byref(big)) > (64 << 20)
    assert L.empc_solve_static(ctypes.byref(c), ctypes.byref(big), fake, 0, 1, fake, fake,
                               None) == 3
    assert "static" in L.empc_last_error().decode()


def test_qp_validation(E):
    # the convex path takes linear problems without the box penalty, at most
    # 1024 knot parameters, and checks its workspace and iteration limit
    L = E.lib()
    fake = ctypes.c_void_p(0x5000)
    c = _problem(E)
    nb = L.empc_qp_workspace_bytes(ctypes.byref(c))
    assert nb >= 8 * (c.T * c.n * c.p * c.m + (c.p * c.m) ** 2)
    info = ctypes.c_void_p(0x6000)
    assert L.empc_qp_solve(ctypes.byref(c), fake, fake, fake, fake, nb, 0, fake, fake, info,
                           None) == 1
    assert L.empc_qp_solve(ctypes.byref(c), fake, fake, fake, fake, nb - 1, 10, fake, fake, info,
                           None) == 4
    assert L.empc_qp_form(ctypes.byref(c), fake, fake, nb, None, fake, fake, None) == 1
    boxed = _problem(E, qb=fake, x_min=fake, x_max=fake)
    assert L.empc_qp_workspace_bytes(ctypes.byref(boxed)) == 0
    assert L.empc_qp_form(ctypes.byref(boxed), fake, fake, nb, fake, fake, fake, None) == 3
    big = _problem(E, m=40, T=40, p=30)
    assert L.empc_qp_workspace_bytes(ctypes.byref(big)) == 0


def test_nlink_validation(E):
    # the N-link robot's calls check the robot and the step on the host
    L = E.lib()
    fake = ctypes.c_void_p(0x4000)
    R = E.binding.EmpcNLink()
    R.links, R.dtype, R.mass, R.length, R.damping = 3, 1, fake, fake, 0.01
    assert L.empc_nlink_step(ctypes.byref(R), 0.01, 0, fake, fake, fake, None) == 1
    assert L.empc_nlink_step(ctypes.byref(R), 0.0, 1, fake, fake, fake, None) == 1
    assert L.empc_nlink_linearize(ctypes.byref(R), float("nan"), fake, fake, fake, fake, fake,
                                  None) == 1
    assert L.empc_nlink_linearize(ctypes.byref(R), 0.01, fake, fake, None, fake, fake, None) == 1
    R.links = 17
    assert L.empc_nlink_linearize(ctypes.byref(R), 0.01, fake, fake, fake, fake, fake, None) == 3
    R.links = 0
    assert L.empc_nlink_step(ctypes.byref(R), 0.01, 1, fake, fake, fake, None) == 1
    R.links, R.dtype = 3, 5
    assert L.empc_nlink_step(ctypes.byref(R), 0.01, 1, fake, fake, fake, None) == 1
    assert L.empc_nlink_step(None, 0.01, 1, fake, fake, fake, None) == 1


def test_autotune_table_validation(E):
    # recording choices by hand is a host operation: bad codes and shapes are
    # refused, good ones recorded, and the table cleared
    L = E.lib()
    c = _problem(E)
    g = E.EmpcGA()
    g.pop, g.n_elite, g.generations, g.elitism, g.sigma, g.seed = 100, 10, 2, 1, 0.1, 0
    assert L.empc_autotune(ctypes.byref(c), ctypes.byref(g), 0, 0, None, None) == 1
    assert L.empc_autotune_set(ctypes.byref(c), ctypes.byref(g), 9, 0) == 1
    assert L.empc_autotune_set(ctypes.byref(c), ctypes.byref(g), 11, 0) == 1   # chain code
    assert L.empc_autotune_set(ctypes.byref(c), ctypes.byref(g), 1, 3) == 1
    assert L.empc_autotune_set(ctypes.byref(c), ctypes.byref(g), 4, 0) == 3    # n = 4: no split
    big = _problem(E, n=20)
    assert L.empc_autotune_set(ctypes.byref(big), ctypes.byref(g), 5, 0) == 3  # VALU: n <= 16
    assert L.empc_autotune_set(ctypes.byref(c), ctypes.byref(g), 5, 2) == 0
    assert L.empc_autotune_reset() == 0


def test_generation_validation(E):
    c = _problem(E)
    g = E.EmpcGA()
    g.pop, g.n_elite, g.generations, g.elitism, g.sigma, g.seed = 64, 8, 1, 1, 0.1, 0
    L = E.lib()
    fake = ctypes.c_void_p(0x10000)
    # warm start without elite_idx
    assert L.empc_generation(ctypes.byref(c), ctypes.byref(g), fake, 64, fake,
                             ctypes.c_void_p(0x900000), 64, None, None, 0, 0, None) == 1
    # overlapping in / out populations
    assert L.empc_generation(ctypes.byref(c), ctypes.byref(g), fake, 64, fake, fake, 64,
                             fake, None, 0, 0, None) == 1
    # ld_out below pop
    assert L.empc_generation(ctypes.byref(c), ctypes.byref(g), None, 0, None, fake, 63,
                             None, None, 0, 0, None) == 1


def test_grad_limits(E):
    c = _problem(E, n=70, m=10)
    fake = ctypes.c_void_p(0x1000)
    assert E.lib().empc_grad(ctypes.byref(c), fake, fake, 4, 4, fake, None, None) == 3
    c = _problem(E)
    assert E.lib().empc_refine(ctypes.byref(c), fake, fake, 4, 4, fake, -1.0, 5, None) == 1


def test_profile_session_errors(E):
    L = E.lib()
    assert L.empc_profile_end(None, None) == 1
    assert L.empc_profile_begin(0) == 1


def test_status_strings(E):
    for s in range(5):
        assert E.lib().empc_status_str(s).decode()


def test_bench_refuses_several_gpus():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


# ---------------------------------------------------------------------------
# the binding's own checks of torch tensors (dtype, size, contiguity): the
# library sees raw pointers only, so these are caught before any call


def _torch_problem(E, dtype=0, n=4, m=2, p=3):
    c = _problem(E, n=n, m=m, p=p, dtype=dtype)
    return c


@pytest.mark.parametrize("case", ["dtype", "knots_short", "x0_short", "cost_short",
                                  "noncontig", "cpu"])
def test_binding_rejects_bad_tensors(E, case):
    import torch

    c = _torch_problem(E, dtype=1)  # FP64 problem, n = 4, m = 2, p = 3
    f64 = torch.float64
    x0 = torch.zeros(4, dtype=f64)
    knots = torch.zeros(6, 10, dtype=f64)
    cost = torch.zeros(10, dtype=f64)
    if case == "dtype":
        knots = knots.float()  # 4-byte elements where the kernels read 8
        msg = "dtype"
    elif case == "knots_short":
        knots = torch.zeros(5, 10, dtype=f64)  # fewer than p*m rows
        msg = "knots holds"
    elif case == "x0_short":
        x0 = torch.zeros(3, dtype=f64)
        msg = "x0 holds"
    elif case == "cost_short":
        cost = torch.zeros(9, dtype=f64)
        msg = "cost holds"
    elif case == "noncontig":
        knots = torch.zeros(10, 6, dtype=f64).t()
        msg = "contiguous"
    else:
        msg = "GPU tensor"  # right sizes, but host memory
    with pytest.raises(ValueError, match=msg):
        E.empc_rollout_cost(c, x0, knots, 10, 10, cost)


def test_binding_rejects_bad_solve_and_plant_tensors(E):
    import torch

    c = _torch_problem(E, dtype=0)  # FP32, n = 4, m = 2
    g = E.EmpcGA()
    g.pop, g.n_elite, g.generations, g.sigma = 32, 4, 1, 0.1
    ws = torch.zeros(64, dtype=torch.uint8)
    x0 = torch.zeros(4)
    u = torch.zeros(2)
    b = torch.zeros(1)
    with pytest.raises(ValueError, match="u_star holds"):
        E.empc_solve(c, g, ws, x0, 0, torch.zeros(1), b)
    with pytest.raises(ValueError, match="dtype"):
        E.empc_solve(c, g, ws, x0.double(), 0, u, b)
    with pytest.raises(ValueError, match="workspace has dtype"):
        E.empc_solve(c, g, torch.zeros(16), x0, 0, u, b)
    with pytest.raises(ValueError, match="x_next holds"):
        E.empc_plant_step(c, x0, u, None, torch.zeros(2))
    with pytest.raises(ValueError, match="noise holds"):
        E.empc_plant_step(c, x0, u, torch.zeros(3), torch.zeros(4))
    with pytest.raises(ValueError, match="dJ holds"):
        E.empc_grad(c, x0, torch.zeros(6, 5), 5, 5, torch.zeros(6, 4), None)
    with pytest.raises(ValueError, match="elite_idx has dtype"):
        E.empc_generation(c, g, torch.zeros(6, 32), 32, torch.zeros(32), torch.zeros(6, 32), 32,
                          torch.zeros(4, dtype=torch.int32), None, 0, 1)


@pytest.mark.parametrize("cname,pyname", [("empc_problem", "EmpcProblem"), ("empc_ga", "EmpcGA"),
                                          ("empc_nlink", "EmpcNLink")])
def test_binding_structs_match_the_header(cname, pyname, tmp_path):
    """Every field of the ctypes mirror sits at the offset the C compiler
    gives the header's struct, and the sizes agree."""
    import shutil
    import subprocess

    from paper_2001_04931_amd import binding

    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    py = getattr(binding, pyname)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "empc.h"', "int main(void) {",
             '  printf("size %%zu\\n", sizeof(%s));' % cname]
    for f, _ in py._fields_:
        lines.append('  printf("%s %%zu\\n", offsetof(%s, %s));' % (f, cname, f))
    lines.append("  return 0;\n}\n")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(py)
    for f, _ in py._fields_:
        assert int(out[f]) == getattr(py, f).offset, f
