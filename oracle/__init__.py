"""Python access to the FP64 EMPC oracle (C, single-threaded).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is shared
with, or imported by, the HIP library or its binding.

The oracle follows the paper (Hyatt, Williams, Killpack 2020): eq. 2 for the
linear step, eq. 3 for the cost, Sec. IV-C for the knot interpolation,
Sec. V / Alg. 1 for the evolutionary step.  See empc_oracle.h for how each
function is pinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "empc_oracle.c")
_SRC_NLINK = os.path.join(_HERE, "nlink_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC,
                        _SRC_NLINK, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _OrProblem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("n", ctypes.c_int), ("m", ctypes.c_int),
                ("T", ctypes.c_int), ("p", ctypes.c_int),
                ("Ad", _dp), ("Bd", _dp), ("wd", _dp),
                ("stiff", _dp), ("damp", _dp), ("mass", _dp), ("len", _dp),
                ("gravity", ctypes.c_double), ("dt", ctypes.c_double),
                ("q", _dp), ("r", _dp), ("qf", _dp), ("x_goal", _dp), ("u_goal", _dp),
                ("u_min", _dp), ("u_max", _dp), ("x_min", _dp), ("x_max", _dp), ("qb", _dp),
                ("sb", _dp), ("q_min", _dp), ("q_max", _dp), ("restitution", ctypes.c_double),
                ("Q", _dp), ("R", _dp), ("Qf", _dp), ("fric_c", _dp), ("fric_s", _dp)]


class _OrGA(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int), ("n_elite", ctypes.c_int),
                ("generations", ctypes.c_int), ("elitism", ctypes.c_int),
                ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("shift", ctypes.c_int), ("sigma_min", ctypes.c_double),
                ("sigma_dist", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.or_knot_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      _dp]
        L.or_step.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, _dp]
        L.or_plant_step.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, _dp, _dp]
        L.or_rollout_one.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, ctypes.c_int64,
                                     ctypes.c_int64, _dp]
        L.or_rollout_one.restype = ctypes.c_double
        L.or_rollout_cost.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, ctypes.c_int64,
                                      ctypes.c_int64, _dp]
        L.or_select.argtypes = [_dp, ctypes.c_int64, ctypes.c_int, _i64p, _i64p]
        L.or_next_population.argtypes = [ctypes.POINTER(_OrProblem), ctypes.POINTER(_OrGA), _dp,
                                         ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, _dp,
                                         ctypes.c_int64]
        L.or_solve.argtypes = [ctypes.POINTER(_OrProblem), ctypes.POINTER(_OrGA), _dp,
                               ctypes.POINTER(ctypes.c_int), _dp, ctypes.c_uint32, _dp, _dp, _dp,
                               _dp, _dp, _i64p, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.or_solve.restype = ctypes.c_int
        L.or_shift_knots.argtypes = [ctypes.POINTER(_OrProblem), _dp, ctypes.c_int]
        L.or_sigma_at.argtypes = [ctypes.POINTER(_OrProblem), ctypes.POINTER(_OrGA), _dp]
        L.or_sigma_at.restype = ctypes.c_double
        L.or_grad.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, ctypes.c_int64,
                              ctypes.c_int64, _dp, _dp]
        L.or_refine.argtypes = [ctypes.POINTER(_OrProblem), _dp, _dp, ctypes.c_int64,
                                ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_int]
        L.or_nlink_mass_matrix.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_nlink_kinetic.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        L.or_nlink_kinetic.restype = ctypes.c_double
        L.or_nlink_deriv.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _dp, _dp]
        L.or_nlink_jacobian.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _dp, _dp,
                                        _dp, _dp]
        L.or_nlink_rk4.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _dp,
                                   ctypes.c_double, ctypes.c_int, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class OracleProblem:
    """Holds float64 copies of a workloads.Problem and the C struct over them."""

    def __init__(self, prob):
        self.prob = prob
        self._keep = {}
        s = _OrProblem()
        s.model, s.n, s.m, s.T, s.p = prob.model, prob.n, prob.m, prob.T, prob.p
        for name, cname in (("Ad", "Ad"), ("Bd", "Bd"), ("wd", "wd"), ("stiffness", "stiff"),
                            ("damping", "damp"), ("mass", "mass"), ("length", "len"),
                            ("q", "q"), ("r", "r"), ("qf", "qf"), ("x_goal", "x_goal"),
                            ("u_goal", "u_goal"), ("u_min", "u_min"), ("u_max", "u_max"),
                            ("x_min", "x_min"), ("x_max", "x_max"), ("qb", "qb"),
                            ("sb", "sb"), ("q_min", "q_min"), ("q_max", "q_max"),
                            ("Q", "Q"), ("R", "R"), ("Qf", "Qf"), ("fric_c", "fric_c"),
                            ("fric_s", "fric_s")):
            v = getattr(prob, name, None)
            if v is not None:
                v = _f64(v)
                self._keep[name] = v
                setattr(s, cname, _ptr(v))
        s.gravity = float(prob.gravity)
        s.dt = float(prob.dt)
        s.restitution = float(getattr(prob, "restitution", 0.0) or 0.0)
        self.s = s

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _ga_struct(ga, pop=None):
    g = _OrGA()
    g.pop = ga.pop if pop is None else pop
    g.n_elite, g.generations = ga.n_elite, ga.generations
    g.elitism = 1 if ga.elitism else 0
    g.sigma = float(ga.sigma)
    g.seed = int(ga.seed)
    g.shift = 1 if getattr(ga, "shift", False) else 0
    g.sigma_min = float(getattr(ga, "sigma_min", 0.0))
    g.sigma_dist = float(getattr(ga, "sigma_dist", 0.0))
    return g


def shift_knots(prob, rows):
    """Parent rows [k][p*m] moved one control step later (a copy)."""
    P = OracleProblem(prob)
    out = np.array(rows, dtype=np.float64, order="C", copy=True)
    lib().or_shift_knots(P.ref, _ptr(out), out.shape[0])
    return out


def sigma_at(prob, ga, x0):
    """Mutation noise of a solve from state x0."""
    P = OracleProblem(prob)
    G = _ga_struct(ga)
    x0 = _f64(x0)
    return float(lib().or_sigma_at(P.ref, ctypes.byref(G), _ptr(x0)))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def knot_weights(T, p, k):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    lib().or_knot_weights(T, p, k, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def step(prob, x, u, noise=None):
    P = OracleProblem(prob)
    x, u = _f64(x), _f64(u)
    out = np.zeros(prob.n)
    nz = None if noise is None else _f64(noise)
    lib().or_plant_step(P.ref, _ptr(x), _ptr(u), _ptr(nz), _ptr(out))
    return out


def rollout_one(prob, x0, knots, cand=0):
    """Cost of one candidate and its trajectory x_0..x_T, shape (T+1, n)."""
    P = OracleProblem(prob)
    x0, knots = _f64(x0), _f64(knots)
    ld = knots.shape[1]
    traj = np.zeros((prob.T + 1, prob.n))
    J = lib().or_rollout_one(P.ref, _ptr(x0), _ptr(knots), ld, cand, _ptr(traj))
    return J, traj


def rollout_cost(prob, x0, knots, ncand=None):
    """Costs of candidates 0..ncand-1; knots SoA [p*m][ld]."""
    P = OracleProblem(prob)
    x0, knots = _f64(x0), _f64(knots)
    ld = knots.shape[1]
    ncand = ld if ncand is None else ncand
    cost = np.zeros(ncand)
    lib().or_rollout_cost(P.ref, _ptr(x0), _ptr(knots), ncand, ld, _ptr(cost))
    return cost


def select(cost, k):
    """(elite indices ascending, best index) of the k lowest (J, index)."""
    cost = _f64(cost)
    idx = np.zeros(k, dtype=np.int64)
    best = ctypes.c_int64()
    lib().or_select(_ptr(cost), cost.shape[0], k, idx.ctypes.data_as(_i64p), ctypes.byref(best))
    return idx, best.value


def next_population(prob, ga, elite_knots, cold, tick, gen, pop=None):
    """Next population [p*m][pop] from elite rows [k][p*m]."""
    P = OracleProblem(prob)
    G = _ga_struct(ga, pop)
    pm = prob.p * prob.m
    ek = _f64(elite_knots if elite_knots is not None else np.zeros((ga.n_elite, pm)))
    out = np.zeros((pm, G.pop))
    lib().or_next_population(P.ref, ctypes.byref(G), _ptr(ek), 1 if cold else 0, tick, gen,
                             _ptr(out), G.pop)
    return out


def _smooth_diagonal(prob):
    """The adjoint covers diagonal weights and smooth dynamics only: full Q,
    R, Qf, joint limits with impacts and dry friction have no gradient here
    (the step charge sb has derivative zero off the box faces and is
    allowed)."""
    for name in ("Q", "R", "Qf", "q_min", "q_max", "fric_c", "fric_s"):
        if getattr(prob, name, None) is not None:
            raise ValueError("the adjoint does not cover %s" % name)


def grad(prob, x0, knots, ncand=None):
    """(dJ/dknots [p*m][ld], cost [ncand]) by the adjoint, full storage."""
    _smooth_diagonal(prob)
    P = OracleProblem(prob)
    x0, knots = _f64(x0), _f64(knots)
    ld = knots.shape[1]
    ncand = ld if ncand is None else ncand
    dJ = np.zeros_like(knots)
    cost = np.zeros(ncand)
    lib().or_grad(P.ref, _ptr(x0), _ptr(knots), ncand, ld, _ptr(dJ), _ptr(cost))
    return dJ, cost


def refine(prob, x0, knots, cost, lr=0.01, steps=5):
    """Adam refinement of candidates in place of copies; returns (knots, cost)."""
    _smooth_diagonal(prob)
    P = OracleProblem(prob)
    x0 = _f64(x0)
    knots = _f64(knots).copy()
    cost = _f64(cost).copy()
    lib().or_refine(P.ref, _ptr(x0), _ptr(knots), knots.shape[1], knots.shape[1], _ptr(cost),
                    lr, steps)
    return knots, cost


class Solver:
    """Warm-started EMPC controller state for one problem (oracle side)."""

    def __init__(self, prob, ga, refine=False, lr=0.01, adam_steps=5):
        if refine:
            _smooth_diagonal(prob)
        self.prob, self.ga = prob, ga
        self.P = OracleProblem(prob)
        self.G = _ga_struct(ga)
        pm = prob.p * prob.m
        self.elite_knots = np.zeros((ga.n_elite, pm))
        self.has_elites = ctypes.c_int(0)
        self.knots_ws = np.zeros((pm, ga.pop))
        self.cost_ws = np.zeros(ga.pop)
        self.idx_ws = np.zeros(ga.n_elite, dtype=np.int64)
        self.refine, self.lr, self.adam_steps = refine, lr, adam_steps
        self.best_slot = 0

    def solve(self, x0, tick):
        """Returns (u*, best cost, per-generation best costs)."""
        x0 = _f64(x0)
        u = np.zeros(self.prob.m)
        best = ctypes.c_double()
        gen_best = np.zeros(self.ga.generations)
        self.best_slot = lib().or_solve(self.P.ref, ctypes.byref(self.G), _ptr(self.elite_knots),
                                        ctypes.byref(self.has_elites), _ptr(x0), tick, _ptr(u),
                                        ctypes.byref(best), _ptr(gen_best), _ptr(self.knots_ws),
                                        _ptr(self.cost_ws),
                                        self.idx_ws.ctypes.data_as(_i64p),
                                        1 if self.refine else 0, self.lr, self.adam_steps)
        return u, best.value, gen_best


# ---------------------------------------------------------------------------
# N-link planar robot (nlink_oracle.c): point masses at the link ends, plane
# perpendicular to gravity, M(q) qdd + C(q, qd) + b qd = tau.


def _nl_check(rc):
    if rc != 0:
        raise ValueError("N-link oracle: links outside [1, 16] or bad substeps")


def nlink_mass_matrix(mass, length, q, qd=None):
    """(M(q) [N][N], C(q, qd) [N] or None)."""
    mass, length, q = _f64(mass), _f64(length), _f64(q)
    N = mass.shape[0]
    M = np.zeros((N, N))
    C = np.zeros(N) if qd is not None else None
    qd = None if qd is None else _f64(qd)
    _nl_check(lib().or_nlink_mass_matrix(N, _ptr(mass), _ptr(length), _ptr(q), _ptr(M), _ptr(C),
                                         _ptr(qd)))
    return M, C


def nlink_kinetic(mass, length, q, qd):
    mass, length, q, qd = _f64(mass), _f64(length), _f64(q), _f64(qd)
    return float(lib().or_nlink_kinetic(mass.shape[0], _ptr(mass), _ptr(length), _ptr(q),
                                        _ptr(qd)))


def nlink_deriv(mass, length, b, x, tau):
    """State derivative [qd; qdd] of x = [q; qd]."""
    mass, length, x, tau = _f64(mass), _f64(length), _f64(x), _f64(tau)
    f = np.zeros(x.shape[0])
    _nl_check(lib().or_nlink_deriv(mass.shape[0], _ptr(mass), _ptr(length), float(b), _ptr(x),
                                   _ptr(tau), _ptr(f)))
    return f


def nlink_jacobian(mass, length, b, x, tau):
    """(A = df/dx [2N][2N], B = df/dtau [2N][N], f(x, tau)) by the complex step."""
    mass, length, x, tau = _f64(mass), _f64(length), _f64(x), _f64(tau)
    N = mass.shape[0]
    A = np.zeros((2 * N, 2 * N))
    B = np.zeros((2 * N, N))
    f0 = np.zeros(2 * N)
    _nl_check(lib().or_nlink_jacobian(N, _ptr(mass), _ptr(length), float(b), _ptr(x), _ptr(tau),
                                      _ptr(A), _ptr(B), _ptr(f0)))
    return A, B, f0


def nlink_rk4(mass, length, b, x, tau, dt, substeps):
    """The simulated robot over dt: `substeps` RK4 steps, tau held."""
    mass, length, x, tau = _f64(mass), _f64(length), _f64(x), _f64(tau)
    out = np.zeros(x.shape[0])
    _nl_check(lib().or_nlink_rk4(mass.shape[0], _ptr(mass), _ptr(length), float(b), _ptr(x),
                                 _ptr(tau), float(dt), int(substeps), _ptr(out)))
    return out


def nlink_linearize(mass, length, b, x, tau, dt):
    """Discrete affine model (A_d, B_d, w_d) of the robot at (x, tau): the
    exact Jacobians A, B and the offset w = f(x, tau) - A x - B tau of the
    first-order expansion, held over dt by the zero-order hold, i.e. the
    matrix exponential of [[A, B, w], [0, 0, 0]] dt (scipy's expm)."""
    import scipy.linalg

    A, B, f0 = nlink_jacobian(mass, length, b, x, tau)
    n, m = A.shape[0], B.shape[1]
    w = f0 - A @ _f64(x) - B @ _f64(tau)
    Z = np.zeros((n + m + 1, n + m + 1))
    Z[:n, :n], Z[:n, n:n + m], Z[:n, n + m] = A, B, w
    E = scipy.linalg.expm(Z * dt)
    return E[:n, :n].copy(), E[:n, n:n + m].copy(), E[:n, n + m].copy()
