"""Seeded synthetic inputs for EMPC, shared by the oracle tests and the GPU path.

This module holds no EMPC arithmetic: no knot interpolation, no rollout, no
cost, no selection, no random draws of the evolutionary algorithm.  It only
draws problem instances (model parameters, initial states, knot populations,
process noise) from numpy's seeded PCG64 generator and turns the continuous
linear chain into the discrete matrices A_d, B_d that the method takes as
input (eq. 2 of the paper lets any discretisation feed the method; this
module uses zero-order hold).

Instances follow the synthetic workloads of the benchmark configurations:
 - linear mass-spring-damper chain: wall-(k1,c1)-m1-(k2,c2)-m2-...-md, one
   force input per mass, state [positions; velocities], masses U[0.5,2] kg,
   stiffness U[10,100] N/m, damping U[0.5,5] N s/m, ZOH at dt = 0.01 s;
 - nonlinear planar pendulum chain: joint stiffness U[5,50], joint damping
   U[0.1,1], link mass U[0.2,1] kg, link length U[0.1,0.3] m, gravity 9.81,
   semi-implicit Euler at dt = 0.005 s (the integration itself belongs to the
   method and is implemented separately by each side);
 - cost Q = diag(1 on positions/angles, 0.1 on velocities), R = 0.01 I,
   goal 0, |u| <= 1, x0 ~ N(0, 0.5^2).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg

LINEAR = 0
PENDULUM_CHAIN = 1

GRAVITY = 9.81


@dataclasses.dataclass
class Problem:
    """One MPC problem instance (host arrays, float64).

    n, m: state / input counts; T: horizon steps; p: knots per input.
    For LINEAR, Ad (n,n), Bd (n,m), wd (n,) are the discrete model.
    For PENDULUM_CHAIN (d = m joints, n = 2d), the raw physical parameters
    stiffness, damping, mass, length (each (d,)) plus gravity and dt.
    q, r, qf: diagonal state / input / terminal weights; x_goal, u_goal;
    u_min, u_max: input bounds.
    """

    model: int
    n: int
    m: int
    T: int
    p: int
    q: np.ndarray
    r: np.ndarray
    qf: np.ndarray
    x_goal: np.ndarray
    u_goal: np.ndarray
    u_min: np.ndarray
    u_max: np.ndarray
    Ad: Optional[np.ndarray] = None
    Bd: Optional[np.ndarray] = None
    wd: Optional[np.ndarray] = None
    stiffness: Optional[np.ndarray] = None
    damping: Optional[np.ndarray] = None
    mass: Optional[np.ndarray] = None
    length: Optional[np.ndarray] = None
    # state box as a soft constraint (None: none): qb_i times the squared
    # distance of x_i to [x_min_i, x_max_i], on every state x_1..x_T
    x_min: Optional[np.ndarray] = None
    x_max: Optional[np.ndarray] = None
    qb: Optional[np.ndarray] = None
    # non-smooth terms (None: none): sb_i charged for every state x_1..x_T
    # outside [x_min_i, x_max_i] (needs the box, qb may be zeros); chain
    # joint limits [q_min_j, q_max_j] with impacts of the given restitution
    sb: Optional[np.ndarray] = None
    q_min: Optional[np.ndarray] = None
    q_max: Optional[np.ndarray] = None
    restitution: float = 0.0
    # chain dry friction (None: none): sliding torque fric_c, breakaway
    # torque fric_s >= fric_c per joint (stick-slip)
    fric_c: Optional[np.ndarray] = None
    fric_s: Optional[np.ndarray] = None
    # full symmetric weights of the linear model (None: the diagonals q, r, qf)
    Q: Optional[np.ndarray] = None
    R: Optional[np.ndarray] = None
    Qf: Optional[np.ndarray] = None
    gravity: float = GRAVITY
    dt: float = 0.0

    def cast(self, dtype) -> "Problem":
        """Copy whose float arrays are rounded to `dtype` and stored as float64.

        Feeding the rounded values to both the FP64 oracle and an FP32 kernel
        makes the two see identical inputs.
        """
        out = dataclasses.replace(self)
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            if isinstance(v, np.ndarray):
                setattr(out, f.name, v.astype(dtype).astype(np.float64))
        if dtype == np.float32:
            out.gravity = float(np.float32(self.gravity))
            out.dt = float(np.float32(self.dt))
            out.restitution = float(np.float32(self.restitution))
        return out


@dataclasses.dataclass
class GA:
    """Evolutionary-algorithm tunables (numSims, numParents, sigma_noise)."""

    pop: int
    n_elite: int
    generations: int
    sigma: float
    seed: int
    elitism: bool = True
    # warm-start and exploration variants (defaults: the plain method)
    shift: bool = False       # move the carried parents one step later per tick
    sigma_min: float = 0.0    # noise at the goal
    sigma_dist: float = 0.0   # > 0: noise grows linearly up to sigma at this distance


def zoh(A: np.ndarray, B: np.ndarray, dt: float):
    """Zero-order-hold discretisation via the block matrix exponential
    expm([[A, B], [0, 0]] dt) = [[A_d, B_d], [0, I]] (Van Loan)."""
    n, m = B.shape
    M = np.zeros((n + m, n + m))
    M[:n, :n] = A
    M[:n, n:] = B
    E = scipy.linalg.expm(M * dt)
    return E[:n, :n].copy(), E[:n, n:].copy()


def chain_continuous(masses, stiff, damp):
    """Continuous (A, B) of a wall-anchored mass-spring-damper chain."""
    d = len(masses)
    K = np.zeros((d, d))
    C = np.zeros((d, d))
    for i in range(d):
        # spring i joins mass i-1 (or the wall) and mass i
        K[i, i] += stiff[i]
        C[i, i] += damp[i]
        if i > 0:
            K[i - 1, i - 1] += stiff[i]
            K[i - 1, i] -= stiff[i]
            K[i, i - 1] -= stiff[i]
            C[i - 1, i - 1] += damp[i]
            C[i - 1, i] -= damp[i]
            C[i, i - 1] -= damp[i]
    Minv = np.diag(1.0 / masses)
    A = np.zeros((2 * d, 2 * d))
    A[:d, d:] = np.eye(d)
    A[d:, :d] = -Minv @ K
    A[d:, d:] = -Minv @ C
    B = np.zeros((2 * d, d))
    B[d:, :] = Minv
    return A, B


def _cost_and_bounds(d: int, n: int):
    q = np.concatenate([np.full(d, 1.0), np.full(n - d, 0.1)])
    r = np.full(d, 0.01)
    return dict(q=q, r=r, qf=np.zeros(n), x_goal=np.zeros(n), u_goal=np.zeros(d),
                u_min=np.full(d, -1.0), u_max=np.full(d, 1.0))


def linear_chain(d: int, T: int, p: int, seed: int, dt: float = 0.01) -> Problem:
    """d-DoF linear chain (n = 2d states, m = d inputs), ZOH at dt."""
    rng = np.random.default_rng([seed, 2, d])
    masses = rng.uniform(0.5, 2.0, d)
    stiff = rng.uniform(10.0, 100.0, d)
    damp = rng.uniform(0.5, 5.0, d)
    A, B = chain_continuous(masses, stiff, damp)
    Ad, Bd = zoh(A, B, dt)
    n = 2 * d
    return Problem(model=LINEAR, n=n, m=d, T=T, p=p, Ad=Ad, Bd=Bd, wd=np.zeros(n),
                   dt=dt, **_cost_and_bounds(d, n))


def pendulum_chain(d: int, T: int, p: int, seed: int, dt: float = 0.005) -> Problem:
    """d-joint planar pendulum chain hanging under gravity (n = 2d, m = d)."""
    rng = np.random.default_rng([seed, 3, d])
    stiff = rng.uniform(5.0, 50.0, d)
    damp = rng.uniform(0.1, 1.0, d)
    mass = rng.uniform(0.2, 1.0, d)
    length = rng.uniform(0.1, 0.3, d)
    n = 2 * d
    return Problem(model=PENDULUM_CHAIN, n=n, m=d, T=T, p=p, stiffness=stiff, damping=damp,
                   mass=mass, length=length, gravity=GRAVITY, dt=dt, **_cost_and_bounds(d, n))


def draw_x0(n: int, seed: int, count: Optional[int] = None, scale: float = 0.5) -> np.ndarray:
    """Initial state(s) x0 ~ N(0, scale^2)."""
    rng = np.random.default_rng([seed, 4, n])
    shape = (n,) if count is None else (count, n)
    return rng.normal(0.0, scale, shape)


def draw_knots(prob: Problem, ncand: int, seed: int, ld: Optional[int] = None,
               spread: float = 1.0) -> np.ndarray:
    """Candidate knots, SoA layout [p*m][ld]: entry (knot*m + i, cand).

    Values are uniform in [u_min, u_max] scaled by `spread` about the box
    centre (spread > 1 gives out-of-bounds knots for edge-case tests)."""
    ld = ncand if ld is None else ld
    rng = np.random.default_rng([seed, 5, prob.p, prob.m, ncand])
    pm = prob.p * prob.m
    lo = np.tile(prob.u_min, prob.p)[:, None]
    hi = np.tile(prob.u_max, prob.p)[:, None]
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo) * spread
    out = np.zeros((pm, ld))
    out[:, :ncand] = mid + half * rng.uniform(-1.0, 1.0, (pm, ncand))
    return out


def process_noise(n: int, ticks: int, seed: int, std: float = 1e-3) -> np.ndarray:
    """Closed-loop plant noise, (ticks, n) ~ N(0, std^2)."""
    rng = np.random.default_rng([seed, 6, n])
    return rng.normal(0.0, std, (ticks, n))


# ---------------------------------------------------------------------------
# Benchmark configurations (synthetic; no dataset is involved).

def config_c1(seed: int = 0):
    """Plain EMPC, FP64: 2-DoF linear chain, T=20, p=5, pop 256, top-16,
    10 generations, sigma 0.1."""
    prob = linear_chain(2, 20, 5, seed)
    return prob, GA(pop=256, n_elite=16, generations=10, sigma=0.1, seed=seed)


def config_c2(seed: int = 0):
    """Plain EMPC, FP32: 14-DoF linear chain, T=50, p=10, pop 4096, top-64,
    20 generations, 100 closed-loop ticks with N(0, 1e-3^2) process noise."""
    prob = linear_chain(14, 50, 10, seed)
    return prob, GA(pop=4096, n_elite=64, generations=20, sigma=0.1, seed=seed)


def config_c3(seed: int = 0):
    """Plain EMPC, FP32: 36-joint nonlinear pendulum chain, dt=0.005, T=100,
    p=10, pop 16384, top-64, 30 generations."""
    prob = pendulum_chain(36, 100, 10, seed)
    return prob, GA(pop=16384, n_elite=64, generations=30, sigma=0.1, seed=seed)


# ---------------------------------------------------------------------------
# The N-link planar robot of the paper's Sec. IV-F setup and Sec. VI-A EMPC
# experiments: every link 1 kg at 0.25 m, viscous damping 0.01, torques
# within +-2 N m, control at 100 Hz (dt = 0.01 s), horizon 100, 3 knots,
# from rest at an initial position to rest at a goal position, both drawn
# uniformly (here each joint angle in [-1, 1] rad).  The linear model of each
# tick comes from relinearizing the robot at its current state (the method's
# own step, done by each side), so the Problem carries placeholder matrices.

@dataclasses.dataclass
class NLink:
    mass: np.ndarray
    length: np.ndarray
    damping: float


def nlink_robot(N: int) -> NLink:
    return NLink(mass=np.ones(N), length=np.full(N, 0.25), damping=0.01)


def nlink_problem(N: int, T: int = 100, p: int = 3, x_goal=None) -> Problem:
    """Linear-model MPC problem of an N-link robot (n = 2N, m = N); A_d, B_d,
    w_d are placeholders that the relinearization overwrites."""
    n = 2 * N
    cb = _cost_and_bounds(N, n)
    cb["u_min"], cb["u_max"] = np.full(N, -2.0), np.full(N, 2.0)
    if x_goal is not None:
        cb["x_goal"] = np.asarray(x_goal, dtype=np.float64)
    return Problem(model=LINEAR, n=n, m=N, T=T, p=p, Ad=np.eye(n), Bd=np.zeros((n, N)),
                   wd=np.zeros(n), dt=0.01, **cb)


def nlink_start_goal(N: int, seed: int):
    """(x0, x_goal): rest at joint angles ~ U[-1, 1] rad, both."""
    rng = np.random.default_rng([seed, 8, N])
    q0, qg = rng.uniform(-1.0, 1.0, N), rng.uniform(-1.0, 1.0, N)
    return (np.concatenate([q0, np.zeros(N)]), np.concatenate([qg, np.zeros(N)]))


def config_nlink(N: int, seed: int = 0, generations: int = 1):
    """N-link robot EMPC at 100 Hz: T = 100, 3 knots, pop 1024, top-32,
    sigma 0.2 (a tenth of the torque range), `generations` per tick (the
    paper runs 1 and 3)."""
    x0, xg = nlink_start_goal(N, seed)
    prob = nlink_problem(N, 100, 3, xg)
    return (nlink_robot(N), prob, x0,
            GA(pop=1024, n_elite=32, generations=generations, sigma=0.2, seed=seed))


def config_nonsmooth_linear(seed: int = 0):
    """Full weights and a settling band on the 7-DoF linear chain (n = 14,
    m = 7), T = 50, p = 10, pop 4096, top-64, 20 generations: Q charges the
    spring extensions (x_i - x_{i-1})^2 of the positions (plus 0.5 I) and
    0.1 on the velocities, Qf = 5 Q, R = 0.01 (I + tridiagonal 1/2), and a
    charge of 1 per step for every position more than 0.05 from its goal."""
    d = 7
    prob = linear_chain(d, 50, 10, seed)
    n = prob.n
    D = np.eye(d) - np.eye(d, k=-1)
    Q = np.zeros((n, n))
    Q[:d, :d] = 0.5 * np.eye(d) + D.T @ D
    Q[d:, d:] = 0.1 * np.eye(d)
    prob.Q, prob.Qf = Q, 5.0 * Q
    prob.R = 0.01 * (np.eye(d) + 0.5 * (np.eye(d, k=1) + np.eye(d, k=-1)))
    band = np.concatenate([np.full(d, 0.05), np.full(d, np.inf)])
    prob.x_min, prob.x_max = prob.x_goal - band, prob.x_goal + band
    prob.qb = np.zeros(n)
    prob.sb = np.concatenate([np.ones(d), np.zeros(d)])
    return prob, GA(pop=4096, n_elite=64, generations=20, sigma=0.1, seed=seed)


def config_nonsmooth_chain(seed: int = 0):
    """The 36-joint pendulum chain of the C3 configuration with joint limits
    of +-0.6 rad (impacts with restitution 0.5), dry friction on every joint
    (sliding 0.02, breakaway 0.05 N m) and a charge of 0.1 per step for
    every joint angle more than 0.05 rad from its goal."""
    prob, ga = config_c3(seed)
    d = prob.m
    prob.q_min, prob.q_max, prob.restitution = np.full(d, -0.6), np.full(d, 0.6), 0.5
    prob.fric_c, prob.fric_s = np.full(d, 0.02), np.full(d, 0.05)
    band = np.concatenate([np.full(d, 0.05), np.full(d, np.inf)])
    prob.x_min, prob.x_max = prob.x_goal - band, prob.x_goal + band
    prob.qb = np.zeros(prob.n)
    prob.sb = np.concatenate([np.full(d, 0.1), np.zeros(d)])
    return prob, ga


def start_inside_limits(prob, x0):
    """x0 with the joint angles clipped into the problem's joint limits."""
    x0 = np.array(x0, dtype=np.float64)
    if prob.q_min is not None:
        x0[:prob.m] = np.clip(x0[:prob.m], prob.q_min, prob.q_max)
    return x0


C5_DOFS = (2, 7, 14, 21, 36)


def config_c5(nprob: int = 512, seed: int = 0):
    """Batching: nprob independent problems, DoF ~ U{2,7,14,21,36}, linear or
    pendulum chain ~ Bernoulli(1/2), T ~ U{20..100}, p ~ U{5..10}; pop 1024,
    top-32, 1 generation per tick."""
    rng = np.random.default_rng([seed, 7, nprob])
    probs = []
    for i in range(nprob):
        d = int(rng.choice(C5_DOFS))
        kind = int(rng.integers(0, 2))
        T = int(rng.integers(20, 101))
        p = int(rng.integers(5, 11))
        if kind == LINEAR:
            probs.append(linear_chain(d, T, p, seed * 100003 + i))
        else:
            probs.append(pendulum_chain(d, T, p, seed * 100003 + i))
    return probs, GA(pop=1024, n_elite=32, generations=1, sigma=0.1, seed=seed)
