"""ctypes binding of libempc.so (include/empc.h), argument marshalling only.

Every function named like the C entry point takes torch tensors that live on
the GPU, passes their device pointers and the current HIP stream to the
library, and raises EmpcError on a non-OK status.  All arithmetic happens in
the library's HIP kernels; there is no host fallback: a missing library is an
error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libempc.so")

EMPC_OK, EMPC_EINVAL, EMPC_EDEVICE, EMPC_EUNSUPPORTED, EMPC_EWORKSPACE = range(5)
EMPC_F32, EMPC_F64 = 0, 1
EMPC_LINEAR, EMPC_PENDULUM_CHAIN = 0, 1

_vp = ctypes.c_void_p


class EmpcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("empc status %d: %s" % (status, message))
        self.status = status


class EmpcProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("T", ctypes.c_int32),
                ("p", ctypes.c_int32), ("dtype", ctypes.c_int32), ("model", ctypes.c_int32),
                ("Ad", _vp), ("Bd", _vp), ("wd", _vp),
                ("stiffness", _vp), ("damping", _vp), ("mass", _vp), ("length", _vp),
                ("gravity", ctypes.c_double), ("dt", ctypes.c_double),
                ("q", _vp), ("r", _vp), ("qf", _vp), ("x_goal", _vp), ("u_goal", _vp),
                ("u_min", _vp), ("u_max", _vp), ("x_min", _vp), ("x_max", _vp), ("qb", _vp),
                ("sb", _vp), ("q_min", _vp), ("q_max", _vp), ("restitution", ctypes.c_double),
                ("Q", _vp), ("R", _vp), ("Qf", _vp), ("fric_c", _vp), ("fric_s", _vp)]


class EmpcGA(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_int32), ("n_elite", ctypes.c_int32),
                ("generations", ctypes.c_int32), ("elitism", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("shift", ctypes.c_int32), ("sigma_min", ctypes.c_double),
                ("sigma_dist", ctypes.c_double)]


class EmpcNLink(ctypes.Structure):
    _fields_ = [("links", ctypes.c_int32), ("dtype", ctypes.c_int32), ("mass", _vp),
                ("length", _vp), ("damping", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libempc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libempc.so is not built (python -m paper_2001_04931_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, G = ctypes.POINTER(EmpcProblem), ctypes.POINTER(EmpcGA)
        i64, u32, sz = ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
        sigs = {
            "empc_status_str": ([ctypes.c_int], ctypes.c_char_p),
            "empc_last_error": ([], ctypes.c_char_p),
            "empc_rollout_cost": ([P, _vp, _vp, i64, i64, _vp, _vp], ctypes.c_int),
            "empc_generation": ([P, G, _vp, i64, _vp, _vp, i64, _vp, _vp, u32, u32, _vp],
                                ctypes.c_int),
            "empc_workspace_bytes": ([P, G], sz),
            "empc_solve": ([P, G, _vp, sz, _vp, u32, _vp, _vp, _vp], ctypes.c_int),
            "empc_solve_refined": ([P, G, _vp, sz, _vp, u32, ctypes.c_double, ctypes.c_int32, _vp,
                                    _vp, _vp], ctypes.c_int),
            "empc_solve_static": ([P, G, _vp, u32, ctypes.c_int32, _vp, _vp, _vp], ctypes.c_int),
            "empc_autotune": ([P, G, ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_float), _vp], ctypes.c_int),
            "empc_autotune_set": ([P, G, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "empc_autotune_reset": ([], ctypes.c_int),
            "empc_grad": ([P, _vp, _vp, i64, i64, _vp, _vp, _vp], ctypes.c_int),
            "empc_refine": ([P, _vp, _vp, i64, i64, _vp, ctypes.c_double, ctypes.c_int32, _vp],
                            ctypes.c_int),
            "empc_plant_step": ([P, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
            "empc_batch_workspace_bytes": ([P, ctypes.c_int32, G], sz),
            "empc_batch_create": ([P, ctypes.c_int32, G, _vp, sz, _vp, _vp, _vp,
                                   ctypes.POINTER(_vp)], ctypes.c_int),
            "empc_solve_batched": ([_vp, _vp], ctypes.c_int),
            "empc_batch_destroy": ([_vp], ctypes.c_int),
            "empc_batch_autotune": ([_vp, ctypes.c_int32, _vp], ctypes.c_int),
            "empc_batch_classes": ([_vp], ctypes.c_int32),
            "empc_batch_class_info": ([_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
                                      ctypes.c_int),
            "empc_batch_class_times": ([_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)],
                                       ctypes.c_int),
            "empc_batch_set_variant": ([_vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "empc_batch_set_mode": ([_vp, ctypes.c_int32], ctypes.c_int),
            "empc_batch_allow_valu": ([_vp, ctypes.c_int32], ctypes.c_int),
            "empc_qp_workspace_bytes": ([P], sz),
            "empc_qp_form": ([P, _vp, _vp, sz, _vp, _vp, _vp, _vp], ctypes.c_int),
            "empc_qp_solve": ([P, _vp, _vp, _vp, _vp, sz, ctypes.c_int32, _vp, _vp, _vp, _vp],
                              ctypes.c_int),
            "empc_nlink_linearize": ([ctypes.POINTER(EmpcNLink), ctypes.c_double, _vp, _vp, _vp,
                                      _vp, _vp, _vp], ctypes.c_int),
            "empc_nlink_step": ([ctypes.POINTER(EmpcNLink), ctypes.c_double, ctypes.c_int32, _vp,
                                 _vp, _vp, _vp], ctypes.c_int),
            "empc_profile_begin": ([ctypes.c_int32], ctypes.c_int),
            "empc_profile_end": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
                                 ctypes.c_int),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return ["empc_status_str", "empc_last_error", "empc_rollout_cost", "empc_generation",
            "empc_workspace_bytes", "empc_solve", "empc_solve_refined", "empc_solve_static",
            "empc_autotune", "empc_autotune_set", "empc_autotune_reset",
            "empc_grad", "empc_refine", "empc_plant_step",
            "empc_batch_workspace_bytes", "empc_batch_create", "empc_solve_batched",
            "empc_batch_destroy", "empc_batch_autotune", "empc_batch_classes",
            "empc_batch_class_info", "empc_batch_class_times", "empc_batch_set_variant",
            "empc_batch_set_mode", "empc_batch_allow_valu",
            "empc_qp_workspace_bytes", "empc_qp_form", "empc_qp_solve",
            "empc_nlink_linearize", "empc_nlink_step", "empc_profile_begin",
            "empc_profile_end"]


def _check(status: int):
    if status != EMPC_OK:
        msg = lib().empc_last_error().decode()
        raise EmpcError(status, msg or lib().empc_status_str(status).decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _cprob(prob):
    return ctypes.byref(prob.c if hasattr(prob, "c") else prob)


def _shape(prob):
    """(torch dtype, n, m, p*m) of a DeviceProblem or a bare EmpcProblem."""
    c = prob.c if hasattr(prob, "c") else prob
    dt = torch.float64 if c.dtype == EMPC_F64 else torch.float32
    return dt, int(c.n), int(c.m), int(c.p) * int(c.m)


def _need(t, dtype, numel, name, optional=False):
    """The library sees only raw pointers, so the binding checks what it
    cannot: a GPU tensor of the problem's dtype, contiguous, holding at least
    `numel` elements (every element the kernels will touch); _ptr then
    rejects host tensors."""
    if t is None:
        if optional or numel <= 0:
            return
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, the problem needs %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))


def _soa_elems(pm, ld, ncand):
    """Elements a [pm][ld] structure-of-arrays block spans for ncand columns."""
    return 0 if ncand <= 0 else (pm - 1) * int(ld) + int(ncand)


def _cga(ga):
    return ctypes.byref(ga.c if hasattr(ga, "c") else ga)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)


def empc_rollout_cost(prob, x0, knots, ncand, ld, cost, stream=None):
    dt, n, m, pm = _shape(prob)
    if ncand > 0 and ld >= ncand:
        _need(x0, dt, n, "x0")
        _need(knots, dt, _soa_elems(pm, ld, ncand), "knots")
        _need(cost, dt, ncand, "cost")
    _check(lib().empc_rollout_cost(_cprob(prob), _ptr(x0), _ptr(knots), int(ncand), int(ld),
                                   _ptr(cost), _stream(stream)))


def empc_generation(prob, ga, knots_in, ld_in, cost_in, knots_out, ld_out, elite_idx, best_idx,
                    tick, gen, stream=None):
    dt, n, m, pm = _shape(prob)
    g = ga.c if hasattr(ga, "c") else ga
    pop, k = int(g.pop), int(g.n_elite)
    if ld_out >= pop:
        _need(knots_out, dt, _soa_elems(pm, ld_out, pop), "knots_out")
    if knots_in is not None and ld_in >= pop:
        _need(knots_in, dt, _soa_elems(pm, ld_in, pop), "knots_in")
        _need(cost_in, dt, pop, "cost_in")
        _need(elite_idx, torch.int64, k, "elite_idx")
    _need(best_idx, torch.int64, 1, "best_idx", optional=True)
    _check(lib().empc_generation(_cprob(prob), _cga(ga), _ptr(knots_in), int(ld_in),
                                 _ptr(cost_in), _ptr(knots_out), int(ld_out), _ptr(elite_idx),
                                 _ptr(best_idx), int(tick), int(gen), _stream(stream)))


def empc_workspace_bytes(prob, ga) -> int:
    return int(lib().empc_workspace_bytes(_cprob(prob), _cga(ga)))


def _need_solve_io(prob, workspace, x0, u_star, best_cost):
    dt, n, m, _ = _shape(prob)
    _need(workspace, torch.uint8, 1, "workspace")
    _need(x0, dt, n, "x0")
    _need(u_star, dt, m, "u_star")
    _need(best_cost, dt, 1, "best_cost")


def empc_solve(prob, ga, workspace, x0, tick, u_star, best_cost, stream=None):
    _need_solve_io(prob, workspace, x0, u_star, best_cost)
    _check(lib().empc_solve(_cprob(prob), _cga(ga), _ptr(workspace), workspace.numel(),
                            _ptr(x0), int(tick), _ptr(u_star), _ptr(best_cost), _stream(stream)))


def empc_solve_refined(prob, ga, workspace, x0, tick, lr, adam_steps, u_star, best_cost,
                       stream=None):
    _need_solve_io(prob, workspace, x0, u_star, best_cost)
    _check(lib().empc_solve_refined(_cprob(prob), _cga(ga), _ptr(workspace), workspace.numel(),
                                    _ptr(x0), int(tick), float(lr), int(adam_steps), _ptr(u_star),
                                    _ptr(best_cost), _stream(stream)))


def empc_autotune(prob, ga, reps=5, allow_valu=True, stream=None):
    """Tune the single-problem launch shapes of (prob, ga); returns a dict of
    the choice and its measured times (microseconds)."""
    info = (ctypes.c_float * 5)()
    _check(lib().empc_autotune(_cprob(prob), _cga(ga), int(reps), 1 if allow_valu else 0, info,
                               _stream(stream)))
    return {"rollout_form": int(info[0]), "pop_groups": int(info[1]), "rollout_us": info[2],
            "rule_rollout_us": info[3], "population_us": info[4]}


def empc_autotune_set(prob, ga, form, groups=0):
    _check(lib().empc_autotune_set(_cprob(prob), _cga(ga), int(form), int(groups)))


def empc_autotune_reset():
    _check(lib().empc_autotune_reset())


# rollout form codes of empc_autotune / empc_autotune_set
RF_RULE, RF_ONE1, RF_ONE2, RF_ONE4, RF_SPLIT, RF_VALU256, RF_VALU64 = 0, 1, 2, 3, 4, 5, 6
RF_CH64, RF_CH128, RF_CH256 = 11, 12, 13


def empc_solve_static(prob, ga, x0, tick, cold, u_star, best_cost, stream=None):
    dt, n, m, _ = _shape(prob)
    _need(x0, dt, n, "x0")
    _need(u_star, dt, m, "u_star")
    _need(best_cost, dt, 1, "best_cost")
    _check(lib().empc_solve_static(_cprob(prob), _cga(ga), _ptr(x0), int(tick), int(cold),
                                   _ptr(u_star), _ptr(best_cost), _stream(stream)))


def empc_grad(prob, x0, knots, ncand, ld, dJ, cost, stream=None):
    dt, n, m, pm = _shape(prob)
    if ncand > 0 and ld >= ncand:
        _need(x0, dt, n, "x0")
        _need(knots, dt, _soa_elems(pm, ld, ncand), "knots")
        _need(dJ, dt, _soa_elems(pm, ld, ncand), "dJ")
        _need(cost, dt, ncand, "cost", optional=True)
    _check(lib().empc_grad(_cprob(prob), _ptr(x0), _ptr(knots), int(ncand), int(ld), _ptr(dJ),
                           _ptr(cost), _stream(stream)))


def empc_refine(prob, x0, knots, ncand, ld, cost, lr, steps, stream=None):
    dt, n, m, pm = _shape(prob)
    if ncand > 0 and ld >= ncand and steps > 0:
        _need(x0, dt, n, "x0")
        _need(knots, dt, _soa_elems(pm, ld, ncand), "knots")
        _need(cost, dt, ncand, "cost")
    _check(lib().empc_refine(_cprob(prob), _ptr(x0), _ptr(knots), int(ncand), int(ld),
                             _ptr(cost), float(lr), int(steps), _stream(stream)))


def empc_plant_step(prob, x, u, noise, x_next, stream=None):
    dt, n, m, _ = _shape(prob)
    _need(x, dt, n, "x")
    _need(u, dt, m, "u")
    _need(noise, dt, n, "noise", optional=True)
    _need(x_next, dt, n, "x_next")
    _check(lib().empc_plant_step(_cprob(prob), _ptr(x), _ptr(u), _ptr(noise), _ptr(x_next),
                                 _stream(stream)))


def empc_batch_workspace_bytes(cprobs, nprob, ga) -> int:
    return int(lib().empc_batch_workspace_bytes(cprobs, int(nprob), _cga(ga)))


def empc_batch_create(cprobs, nprob, ga, workspace, x0_packed, u_star_packed, best_cost):
    nsum = sum(int(cprobs[i].n) for i in range(int(nprob)))
    msum = sum(int(cprobs[i].m) for i in range(int(nprob)))
    _need(workspace, torch.uint8, 1, "workspace")
    _need(x0_packed, torch.float32, nsum, "x0_packed")
    _need(u_star_packed, torch.float32, msum, "u_star_packed")
    _need(best_cost, torch.float32, int(nprob), "best_cost")
    plan = ctypes.c_void_p()
    _check(lib().empc_batch_create(cprobs, int(nprob), _cga(ga), _ptr(workspace),
                                   workspace.numel(), _ptr(x0_packed), _ptr(u_star_packed),
                                   _ptr(best_cost), ctypes.byref(plan)))
    return plan


def empc_solve_batched(plan, stream=None):
    _check(lib().empc_solve_batched(plan, _stream(stream)))


def empc_batch_destroy(plan):
    _check(lib().empc_batch_destroy(plan))


def empc_batch_autotune(plan, reps=5, stream=None):
    _check(lib().empc_batch_autotune(plan, int(reps), _stream(stream)))


def empc_batch_classes(plan) -> int:
    return int(lib().empc_batch_classes(plan))


def empc_batch_class_info(plan, cls) -> dict:
    info = (ctypes.c_int32 * 7)()
    _check(lib().empc_batch_class_info(plan, int(cls), info))
    us = (ctypes.c_float * 4)()
    _check(lib().empc_batch_class_times(plan, int(cls), us))
    return {"model": "linear" if info[0] == EMPC_LINEAR else "pendulum_chain",
            "shape": (int(info[1]), int(info[2])), "problems": int(info[3]),
            "variant": int(info[4]), "variants": int(info[5]), "stream": int(info[6]),
            "tuned_us": [round(float(us[v]), 1) for v in range(int(info[5]))]}


def empc_batch_set_variant(plan, cls, variant):
    _check(lib().empc_batch_set_variant(plan, int(cls), int(variant)))


def empc_profile_begin(max_launches):
    _check(lib().empc_profile_begin(int(max_launches)))


def empc_profile_end():
    """(number of timed rollout launches, their summed duration in ms)."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().empc_profile_end(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


# ---------------------------------------------------------------------------
# device-side problem description


class DeviceProblem:
    """A problem's arrays copied to the GPU, plus the C struct pointing at them.

    `prob` is any object with the fields of the C struct: model, n, m, T, p,
    Ad, Bd, wd (linear) or stiffness, damping, mass, length, gravity, dt
    (chain), and q, r, qf, x_goal, u_goal, u_min, u_max, and optionally the
    state box x_min, x_max, qb with its step charge sb, chain joint limits
    q_min, q_max with restitution, full weights Q, R, Qf, chain dry friction
    fric_c, fric_s (host arrays).
    """

    _ARRAYS = ("Ad", "Bd", "wd", "stiffness", "damping", "mass", "length", "q", "r", "qf",
               "x_goal", "u_goal", "u_min", "u_max", "x_min", "x_max", "qb", "sb", "q_min",
               "q_max", "Q", "R", "Qf", "fric_c", "fric_s")
    # may be None (NULL); the zero-droppable ones are also passed as NULL
    # when all zero (x_min / x_max are bounds: a zero bound is kept)
    _OPTIONAL = ("wd", "qf", "x_goal", "u_goal", "qb", "sb")

    def __init__(self, prob, dtype=torch.float32, device="cuda", keep=()):
        """keep: names of optional arrays to place on the device even when
        they are all zero (a model rewritten in place later, e.g. the w_d of
        a relinearized robot)."""
        self.prob, self.dtype, self.device = prob, dtype, torch.device(device)
        self.tensors = {}
        c = EmpcProblem()
        c.n, c.m, c.T, c.p = int(prob.n), int(prob.m), int(prob.T), int(prob.p)
        c.dtype = EMPC_F64 if dtype == torch.float64 else EMPC_F32
        c.model = int(prob.model)
        sb = getattr(prob, "sb", None)
        if sb is not None and np.any(np.asarray(sb)):
            keep = tuple(keep) + ("qb",)  # the step charge needs the box, zero weights or not
        for name in self._ARRAYS:
            v = getattr(prob, name, None)
            # optional arrays that are all zero are passed as NULL (= 0 by the
            # ABI), which lets the kernels skip them
            if v is None or (name in self._OPTIONAL and name not in keep and
                             not np.any(np.asarray(v))):
                setattr(c, name, None)
                continue
            t = torch.as_tensor(v, dtype=dtype).contiguous().to(self.device)
            self.tensors[name] = t
            setattr(c, name, t.data_ptr())
        c.gravity = float(getattr(prob, "gravity", 0.0) or 0.0)
        c.dt = float(getattr(prob, "dt", 0.0) or 0.0)
        c.restitution = float(getattr(prob, "restitution", 0.0) or 0.0)
        self.c = c

    @property
    def n(self):
        return self.c.n

    @property
    def m(self):
        return self.c.m

    @property
    def pm(self):
        return self.c.p * self.c.m


def make_ga(ga) -> EmpcGA:
    g = EmpcGA()
    g.pop, g.n_elite, g.generations = int(ga.pop), int(ga.n_elite), int(ga.generations)
    g.elitism = 1 if getattr(ga, "elitism", True) else 0
    g.sigma, g.seed = float(ga.sigma), int(ga.seed)
    g.shift = 1 if getattr(ga, "shift", False) else 0
    g.sigma_min = float(getattr(ga, "sigma_min", 0.0))
    g.sigma_dist = float(getattr(ga, "sigma_dist", 0.0))
    return g


class Solver:
    """Warm-started EMPC controller for one problem: owns the workspace."""

    def __init__(self, dprob: DeviceProblem, ga):
        self.dprob = dprob
        self.ga = make_ga(ga)
        nbytes = empc_workspace_bytes(dprob, self.ga)
        if nbytes == 0:
            _check(EMPC_EINVAL)
        self.workspace = torch.zeros(nbytes, dtype=torch.uint8, device=dprob.device)
        self.u_star = torch.zeros(dprob.m, dtype=dprob.dtype, device=dprob.device)
        self.best_cost = torch.zeros(1, dtype=dprob.dtype, device=dprob.device)

    def reset(self):
        self.workspace.zero_()

    def solve(self, x0: torch.Tensor, tick: int, stream=None, refine_steps: int = 0,
              lr: float = 0.01):
        """Runs one tick; returns (u*, best cost) device tensors (asynchronous).
        refine_steps > 0 refines the parents of every generation by Adam."""
        if refine_steps > 0:
            empc_solve_refined(self.dprob, self.ga, self.workspace, x0, tick, lr, refine_steps,
                               self.u_star, self.best_cost, stream)
        else:
            empc_solve(self.dprob, self.ga, self.workspace, x0, tick, self.u_star,
                       self.best_cost, stream)
        return self.u_star, self.best_cost


class EmpcCost(torch.autograd.Function):
    """cost[c] = J(knots[:, c]) with the hand-written adjoint as backward.

    forward(knots [p*m, ncand] GPU tensor, x0 [n], dprob) -> cost [ncand]
    """

    @staticmethod
    def forward(ctx, knots, x0, dprob):
        knots = knots.contiguous()
        ncand = knots.shape[1]
        cost = torch.empty(ncand, dtype=knots.dtype, device=knots.device)
        if not ctx.needs_input_grad[0]:
            # forward only: the rollout kernel, no adjoint pass
            empc_rollout_cost(dprob, x0.contiguous(), knots, ncand, ncand, cost)
            return cost
        dJ = torch.empty_like(knots)
        empc_grad(dprob, x0.contiguous(), knots, ncand, ncand, dJ, cost)
        ctx.save_for_backward(dJ)
        return cost

    @staticmethod
    def backward(ctx, grad_cost):
        (dJ,) = ctx.saved_tensors
        return dJ * grad_cost.unsqueeze(0), None, None


class BatchSolver:
    """Warm-started EMPC for many independent FP32 problems, one tick per call.

    dprobs: DeviceProblem list (float32).  x0 is the packed device tensor of
    initial states (problem after problem); u_star and best_cost are the
    packed outputs.  The device tick counter starts at 0 and advances by one
    per solve()."""

    def __init__(self, dprobs, ga, autotune=True, tune_reps=5, allow_valu=False):
        self.dprobs = list(dprobs)
        self.ga = make_ga(ga)
        n = len(self.dprobs)
        arr = (EmpcProblem * n)(*[d.c for d in self.dprobs])
        self._arr = arr
        nbytes = empc_batch_workspace_bytes(arr, n, self.ga)
        if nbytes == 0:
            _check(EMPC_EINVAL)
        dev = self.dprobs[0].device
        self.workspace = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.x_off = np.concatenate([[0], np.cumsum([d.n for d in self.dprobs])])
        self.u_off = np.concatenate([[0], np.cumsum([d.m for d in self.dprobs])])
        self.x0 = torch.zeros(int(self.x_off[-1]), dtype=torch.float32, device=dev)
        self.u_star = torch.zeros(int(self.u_off[-1]), dtype=torch.float32, device=dev)
        self.best_cost = torch.zeros(n, dtype=torch.float32, device=dev)
        self.plan = empc_batch_create(arr, n, self.ga, self.workspace, self.x0, self.u_star,
                                      self.best_cost)
        if allow_valu:
            self.allow_valu(True)
        if autotune:
            self.autotune(tune_reps)

    def autotune(self, reps=5, stream=None):
        """Time every launch shape of every kernel class on these problems
        and keep the fastest (results do not depend on the choice)."""
        empc_batch_autotune(self.plan, reps, stream)

    def classes(self):
        return [empc_batch_class_info(self.plan, i) for i in range(empc_batch_classes(self.plan))]

    def set_variant(self, cls, variant):
        empc_batch_set_variant(self.plan, cls, variant)

    def allow_valu(self, allow=True):
        """Offer the vector-ALU form as a launch shape of the linear classes
        of at most 16 states and inputs (its cost is summed in another order
        than the matrix-core shapes', so results may differ in the last
        bits); call autotune() afterwards to let it be picked."""
        _check(lib().empc_batch_allow_valu(self.plan, 1 if allow else 0))

    def set_mode(self, mode):
        """0: a launch per kernel class (default); 1: the persistent
        work-queue form (same results)."""
        _check(lib().empc_batch_set_mode(self.plan, int(mode)))

    def set_x0(self, i, x):
        self.x0[int(self.x_off[i]):int(self.x_off[i + 1])] = torch.as_tensor(
            x, dtype=torch.float32, device=self.x0.device)

    def solve(self, stream=None):
        empc_solve_batched(self.plan, stream)
        return self.u_star, self.best_cost

    def u_of(self, i):
        return self.u_star[int(self.u_off[i]):int(self.u_off[i + 1])]

    def close(self):
        if self.plan is not None:
            empc_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NLinkRobot:
    """The N-link planar robot's parameters on the GPU plus the C struct.

    mass, length: host arrays (N,); damping: b."""

    def __init__(self, mass, length, damping, dtype=torch.float64, device="cuda"):
        self.dtype = dtype
        self.mass = torch.as_tensor(np.asarray(mass), dtype=dtype).contiguous().to(device)
        self.length = torch.as_tensor(np.asarray(length), dtype=dtype).contiguous().to(device)
        c = EmpcNLink()
        c.links = int(self.mass.numel())
        c.dtype = EMPC_F64 if dtype == torch.float64 else EMPC_F32
        c.mass, c.length = self.mass.data_ptr(), self.length.data_ptr()
        c.damping = float(damping)
        self.c = c

    @property
    def links(self):
        return self.c.links


def empc_nlink_linearize(robot, dt, x, u, Ad, Bd, wd, stream=None):
    N, dt_ = robot.links, robot.dtype
    _need(x, dt_, 2 * N, "x")
    _need(u, dt_, N, "u")
    _need(Ad, dt_, 4 * N * N, "Ad")
    _need(Bd, dt_, 2 * N * N, "Bd")
    _need(wd, dt_, 2 * N, "wd")
    _check(lib().empc_nlink_linearize(ctypes.byref(robot.c), float(dt), _ptr(x), _ptr(u),
                                      _ptr(Ad), _ptr(Bd), _ptr(wd), _stream(stream)))


def empc_nlink_step(robot, dt, substeps, x, u, x_next, stream=None):
    N, dt_ = robot.links, robot.dtype
    _need(x, dt_, 2 * N, "x")
    _need(u, dt_, N, "u")
    _need(x_next, dt_, 2 * N, "x_next")
    _check(lib().empc_nlink_step(ctypes.byref(robot.c), float(dt), int(substeps), _ptr(x),
                                 _ptr(u), _ptr(x_next), _stream(stream)))


def empc_qp_workspace_bytes(prob) -> int:
    return int(lib().empc_qp_workspace_bytes(_cprob(prob)))


def empc_qp_form(prob, x0, workspace, P, q, c, stream=None):
    dt, n, m, pm = _shape(prob)
    _need(x0, dt, n, "x0")
    _need(workspace, torch.uint8, 1, "workspace")
    _need(P, dt, pm * pm, "P")
    _need(q, dt, pm, "q")
    _need(c, dt, 1, "c")
    _check(lib().empc_qp_form(_cprob(prob), _ptr(x0), _ptr(workspace), workspace.numel(),
                              _ptr(P), _ptr(q), _ptr(c), _stream(stream)))


def empc_qp_solve(prob, P, q, c, workspace, max_iter, z, cost, info, stream=None):
    dt, n, m, pm = _shape(prob)
    _need(P, dt, pm * pm, "P")
    _need(q, dt, pm, "q")
    _need(c, dt, 1, "c")
    _need(workspace, torch.uint8, 1, "workspace")
    _need(z, dt, pm, "z")
    _need(cost, dt, 1, "cost")
    _need(info, torch.int32, 2, "info")
    _check(lib().empc_qp_solve(_cprob(prob), _ptr(P), _ptr(q), _ptr(c), _ptr(workspace),
                               workspace.numel(), int(max_iter), _ptr(z), _ptr(cost), _ptr(info),
                               _stream(stream)))


class ConvexSolver:
    """Parameterized small-matrix convex MPC of one linear problem on the
    GPU: form P, q, c at x0, then the box QP; owns the buffers."""

    def __init__(self, dprob, max_iter=100):
        self.dprob = dprob
        dt, n, m, pm = _shape(dprob)
        nbytes = empc_qp_workspace_bytes(dprob)
        if nbytes == 0:
            _check(EMPC_EUNSUPPORTED)
        dev = dprob.device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.P = torch.empty(pm, pm, dtype=dt, device=dev)
        self.q = torch.empty(pm, dtype=dt, device=dev)
        self.c = torch.empty(1, dtype=dt, device=dev)
        self.z = torch.empty(pm, dtype=dt, device=dev)
        self.cost = torch.empty(1, dtype=dt, device=dev)
        self.info = torch.zeros(2, dtype=torch.int32, device=dev)
        self.max_iter = max_iter

    def solve(self, x0, stream=None):
        """(z [p*m], J(z) [1], info [iterations, converged]) device tensors;
        u* = z[:m]."""
        empc_qp_form(self.dprob, x0, self.workspace, self.P, self.q, self.c, stream)
        empc_qp_solve(self.dprob, self.P, self.q, self.c, self.workspace, self.max_iter, self.z,
                      self.cost, self.info, stream)
        return self.z, self.cost, self.info
