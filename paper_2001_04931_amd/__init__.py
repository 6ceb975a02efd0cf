"""EMPC on MI355X (gfx950): parameterized Evolutionary MPC hot path.

The compute lives in libempc.so (hand-written HIP kernels behind the C ABI of
include/empc.h); `binding` marshals torch GPU tensors into it.
"""
from .binding import (BatchSolver, ConvexSolver, DeviceProblem, EmpcCost, EmpcError, EmpcGA, EmpcProblem,  # noqa: F401
                      NLinkRobot, Solver, empc_autotune, empc_autotune_reset,
                      empc_autotune_set, empc_generation, empc_grad, empc_nlink_linearize,
                      empc_nlink_step, empc_plant_step, empc_profile_begin,
                      empc_profile_end, empc_refine,
                      empc_rollout_cost, empc_solve, empc_solve_static, empc_workspace_bytes, lib,
                      empc_qp_form, empc_qp_solve, empc_qp_workspace_bytes, make_ga)
from .binding import (EMPC_EDEVICE, EMPC_EINVAL, EMPC_EUNSUPPORTED, EMPC_EWORKSPACE,  # noqa: F401
                      EMPC_OK, RF_CH64, RF_CH128, RF_CH256, RF_ONE1, RF_ONE2, RF_ONE4, RF_RULE,
                      RF_SPLIT, RF_VALU64, RF_VALU256)
