"""gfx950 (MI355X) implementation of the solver loop of "Agent-Based Optimal
Control for Image Processing" (arXiv 2510.16154).

The compute path is the HIP library ``libabc.so`` (C ABI in include/abc.h);
``binding`` marshals torch tensors into it.  ``synth`` holds the seeded
synthetic inputs and ``workloads`` the named problem sizes.
"""
from .binding import (  # noqa: F401
    ABC_COST_QUADRATIC, ABC_COST_TV, ABC_EHIP, ABC_EINVAL, ABC_ENOCONV, ABC_ENONFINITE, ABC_OK, ABC_WS_ADJOINT, ABC_WS_FORWARD, ABC_WS_PD,
    ABC_WS_SOLVE, AbcError, Params, abc_adjoint_dynamics, abc_adjoint_dynamics_noalloc, abc_default_params, abc_forward_dynamics,
    ABC_FLAG_AUTOTUNE, ABC_FLAG_NO_GRAPHS, ABC_FLAG_PERSISTENT, ABC_MAX_DIRECT_RADIUS, ABC_MAX_RADIUS,
    ABC_RADIUS_SUPPORT, ABC_WS_TUNE, abc_support_radius, abc_autotune, abc_pd_step, abc_pd_terminal, abc_solve, abc_solve_batched, abc_traj_slots, abc_version, abc_workspace_bytes,
    abc_workspace_bytes_batched, abc_segment, abc_segment_workspace_bytes, abc_wsnet_adam, abc_wsnet_forward,
    abc_wsnet_loss_grad, abc_wsnet_param_count,
)
