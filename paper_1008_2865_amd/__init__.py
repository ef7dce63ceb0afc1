"""MI355X-native two-belt Shan-Chen lattice Boltzmann hot path.

The fused D2Q9 stream + BGK collide step with the two-belt (24-link)
pseudopotential force, and the pseudo-potential energy and mass reductions,
as hand-written HIP kernels for gfx950 behind the C ABI of include/lb.h.
``binding`` exposes the lb_* calls; ``sim.LBSim`` wraps one lattice.
"""
from .binding import (LB_F16DEV, LB_F32, LB_F64, LBError, LBLibraryMissing,  # noqa: F401
                      lb_destroy, lb_get_state, lb_init, lb_last_error, lb_launch_shape,
                      lb_moments, lb_params, lb_pseudo_energy, lb_set_state, lb_step,
                      lb_tables, lb_time, lb_trace, lb_validate, lb_workspace_bytes,
                      make_params)
