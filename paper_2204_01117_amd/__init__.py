"""MI355X (gfx950) implementation of one UrbanFlow RANS time step.

Thin Python binding of the C ABI in ``include/uf.h`` (libuf.so, built from
``csrc/`` by ``build.py``).  The functions ``uf_*`` are the C entry points
with the same names; :class:`Grid` marshals torch CUDA tensors (used for
device memory and streams only) into them.  Every stage of the step runs in
the library's HIP kernels; there is no Python or CPU fallback, and importing
this package fails when libuf.so is missing.
"""
from ._lib import (lib, LIB_PATH, UFError, uf_config, uf_step_stats, make_config,
                   uf_objective_spec, make_objective_spec, uf_mesh_set, STATUS, FIELDS, FIELD_IDS)
from ._lib import (uf_create_grid, uf_destroy_grid, uf_set_porosity, uf_set_field,
                   uf_get_field, uf_field_extent, uf_resolve_bc, uf_step, uf_pressure_solve,
                   uf_apply_operator, uf_objective, uf_adjoint_step, uf_adjoint_step_at, uf_set_stream,
                   uf_kernel_timer_enable, uf_kernel_timer_read, uf_last_error, TIMED_KERNELS,
                   uf_voxelize, uf_step_batch, uf_smooth_porosity, uf_smooth_porosity_grad,
                   uf_smooth_porosity_grad_noalloc, uf_smooth_objects, uf_batch_create, uf_batch_autotune,
                   uf_batch_step, uf_batch_destroy, uf_batch_tuning)
from .grid import Grid, step_batch, Batch
from .voxelize import voxelize, smooth_porosity, smooth_porosity_grad
from .design import BoxDesign
from .optimize import (SimulationObjective, AdjointObjective, design_objective, forward_difference_gradient,
                       gradient_descent)

__all__ = ["lib", "LIB_PATH", "UFError", "uf_config", "uf_step_stats", "make_config",
           "uf_objective_spec", "make_objective_spec", "uf_mesh_set", "uf_voxelize", "voxelize", "uf_step_batch",
           "step_batch", "uf_smooth_porosity", "uf_smooth_porosity_grad", "uf_smooth_porosity_grad_noalloc",
           "uf_smooth_objects", "uf_batch_create", "uf_batch_autotune", "uf_batch_step", "uf_batch_destroy",
           "uf_batch_tuning", "Batch", "smooth_porosity",
           "smooth_porosity_grad", "BoxDesign", "SimulationObjective", "AdjointObjective", "design_objective",
           "forward_difference_gradient", "gradient_descent",
           "STATUS", "FIELDS", "FIELD_IDS", "Grid",
           "uf_create_grid", "uf_destroy_grid", "uf_set_porosity", "uf_set_field",
           "uf_get_field", "uf_field_extent", "uf_resolve_bc", "uf_step", "uf_pressure_solve",
           "uf_apply_operator", "uf_objective", "uf_adjoint_step", "uf_adjoint_step_at", "uf_set_stream",
           "uf_kernel_timer_enable", "uf_kernel_timer_read", "uf_last_error", "TIMED_KERNELS"]
