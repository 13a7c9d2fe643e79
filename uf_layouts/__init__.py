"""Seeded synthetic urban layouts and solver configurations.

This package is the only code shared by the HIP path and the FP64 oracle.
It holds plain data (configuration dictionaries with the workload sizes) and
the seeded generator of porosity fields; it computes nothing of the flow
solver itself.  The porosity of a cell follows the paper's unified porosity
encoding (Sec. 3, "Urban model resolving"): phi = 1 - V_s/V, with cut cells
resolved by uniform sub-sampling.
"""
from .configs import (BC_AUTO, BC_INLET, BC_OUTLET, BC_WALL, BC_SLIP,
                      INFLOW_UNIFORM, INFLOW_LOGLAW, INFLOW_PROFILE,
                      TURB_OFF, TURB_KOMEGA,
                      PC_NONE, PC_JACOBI, PC_AI1, PC_AI2, PC_MG,
                      STAGE_ADVECT, STAGE_DIFFUSE, STAGE_DRAG, STAGE_PROJECT,
                      STAGE_TURB, STAGE_ALL,
                      default_config, preset, PRESETS)
from .porosity import (Box, Cylinder, porosity_field, random_city,
                       preset_porosity)
from .fields import smooth_noise, perturbed_state
from .meshes import (box_mesh, prism_mesh, ring_mesh, uv_sphere_mesh, meshes_of,
                     city_meshes)

__all__ = [n for n in dir() if not n.startswith("_")]
