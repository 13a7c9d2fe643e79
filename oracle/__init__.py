"""FP64 CPU oracle of one UrbanFlow RANS time step -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct restatement of the paper's
solver (Sec. 3 "Fast Urban Flow Simulation") in NumPy/SciPy float64.  It
exists to check the HIP path: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library and never calls it.

Parity status of each function is stated in its docstring.  Functions whose
result no closed form or paper number fixes are marked "parity unpinned";
everything else is pinned by tests under ``tests/test_oracle_*.py``.
"""
from .bc import (INLET, OUTLET, WALL, SLIP, Geometry, resolve_bc)
from .solver import OracleGrid, FIELDS
from .objective import cell_speed, region_means, region_objective, plane_objective, field_objective, fd_gradient
from .voxelize import voxelize, inside, ray_crossings

__all__ = ["INLET", "OUTLET", "WALL", "SLIP", "Geometry", "resolve_bc",
           "OracleGrid", "FIELDS", "cell_speed", "region_means", "region_objective", "plane_objective", "field_objective", "fd_gradient",
           "voxelize", "inside", "ray_crossings"]
