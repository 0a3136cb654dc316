"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

Nothing in this package performs any step of the method: it only produces
velocity models, point sources, random test vectors and the coefficient table
file. Both the GPU library and the oracle consume these inputs.

Array conventions
-----------------
* Grid functions are stored ``[z][y][x]`` with x fastest (C order).
* Velocity models live on the *physical* nodes: shape ``(nz+1, ny+1, nx+1)``
  for ``nx, ny, nz`` physical intervals.
* Complex vectors live on the *total* grid (physical plus ``n_pml`` cells per
  face): shape ``(Nz+1, Ny+1, Nx+1)`` with ``N_a = n_a + 2 n_pml``.
"""
from .table import load_iofd_table, table_flat, random_table, constant_table  # noqa: F401
from .media import (  # noqa: F401
    homogeneous, gaussian_random_field, grf_velocity, layered_velocity,
    ellipsoid_grf_velocity, lens_velocity, wedge_velocity, barrier_velocity,
)
from .vectors import point_source, random_complex, zero_boundary  # noqa: F401
from .configs import CONFIGS, omega_for_ppw  # noqa: F401
