"""Seeded right-hand sides and random test vectors on the total grid."""
import numpy as np


def point_source(total_dims, idx, h, dtype=np.complex128):
    """f = h^-3 at total-grid node idx = (ix, iy, iz), zero elsewhere (point source,
    Section 5.1). total_dims = (Nx, Ny, Nz) intervals."""
    Nx, Ny, Nz = total_dims
    f = np.zeros((Nz + 1, Ny + 1, Nx + 1), dtype=dtype)
    ix, iy, iz = idx
    f[iz, iy, ix] = h ** -3
    return f


def zero_boundary(v):
    """Set every node with an index 0 or N on any axis to zero (in place)."""
    v[0], v[-1] = 0, 0
    v[:, 0], v[:, -1] = 0, 0
    v[:, :, 0], v[:, :, -1] = 0, 0
    return v


def random_complex(dims, seed, dtype=np.complex128, boundary_zero=True):
    """Seeded standard complex normal vector on a grid of dims = (Nx, Ny, Nz) intervals."""
    Nx, Ny, Nz = dims
    rng = np.random.default_rng(seed)
    shp = (Nz + 1, Ny + 1, Nx + 1)
    v = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)).astype(dtype)
    if boundary_zero:
        zero_boundary(v)
    return v
