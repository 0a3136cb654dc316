"""Seeded velocity models on physical nodes, shape (nz+1, ny+1, nx+1), in m/s.

Recipes follow the workloads the paper measures on (Section 6.2 closed-form
media) and the synthetic heterogeneous models used for the benchmarks:
Gaussian random fields, layered models and a high-contrast inclusion.
"""
import numpy as np


def _shape(nx, ny, nz):
    return (nz + 1, ny + 1, nx + 1)


def homogeneous(nx, ny, nz, c=1500.0):
    return np.full(_shape(nx, ny, nz), c, dtype=np.float32)


# fields with more nodes than this are filtered with scipy's real FFT on all host
# threads (same filter; rounding differs from the numpy path at the 1e-16 level)
_FAST_FFT_NODES = 1 << 27


def gaussian_random_field(nx, ny, nz, corr_len, seed):
    """White noise convolved (FFT, periodic) with a Gaussian of std corr_len/2,
    so the covariance is proportional to exp(-r^2 / corr_len^2); normalised to
    max |g| = 1. Returns float64."""
    rng = np.random.default_rng(seed)
    shp = _shape(nx, ny, nz)
    w = rng.standard_normal(shp)
    s = corr_len / 2.0
    if w.size > _FAST_FFT_NODES:
        import os
        import scipy.fft as sfft
        workers = os.cpu_count() or 1
        ks = [np.fft.fftfreq(n) * 2 * np.pi for n in shp[:2]] + [np.fft.rfftfreq(shp[2]) * 2 * np.pi]
        kz, ky, kx = np.meshgrid(*ks, indexing="ij", sparse=True)
        W = sfft.rfftn(w, workers=workers)
        del w
        W *= np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
        g = sfft.irfftn(W, s=shp, workers=workers)
        del W
        g /= np.abs(g).max()
        return g
    ks = [np.fft.fftfreq(n) * 2 * np.pi for n in shp]
    kz, ky, kx = np.meshgrid(*ks, indexing="ij", sparse=True)
    filt = np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
    g = np.fft.ifftn(np.fft.fftn(w) * filt).real
    return g / np.abs(g).max()


def grf_velocity(nx, ny, nz, seed, c0=2000.0, rel=0.25, corr_len=20.0, clip=(1500.0, 3000.0)):
    g = gaussian_random_field(nx, ny, nz, corr_len, seed)
    c = np.clip(c0 * (1.0 + rel * g), clip[0], clip[1])
    return c.astype(np.float32)


def layered_velocity(nx, ny, nz, seed, nlayers=8, vmin=1500.0, vmax=4000.0, min_gap=8):
    """Horizontal layers (constant in x, y) with sharp interfaces at seeded depths."""
    rng = np.random.default_rng(seed)
    while True:
        cuts = np.sort(rng.choice(np.arange(min_gap, nz + 1 - min_gap), nlayers - 1, replace=False))
        if np.all(np.diff(cuts) >= min_gap):
            break
    vel = rng.uniform(vmin, vmax, nlayers)
    vel[0] = vmin                                      # keep c_min attained
    c = np.empty(_shape(nx, ny, nz), dtype=np.float32)
    edges = np.r_[0, cuts, nz + 1]
    for L in range(nlayers):
        c[edges[L]:edges[L + 1]] = vel[L]
    return c


def ellipsoid_grf_velocity(nx, ny, nz, seed, c_bg=1500.0, c_inc=4500.0, semi=(150, 120, 90),
                           rel=0.10, corr_len=20.0):
    """Background with an ellipsoidal inclusion (semi-axes in cells, x/y/z), the
    centre seeded fully inside the box, times (1 + rel*GRF)."""
    rng = np.random.default_rng(seed)
    ax, ay, az = semi
    cx = rng.uniform(ax, nx - ax) if nx > 2 * ax else nx / 2
    cy = rng.uniform(ay, ny - ay) if ny > 2 * ay else ny / 2
    cz = rng.uniform(az, nz - az) if nz > 2 * az else nz / 2
    z, y, x = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij", sparse=True)
    g = gaussian_random_field(nx, ny, nz, corr_len, seed + 1000)
    out = np.empty(g.shape, np.float32)
    for k in range(nz + 1):              # one plane at a time keeps the host memory small
        inside = ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((k - cz) / az) ** 2 <= 1.0
        out[k] = np.where(inside, c_inc, c_bg) * (1.0 + rel * g[k])
    return out


def _normalized(nx, ny, nz):
    z, y, x = np.meshgrid(np.linspace(0, 1, nz + 1), np.linspace(0, 1, ny + 1),
                          np.linspace(0, 1, nx + 1), indexing="ij", sparse=True)
    return x, y, z


def lens_velocity(nx, ny, nz):
    """Converging lens in normalised coordinates (Section 6.2)."""
    x, y, z = _normalized(nx, ny, nz)
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    return (4.0 / 3.0 * (1.0 - 0.5 * np.exp(-32.0 * r2))).astype(np.float32) * np.ones(_shape(nx, ny, nz), np.float32)


def wedge_velocity(nx, ny, nz):
    x, y, z = _normalized(nx, ny, nz)
    c = np.where(z <= 0.4 + 0.1 * y, 2.0, np.where(z <= 0.8 - 0.2 * y, 1.5, 3.0))
    return (c * np.ones(_shape(nx, ny, nz))).astype(np.float32)


def barrier_velocity(nx, ny, nz):
    x, y, z = _normalized(nx, ny, nz)
    inside = (y >= 0.25) & (y <= 0.3) & (z <= 0.75) & (x >= 0) & (x <= 1)
    return (np.where(inside, 1e10, 1.0) * np.ones(_shape(nx, ny, nz))).astype(np.float32)
