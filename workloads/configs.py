"""The five synthetic workloads (grid, PML, medium, sources, precision, tolerance).

Physical intervals per axis ``n``; ``n_pml`` cells per face; total intervals
``n + 2 n_pml`` (divisible by 4). Spacing h = 10 m; the angular frequency puts
six fine-grid points in the shortest wavelength: omega = 2 pi c_min / (6 h).
"""
import math

H = 10.0


def omega_for_ppw(c_min, h=H, ppw=6.0):
    return 2.0 * math.pi * c_min / (ppw * h)


CONFIGS = {
    "c1": dict(name="homogeneous-64-fp64", n=44, n_pml=10, medium="homogeneous", c=1500.0,
               precision="fp64", tol=1e-6, sources="centre"),
    "c2": dict(name="grf-352-fp32", n=320, n_pml=16, medium="grf", seed=2,
               precision="fp32", tol=1e-6, sources="seeded-1"),
    "c3": dict(name="layered-288-fp32-64rhs", n=256, n_pml=16, medium="layered", seed=3,
               precision="fp32", tol=1e-6, sources="grid-8x8-z20"),
    "c4": dict(name="ellipsoid-800-mixed", n=768, n_pml=16, medium="ellipsoid", seed=4,
               precision="mixed", tol=1e-6, sources="seeded-1"),
    "c5": dict(name="grf-216-grad", n=192, n_pml=12, medium="grf", seed=5,
               precision="fp32", tol=1e-6, sources="grid-4x4-z15"),
}
