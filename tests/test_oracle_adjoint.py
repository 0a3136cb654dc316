"""Pins of the oracle's adjoint pieces: the transposed operators against the
transposed dense matrices of the (separately pinned) forward operators, the
row derivatives in m = 1/c^2 against central differences of the forward
operators, and the whole gradient against central differences of a misfit
computed with converged forward solves."""
import numpy as np
import pytest

from workloads import grf_velocity, random_complex
from tests.test_oracle_solver import _dense

H = 10.0
OMEGA = 2 * np.pi * 1500.0 / (6 * H)
OP_A, OP_B, OP_Q = 0, 1, 2


@pytest.fixture(scope="module")
def pml_grid(oracle_lib, table):
    vel = grf_velocity(8, 4, 4, seed=31, corr_len=2.0)     # total 12 x 8 x 8 with n_pml = 2
    return oracle_lib.Hierarchy(vel, H, OMEGA, 2, table)


def _rand(Hh, level, seed):
    nx, ny, nz = Hh.dims(level)
    return random_complex((nx, ny, nz), seed, boundary_zero=True).astype(complex)


@pytest.mark.parametrize("level,op", [(0, OP_A), (0, OP_B), (0, OP_Q), (1, OP_A), (1, OP_B), (2, OP_B)])
def test_transpose_is_the_transposed_matrix(pml_grid, level, op):
    """apply_t is the transpose (not the conjugate transpose) of apply, entry by
    entry, with PML and a variable velocity (where A itself is not symmetric)."""
    Hh = pml_grid
    A = _dense(Hh, level, lambda e: Hh.apply(level, op, e))
    At = _dense(Hh, level, lambda e: Hh.apply_t(level, op, e))
    assert np.abs(A - A.T).max() > 1e-6 * np.abs(A).max()    # the check is not vacuous
    assert np.abs(At - A.T).max() <= 1e-13 * np.abs(A).max()


def _extend(Hh, phys):
    """Physical-node field on the total fine grid by nearest physical node."""
    nx, ny, nz = Hh.dims(0)
    p = Hh.n_pml
    px, py, pz = Hh.phys
    ix = np.clip(np.arange(nx + 1) - p, 0, px)
    iy = np.clip(np.arange(ny + 1) - p, 0, py)
    iz = np.clip(np.arange(nz + 1) - p, 0, pz)
    return phys[np.ix_(iz, iy, ix)]


def _perturbed(oracle_lib, table, vel, eps, seed):
    """Velocities c0 (1 +- eps r) rounded to float32 (the oracle's input type) and
    the exact squared-slowness difference m+ - m- they represent.  The coefficient
    tables are cubic Hermite interpolants, only C^1 at their knots, so the step is
    kept small (1e-5) to leave few nodes whose difference straddles a knot."""
    r = np.random.default_rng(seed).uniform(-1.0, 1.0, vel.shape)
    cp = (vel * (1 + eps * r)).astype(np.float32)
    cm = (vel * (1 - eps * r)).astype(np.float32)
    dm = 1.0 / cp.astype(np.float64) ** 2 - 1.0 / cm.astype(np.float64) ** 2
    return (oracle_lib.Hierarchy(cp, H, OMEGA, 2, table), oracle_lib.Hierarchy(cm, H, OMEGA, 2, table), dm)


@pytest.mark.parametrize("op", [OP_A, OP_Q])
def test_row_derivative_matches_central_difference(oracle_lib, table, op):
    """Row i of A_h (and of Q_h) depends on m_i only; (op(m+) - op(m-)) x equals
    dm_i (d_i op x)_i to second order in the step."""
    vel = grf_velocity(8, 4, 4, seed=32, corr_len=2.0).astype(np.float32)
    H0 = oracle_lib.Hierarchy(vel, H, OMEGA, 2, table)
    Hp, Hm, dm = _perturbed(oracle_lib, table, vel, 1e-5, 33)
    x = _rand(H0, 0, 34)
    fd = Hp.apply(0, op, x) - Hm.apply(0, op, x)
    an = _extend(H0, dm) * H0.apply_dm(op, x)
    err = np.linalg.norm(fd - an) / np.linalg.norm(fd)
    assert err <= 1e-5, err


def test_gradient_matches_central_difference(oracle_lib, table):
    """dJ/dm for J = Re sum conj(s) u(m), u = Q_h v, A_h v = Q_h f, against
    (J(m+) - J(m-)) along eight seeded random directions, with the PML nodes
    following their nearest physical node; forward and adjoint solves to 1e-12."""
    vel = grf_velocity(8, 4, 4, seed=35, corr_len=2.0).astype(np.float32)
    H0 = oracle_lib.Hierarchy(vel, H, OMEGA, 2, table)
    f = _rand(H0, 0, 36)
    s = _rand(H0, 0, 37)
    g, its, rel, st = H0.grad(f, s, 1e-12)
    assert st == 0 and rel.max() <= 1e-12, (its, rel)
    for seed in range(38, 46):
        Hp, Hm, dm = _perturbed(oracle_lib, table, vel, 1e-5, seed)
        up, *_ = Hp.solve(f, 1e-12)
        um, *_ = Hm.solve(f, 1e-12)
        fd = float(np.real(np.vdot(s, up) - np.vdot(s, um)))
        an = float(np.sum(g * dm))
        assert abs(fd - an) <= 1e-5 * abs(fd), (seed, fd, an)
    # the physical boundary nodes collect their PML columns: nonzero there
    assert abs(g[0, 4, 4]) > 0 and abs(g[4, 4, 0]) > 0
