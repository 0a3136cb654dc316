"""Pins of the oracle's Algorithm 1 composition and of the coarse-level
velocity sampling.

Algorithm 1 (Sec. 3.3, alg:three-grid) is rebuilt densely in numpy from pieces
that other tests pin (the level operators, J_2, full weighting and trilinear
prolongation): the two smoothing cycles as dense minimal-residual problems,
and the 2h correction as an exact solve with A_2h (K_2h made exact by giving
it at least as many flexible steps as there are 2h unknowns).  The coarse
levels take the velocity at their own nodes from the PML-extended fine field
(Sec. 2.1, Sec. 3.1: sampled, not averaged); that is checked against numpy
indexing of the physical input and through one coarse row of the shell form
(eq. iofd-shell-form) evaluated at the sampled value.
"""
import numpy as np
import pytest

from tests import paper_formulas as pf
from tests.test_oracle_solver import _dense, _embed, _min_res
from workloads import grf_velocity, point_source

H = 10.0
OMEGA = 2 * np.pi * 1500.0 / (6 * H)


def _inner(v):
    return v[1:-1, 1:-1, 1:-1].reshape(-1)


@pytest.fixture(scope="module")
def grid12(oracle_lib, table):
    """12^3 total (8^3 physical + 2 PML cells), GRF velocity; 125 unknowns at 2h."""
    vel = grf_velocity(8, 8, 8, seed=31, corr_len=3.0)
    n2 = 5 ** 3
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, 2, table, params=dict(m_2h=n2 + 5, c_2h=2))
    return Hh


def test_algorithm1_composition(grid12):
    """z = M_h^{-1} r equals the five steps of Algorithm 1 built densely:
    z_pre = S_h(r; 0); r_2h = R(r - A z_pre); e = A_2h^{-1} r_2h;
    z~ = z_pre + P e; z = S_h(r; z~), with S_h the minimal-residual iterate of
    one GMRES(2) cycle right preconditioned by J_2(A_h; 0.8)."""
    Hh = grid12
    A = _dense(Hh, 0, lambda e: Hh.apply(0, 0, e))
    M = _dense(Hh, 0, lambda e: Hh.jacobi(0, 0, e, 2, 0.8))
    A2 = _dense(Hh, 1, lambda e: Hh.apply(1, 0, e))
    rng = np.random.default_rng(41)
    n = A.shape[0]
    r = rng.standard_normal(n) + 1j * rng.standard_normal(n)

    def restrict(v):
        return _inner(Hh.restrict(0, _embed(Hh, 0, v)))

    def prolong(v):
        return _inner(Hh.prolong(1, _embed(Hh, 1, v)))

    z_pre = _min_res(A, M, r, 2)
    r2 = restrict(r - A @ z_pre)
    e2 = np.linalg.solve(A2, r2)
    z_t = z_pre + prolong(e2)
    z = z_t + _min_res(A, M, r - A @ z_t, 2)
    got = _inner(Hh.precond(_embed(Hh, 0, r)))
    np.testing.assert_allclose(got, z, rtol=1e-9, atol=1e-10 * np.abs(z).max())
    # the exact 2h correction matters: the composition without it is far away
    z_no_cgc = z_pre + _min_res(A, M, r - A @ z_pre, 2)
    assert np.linalg.norm(got - z_no_cgc) > 1e-3 * np.linalg.norm(z)


@pytest.mark.parametrize("level", [1, 2])
def test_coarse_velocity_is_sampled_extension(oracle_lib, table, level):
    """Level s = 2^l holds c_ext(s j) with c_ext the nearest-physical-value
    extension into the PML; checked by numpy indexing of the physical input on
    a GRF velocity with distinct axis lengths."""
    npml = 4
    nx, ny, nz = 24, 16, 32
    vel = grf_velocity(nx, ny, nz, seed=33, corr_len=3.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, npml, table)
    s = 2 ** level
    dims = Hh.dims(level)

    def ext_index(j, n_phys):
        return np.clip(s * np.arange(j + 1) - npml, 0, n_phys)

    ix, iy, iz = ext_index(dims[0], nx), ext_index(dims[1], ny), ext_index(dims[2], nz)
    expect = vel[np.ix_(iz, iy, ix)].astype(np.float64)
    np.testing.assert_array_equal(Hh.velocity(level), expect)


@pytest.mark.parametrize("level", [1, 2])
def test_coarse_row_uses_sampled_velocity(oracle_lib, table, level):
    """One interior coarse row (stencil and its neighbours free of stretching)
    equals ell^-2 sum_m C_m S_m (eq. iofd-shell-form, eq. iofd-shell-coefficients)
    with the coefficients taken at the velocity of the fine node s j."""
    npml = 4
    nx, ny, nz = 40, 32, 48
    vel = grf_velocity(nx, ny, nz, seed=34, corr_len=2.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, npml, table)
    s = 2 ** level
    ell = s * H
    dims = Hh.dims(level)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(Hh.shape(level)) + 1j * rng.standard_normal(Hh.shape(level))
    y = Hh.apply(level, 0, x)
    spl = pf.alpha_functions(table)
    checked = 0
    # nodes whose neighbours sit at least one coarse cell inside the physical box
    lo = npml // s + 2
    for jz in range(lo, dims[2] - lo + 1):
        for jy in range(lo, dims[1] - lo + 1):
            jx = lo + (3 * jz + jy) % (dims[0] - 2 * lo + 1)
            c = float(vel[s * jz - npml, s * jy - npml, s * jx - npml])
            es, kappa = pf.eta_star(c, OMEGA, ell)
            a = [float(spl[f](es)) for f in range(5)]
            C = pf.shell_coefficients(a, kappa ** 2)
            S = [0j, 0j, 0j, 0j]
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        S[abs(dx) + abs(dy) + abs(dz)] += x[jz + dz, jy + dy, jx + dx]
            expect = sum(C[m] * S[m] for m in range(4)) / ell ** 2
            np.testing.assert_allclose(y[jz, jy, jx], expect, rtol=1e-12)
            checked += 1
    assert checked >= 30


def test_solution_scales_with_source(oracle_lib, table):
    """The solve is linear: scaling f by 2^60, 1e20 or 1e-20 scales u by the same
    factor (every inner stopping rule is scale-free; a happy-breakdown test
    against the unnormalised residual norm cut cycles short for large f)."""
    vel = grf_velocity(16, 16, 16, seed=35, corr_len=4.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, 4, table)
    f = point_source((24, 24, 24), (11, 12, 13), H)
    u0, its0, rel0, st0 = Hh.solve(f, 1e-8)
    assert st0 == 0
    for s in (2.0 ** 60, 1e20, 1e-20):
        u, its, rel, st = Hh.solve(f * s, 1e-8)
        assert st == 0 and its == its0, (s, its, its0)
        np.testing.assert_allclose(u / s, u0, rtol=1e-9, atol=1e-12 * np.abs(u0).max())
