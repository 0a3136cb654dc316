"""Pins of the oracle's grid transfers and damped Jacobi map:
R = 2^-3 P^* (Sec. 3.1), trilinear reproduction, the transfer symbol of
eq. lfa-transfer-symbol, and the Jacobi polynomial of eq. lfa-bottom-inverse
in the Dirichlet sine basis."""
import numpy as np
import pytest

from tests import paper_formulas as pf
from workloads import homogeneous, grf_velocity

H = 10.0
OMEGA = 2 * np.pi * 1500.0 / (6 * H)


def _hier(oracle_lib, table, dims=(8, 12, 16), npml=0, vel=None):
    nx, ny, nz = (d - 2 * npml for d in dims)
    vel = homogeneous(nx, ny, nz, 1500.0) if vel is None else vel
    return oracle_lib.Hierarchy(vel, H, OMEGA, npml, table)


def _interior_unit(shape, k):
    e = np.zeros(shape, complex)
    e[tuple(i + 1 for i in np.unravel_index(k, tuple(s - 2 for s in shape)))] = 1.0
    return e


@pytest.mark.parametrize("level", [0, 1])
def test_restriction_is_scaled_adjoint_of_prolongation(oracle_lib, table, level):
    """R = 2^-3 P^* on interior unknowns (Sec. 3.1)."""
    Hh = _hier(oracle_lib, table, dims=(8, 16, 12))
    fs, cs = Hh.shape(level), Hh.shape(level + 1)
    nf = int(np.prod([s - 2 for s in fs]))
    nc = int(np.prod([s - 2 for s in cs]))
    R = np.zeros((nc, nf), complex)
    for k in range(nf):
        R[:, k] = Hh.restrict(level, _interior_unit(fs, k))[1:-1, 1:-1, 1:-1].reshape(-1)
    P = np.zeros((nf, nc), complex)
    for k in range(nc):
        P[:, k] = Hh.prolong(level + 1, _interior_unit(cs, k))[1:-1, 1:-1, 1:-1].reshape(-1)
    assert np.abs(R).max() == 0.5 ** 3              # centre weight of full weighting
    np.testing.assert_allclose(R, P.conj().T / 8.0, rtol=0, atol=1e-15)
    # every coarse row carries the full (1/4, 1/2, 1/4)^3 weights, summing to 1
    np.testing.assert_allclose(R.sum(1), 1.0, rtol=1e-15)


def test_prolongation_reproduces_trilinear(oracle_lib, table):
    """Trilinear interpolation is exact on trilinear functions (away from the
    boundary, whose coarse values are zero)."""
    Hh = _hier(oracle_lib, table, dims=(16, 12, 8))
    Z, Y, X = np.meshgrid(*(np.arange(s) for s in Hh.shape(1)), indexing="ij")
    f = lambda x, y, z: 1 + 2 * x - 0.5 * y + 3j * z + 0.25 * x * y - 1j * y * z + 0.1 * x * y * z  # noqa: E731
    coarse = f(X, Y, Z).astype(complex)
    coarse[0], coarse[-1], coarse[:, 0], coarse[:, -1], coarse[:, :, 0], coarse[:, :, -1] = 0, 0, 0, 0, 0, 0
    fine = Hh.prolong(1, coarse)
    z, y, x = np.meshgrid(*(np.arange(s) for s in Hh.shape(0)), indexing="ij")
    expect = f(x / 2, y / 2, z / 2)
    sl = (slice(2, -2),) * 3
    np.testing.assert_allclose(fine[sl], expect[sl], rtol=1e-14)


def test_transfer_symbol(oracle_lib, table):
    """eq. lfa-transfer-symbol: P psi = sum_p phat_p phi_p and R phi_p = phat_p psi
    with psi(j) = e^{2i theta.j}, phi_p(n) = e^{i (theta + pi p).n} (interior nodes
    away from the boundary)."""
    Hh = _hier(oracle_lib, table, dims=(16, 16, 16))
    theta = np.array([0.37, -0.81, 1.23])
    ph = pf.transfer_symbol(theta)
    zc, yc, xc = np.meshgrid(*(np.arange(s) for s in Hh.shape(1)), indexing="ij")
    psi = np.exp(2j * (theta[0] * xc + theta[1] * yc + theta[2] * zc))
    z, y, x = np.meshgrid(*(np.arange(s) for s in Hh.shape(0)), indexing="ij")
    phis = {p: np.exp(1j * ((theta[0] + np.pi * p[0]) * x + (theta[1] + np.pi * p[1]) * y +
                            (theta[2] + np.pi * p[2]) * z)) for p in ph}
    fine = Hh.prolong(1, psi)
    expect = sum(ph[p] * phis[p] for p in ph)
    sl = (slice(2, -2),) * 3
    np.testing.assert_allclose(fine[sl], expect[sl], rtol=1e-13, atol=1e-14)
    for p in ph:
        c = Hh.restrict(0, phis[p])
        np.testing.assert_allclose(c[sl], ph[p] * psi[sl], rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("level,op,nJ,w", [(0, 0, 2, 0.8), (1, 1, 2, 0.8), (2, 1, 2, 0.2), (1, 1, 3, 0.5),
                                           (0, 0, 1, 0.8)])
def test_jacobi_polynomial(oracle_lib, table, level, op, nJ, w):
    """n damped Jacobi sweeps from zero equal the polynomial Xi of
    eq. lfa-bottom-inverse in the Dirichlet sine basis (constant c, no PML)."""
    Hh = _hier(oracle_lib, table, dims=(16, 12, 8) if level < 2 else (16, 16, 16))
    dims = Hh.dims(level)
    ell = H * 2 ** level
    spl = pf.alpha_functions(table)
    es, kappa = pf.eta_star(1500.0, OMEGA, ell)
    a = [float(spl[f](es)) for f in range(5)]
    mu = 1.0 + (0.9j if op == 1 else 0.0)
    d = pf.shell_coefficients(a, mu * kappa ** 2)[0] / ell ** 2
    th = [np.pi * np.arange(1, n) / n for n in dims]
    TZ, TY, TX = np.meshgrid(th[2], th[1], th[0], indexing="ij")
    bhat = pf.symbol(a, mu * kappa ** 2, ell, np.stack([TX, TY, TZ], -1)).reshape(-1)
    Xi = pf.jacobi_polynomial(bhat, d, w, nJ)
    np.testing.assert_allclose(bhat * Xi, 1 - (1 - w * bhat / d) ** nJ, rtol=1e-12)   # telescoping
    Sx, Sy, Sz = (pf.sine_basis(n) for n in dims)
    Phi = np.kron(Sz, np.kron(Sy, Sx))
    rng = np.random.default_rng(level + nJ)
    coef = rng.standard_normal(len(bhat)) + 1j * rng.standard_normal(len(bhat))
    g = np.zeros(Hh.shape(level), complex)
    g[1:-1, 1:-1, 1:-1] = (Phi @ coef).reshape([s - 2 for s in Hh.shape(level)])
    y = Hh.jacobi(level, op, g, nJ, w)
    expect = (Phi @ (Xi * coef)).reshape([s - 2 for s in Hh.shape(level)])
    np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1], expect, rtol=1e-11, atol=1e-12 * np.abs(expect).max())


def test_jacobi_is_literal_sweep_with_pml(oracle_lib, table):
    """With PML and variable c, y1 = w D^-1 g and y2 = y1 + w D^-1 (g - H y1)."""
    n, npml = 12, 2
    vel = grf_velocity(n, n, n, seed=3, corr_len=3.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, npml, table)
    rng = np.random.default_rng(0)
    g = rng.standard_normal(Hh.shape(0)) + 1j * rng.standard_normal(Hh.shape(0))
    g[0], g[-1], g[:, 0], g[:, -1], g[:, :, 0], g[:, :, -1] = 0, 0, 0, 0, 0, 0
    D = Hh.apply(0, 3, np.ones(Hh.shape(0), complex))
    inner = (slice(1, -1),) * 3
    y1 = np.zeros_like(g)
    y1[inner] = 0.8 * g[inner] / D[inner]
    r = g - Hh.apply(0, 0, y1)
    y2 = y1.copy()
    y2[inner] += 0.8 * r[inner] / D[inner]
    np.testing.assert_allclose(Hh.jacobi(0, 0, g, 2, 0.8), y2, rtol=1e-13, atol=1e-15)
