"""Pins of the oracle's Krylov maps, shifted V-cycle, Algorithm 1 and outer
solve: minimal-residual property against dense least squares, the two-grid
error operator of eq. lfa-shifted-vcycle / eq. lfa-shifted-inverse in the
Dirichlet sine basis, a dense direct solve, and the outgoing Green function."""
import itertools

import numpy as np
import pytest

from tests import paper_formulas as pf
from workloads import homogeneous, grf_velocity, point_source

H = 10.0
OMEGA = 2 * np.pi * 1500.0 / (6 * H)


def _dense(Hh, level, fn):
    """Matrix of a linear map on interior unknowns, column by column."""
    shp = Hh.shape(level)
    n = int(np.prod([s - 2 for s in shp]))
    M = np.zeros((n, n), complex)
    inner = tuple(s - 2 for s in shp)
    for k in range(n):
        e = np.zeros(shp, complex)
        e[tuple(i + 1 for i in np.unravel_index(k, inner))] = 1.0
        M[:, k] = fn(e)[1:-1, 1:-1, 1:-1].reshape(-1)
    assert np.abs(M).max() > 0
    return M


def _embed(Hh, level, v):
    out = np.zeros(Hh.shape(level), complex)
    out[1:-1, 1:-1, 1:-1] = v.reshape([s - 2 for s in Hh.shape(level)])
    return out


def _min_res(A, M, r0, m):
    """argmin over c of ||r0 - A M K c||, K = [r0, AM r0, ..., (AM)^{m-1} r0]; returns M K c."""
    K = [r0]
    for _ in range(m - 1):
        K.append(A @ (M @ K[-1]))
    K = np.stack(K, 1)
    c, *_ = np.linalg.lstsq(A @ (M @ K), r0, rcond=None)
    return M @ (K @ c)


@pytest.fixture(scope="module")
def small(oracle_lib, table):
    vel = grf_velocity(4, 4, 4, seed=21, corr_len=2.0)        # total 8^3 with n_pml = 2
    return oracle_lib.Hierarchy(vel, H, OMEGA, 2, table)


@pytest.mark.parametrize("level,op,nJ,w,m", [(0, 0, 2, 0.8, 2), (0, 1, 2, 0.5, 5), (1, 0, 0, 0.0, 4)])
def test_gmres_minimal_residual(small, level, op, nJ, w, m):
    """Right-preconditioned GMRES(m) from x0 returns x0 + M K c with c the
    least-squares minimiser (dense numpy lstsq)."""
    Hh = small
    A = _dense(Hh, level, lambda e: Hh.apply(level, op, e))
    M = np.eye(A.shape[0]) if nJ == 0 else _dense(Hh, level, lambda e: Hh.jacobi(level, op, e, nJ, w))
    rng = np.random.default_rng(m)
    n = A.shape[0]
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = Hh.gmres(level, op, _embed(Hh, level, g), _embed(Hh, level, x0), m=m, nJ=nJ, wJ=w)
    expect = x0 + _min_res(A, M, g - A @ x0, m)
    np.testing.assert_allclose(x[1:-1, 1:-1, 1:-1].reshape(-1), expect, rtol=1e-9,
                               atol=1e-10 * np.abs(expect).max())


def test_smoother_and_bottom_are_minimal_residual(oracle_lib, table, small):
    """S_h (m_h = 2, J_2(A_h; 0.8)) and C_4h (m_4h = 4, J_2(B_4h; 0.2)) against lstsq."""
    Hh = small
    A = _dense(Hh, 0, lambda e: Hh.apply(0, 0, e))
    M = _dense(Hh, 0, lambda e: Hh.jacobi(0, 0, e, 2, 0.8))
    rng = np.random.default_rng(1)
    n = A.shape[0]
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = Hh.smooth(_embed(Hh, 0, g), _embed(Hh, 0, x0))
    np.testing.assert_allclose(x[1:-1, 1:-1, 1:-1].reshape(-1), x0 + _min_res(A, M, g - A @ x0, 2), rtol=1e-9)
    # bottom on a grid with 3^3 interior 4h unknowns
    big = oracle_lib.Hierarchy(grf_velocity(8, 8, 8, seed=22, corr_len=2.0), H, OMEGA, 4, table)
    B4 = _dense(big, 2, lambda e: big.apply(2, 1, e))
    M4 = _dense(big, 2, lambda e: big.jacobi(2, 1, e, 2, 0.2))
    q = rng.standard_normal(B4.shape[0]) + 1j * rng.standard_normal(B4.shape[0])
    e = big.bottom(_embed(big, 2, q))
    np.testing.assert_allclose(e[1:-1, 1:-1, 1:-1].reshape(-1), _min_res(B4, M4, q, 4), rtol=1e-9)


def test_restarted_cycles_compose(small):
    """c restarted cycles equal one cycle started from the previous cycle's result."""
    Hh = small
    rng = np.random.default_rng(4)
    g = rng.standard_normal(Hh.shape(1)) + 1j * rng.standard_normal(Hh.shape(1))
    g[0], g[-1], g[:, 0], g[:, -1], g[:, :, 0], g[:, :, -1] = 0, 0, 0, 0, 0, 0
    x1 = Hh.gmres(1, 0, g, m=3, cycles=1, nJ=2, wJ=0.8)
    x2 = Hh.gmres(1, 0, g, x0=x1, m=3, cycles=1, nJ=2, wJ=0.8)
    np.testing.assert_allclose(Hh.gmres(1, 0, g, m=3, cycles=2, nJ=2, wJ=0.8), x2, rtol=1e-12, atol=1e-14)


def test_vcycle_two_grid_lfa(oracle_lib, table):
    """With an exact 4h solve (m_4h = 27 on 3^3 unknowns), V^sigma_2h on a
    constant-c Dirichlet box is (I - E) B^-1 with
    E = S^n (I - P B_4h^-1 R B) S^n (eq. lfa-shifted-vcycle,
    eq. lfa-shifted-inverse), evaluated in the sine basis, where full
    weighting and linear interpolation couple mode q with its alias n - q."""
    n = 16
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, 1500.0), H, OMEGA, 0, table, params=dict(m_4h=27))
    n2 = n // 2
    sigma, w2, nJ = 0.9, 0.8, 2
    spl = pf.alpha_functions(table)
    mu = 1 + 1j * sigma

    def level_symbol(ell, th):
        es, kappa = pf.eta_star(1500.0, OMEGA, ell)
        a = [float(spl[f](es)) for f in range(5)]
        return pf.symbol(a, mu * kappa ** 2, ell, th), pf.shell_coefficients(a, mu * kappa ** 2)[0] / ell ** 2

    modes = list(itertools.product(range(1, n2), repeat=3))          # (px, py, pz)
    th = np.array([[np.pi * p / n2 for p in m] for m in modes])
    b2, d2 = level_symbol(2 * H, th)
    S = 1 - w2 * b2 / d2
    cmodes = list(itertools.product(range(1, n2 // 2), repeat=3))
    cth = np.array([[np.pi * q / (n2 // 2) for q in m] for m in cmodes])
    b4, _ = level_symbol(4 * H, cth)
    index = {m: i for i, m in enumerate(modes)}
    R = np.zeros((len(cmodes), len(modes)))
    for ci, q in enumerate(cmodes):
        for alias in itertools.product((0, 1), repeat=3):
            p = tuple(q[a] if not alias[a] else n2 - q[a] for a in range(3))
            w = 1.0
            for a in range(3):
                cq = np.cos(np.pi * q[a] / n2)
                w *= 0.5 * (1 + cq) if not alias[a] else -0.5 * (1 - cq)
            R[ci, index[p]] = w
    P = R.T.copy()                      # coefficient-space prolongation (same entries)
    Sn = np.diag(S ** nJ)
    E = Sn @ (np.eye(len(modes)) - P @ np.diag(1 / b4) @ R @ np.diag(b2)) @ Sn
    V_hat = (np.eye(len(modes)) - E) @ np.diag(1 / b2)
    # sine basis in (x fastest) flat order of the interior unknowns
    Sb = pf.sine_basis(n2)
    Phi = np.kron(Sb, np.kron(Sb, Sb))
    # Phi columns are ordered (pz, py, px) with px fastest; map them to the mode list
    col_modes = [(px, py, pz) for pz in range(1, n2) for py in range(1, n2) for px in range(1, n2)]
    perm = [index[m] for m in col_modes]
    Vn = Phi @ V_hat[np.ix_(perm, perm)] @ np.linalg.inv(Phi)
    rng = np.random.default_rng(2)
    q = rng.standard_normal(Phi.shape[0]) + 1j * rng.standard_normal(Phi.shape[0])
    y = Hh.vcycle(_embed(Hh, 1, q))
    expect = Vn @ q
    np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1].reshape(-1), expect, rtol=1e-9, atol=1e-10 * np.abs(expect).max())


def test_k2h_solves_unshifted_coarse_equation(oracle_lib, table):
    """With enough flexible steps, K_2h converges to A_2h^-1 r (unshifted A_2h,
    right preconditioning by the shifted cycle)."""
    vel = grf_velocity(12, 12, 12, seed=5, corr_len=3.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, 2, table, params=dict(m_2h=30, c_2h=2))
    A2 = _dense(Hh, 1, lambda e: Hh.apply(1, 0, e))
    rng = np.random.default_rng(8)
    r = rng.standard_normal(A2.shape[0]) + 1j * rng.standard_normal(A2.shape[0])
    e = Hh.k2h(_embed(Hh, 1, r))
    np.testing.assert_allclose(e[1:-1, 1:-1, 1:-1].reshape(-1), np.linalg.solve(A2, r), rtol=1e-6)


def test_solve_matches_dense_direct(oracle_lib, table):
    """FGMRES + Algorithm 1 converges to the solution of A_h v = Q_h f, u = Q_h v,
    computed by a dense direct solve on a 16^3 grid (3375 unknowns)."""
    vel = grf_velocity(8, 8, 8, seed=6, corr_len=3.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, 4, table)
    A = _dense(Hh, 0, lambda e: Hh.apply(0, 0, e))
    Q = _dense(Hh, 0, lambda e: Hh.apply(0, 2, e))
    f = point_source((16, 16, 16), (7, 9, 8), H)
    fi = f[1:-1, 1:-1, 1:-1].reshape(-1)
    u_direct = Q @ np.linalg.solve(A, Q @ fi)
    u, its, rel, st = Hh.solve(f, 1e-11)
    assert st == 0 and rel <= 1e-11 and its > 0
    np.testing.assert_allclose(u[1:-1, 1:-1, 1:-1].reshape(-1), u_direct, rtol=1e-8,
                               atol=1e-9 * np.abs(u_direct).max())


def test_solve_failure_modes(oracle_lib, table):
    vel = homogeneous(8, 8, 8, 1500.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA, 4, table)
    f = point_source((16, 16, 16), (8, 8, 8), H)
    u, its, rel, st = Hh.solve(f, 1e-14, max_outer=1)
    assert st == 1 and its == 1 and rel > 1e-14
    u, its, rel, st = Hh.solve(np.zeros_like(f), 1e-6)
    assert st == 0 and its == 0 and np.all(u == 0)


@pytest.mark.slow
def test_green_function_64(oracle_lib, table):
    """Homogeneous medium, point source h^-3 at the centre (eq. point-source):
    the field matches the outgoing Green function e^{ikr}/(4 pi r) in the
    distance-scaled relative l1 metric of Sec. 5.1 on the 4h receiver lattice
    (64^3 total, 10 PML cells, 6 points per wavelength, tol 1e-6)."""
    n, npml = 44, 10
    c = 1500.0
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, c), H, OMEGA, npml, table)
    N = n + 2 * npml
    s = N // 2
    f = point_source((N, N, N), (s, s, s), H)
    u, its, rel, st = Hh.solve(f, 1e-6)
    assert st == 0 and rel <= 1e-6
    k = OMEGA / c
    z, y, x = np.meshgrid(*(np.arange(N + 1),) * 3, indexing="ij")
    r = H * np.sqrt((x - s) ** 2 + (y - s) ** 2 + (z - s) ** 2)
    rs = np.maximum(r, 1e-9)
    G = np.exp(1j * k * rs) / (4 * np.pi * rs)
    phys = lambda v: (v >= npml) & (v <= N - npml)  # noqa: E731
    mask = phys(x) & phys(y) & phys(z) & (r >= 2 * np.pi / k) & (x % 4 == 0) & (y % 4 == 0) & (z % 4 == 0)
    W = r[mask]
    err = (np.abs(W * (G - u).real[mask]).sum() / np.abs(W * G.real[mask]).sum() +
           np.abs(W * (G - u).imag[mask]).sum() / np.abs(W * G.imag[mask]).sum())
    assert err < 5e-3, err
    # the solution is invariant under the 48 symmetries of the cube
    for perm in itertools.permutations(range(3)):
        np.testing.assert_allclose(np.transpose(u, perm), u, rtol=1e-6, atol=1e-9 * np.abs(u).max())
    np.testing.assert_allclose(u[::-1], u, rtol=1e-6, atol=1e-9 * np.abs(u).max())
