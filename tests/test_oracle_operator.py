"""Pins of the oracle's level operators (A, B, Q, diagonal) against
closed forms of the paper: plane-wave symbols, sine-basis diagonalisation of
the Dirichlet box, the separable (Kronecker) special case with PML, the
7-point textbook reduction, shell/tensor agreement and cube symmetry."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from tests import paper_formulas as pf
from workloads import constant_table, homogeneous, grf_velocity
from workloads.table import random_table, ETA_MAX

H = 10.0
OMEGA_PPW6 = 2 * np.pi * 1500.0 / (6 * H)


def cubic_table(coeffs, K=8):
    """Table whose functions are exact cubics in eta (values and slopes at nodes)."""
    eta = np.linspace(0, ETA_MAX, K + 1)
    value = np.array([np.polyval(c, eta) for c in coeffs])
    slope = np.array([np.polyval(np.polyder(c), eta) for c in coeffs])
    return {"K": K, "eta_max": ETA_MAX, "value": value, "slope": slope}


CUBICS = [
    [0.3, -0.2, 0.1, 0.70], [0.5, 0.1, -0.3, 0.12], [-0.4, 0.2, 0.05, 0.11],
    [0.2, -0.1, 0.3, 0.72], [-0.6, 0.3, -0.1, 0.24], [0.1, 0.2, -0.3, 0.85],
    [0.4, -0.5, 0.2, 0.08], [-0.3, 0.1, 0.4, 0.06],
]


def plane_wave(dims, theta):
    Nx, Ny, Nz = dims
    z, y, x = np.meshgrid(np.arange(Nz + 1), np.arange(Ny + 1), np.arange(Nx + 1), indexing="ij")
    return np.exp(1j * (theta[0] * x + theta[1] * y + theta[2] * z))


@pytest.mark.parametrize("level,op,c", [(0, 0, 1500.0), (0, 1, 2300.0), (1, 0, 1900.0), (1, 1, 1500.0),
                                        (2, 1, 1500.0), (2, 0, 4000.0)])
def test_plane_wave_symbol(oracle_lib, level, op, c):
    """Interior rows act on e^{i theta.j} as multiplication by the printed symbol
    (eq. shifted-iofd-symbol); a_j = alpha_j(eta*) with exact cubic alpha, so
    this also pins the cubic Hermite evaluation, the clamp at 0.4 (level 2,
    c = 1500: kappa/2pi = 2/3) and the kept physical kappa in the mass term."""
    tab = cubic_table(CUBICS)
    n = 16
    vel = homogeneous(n, n, n, c)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA_PPW6, 0, tab, params=dict(sigma=0.9))
    dims = Hh.dims(level)
    ell = H * 2 ** level
    es, kappa = pf.eta_star(c, OMEGA_PPW6, ell)
    a = [np.polyval(CUBICS[f], es) for f in range(5)]
    mu = 1.0 + (0.9j if op == 1 else 0.0)
    rng = np.random.default_rng(level * 10 + op)
    for _ in range(3):
        theta = rng.uniform(-np.pi, np.pi, 3)
        x = plane_wave(dims, theta)
        y = Hh.apply(level, op, x)
        sym = pf.symbol(a, mu * kappa ** 2, ell, theta)
        inner = (slice(2, dims[2] - 1), slice(2, dims[1] - 1), slice(2, dims[0] - 1))
        np.testing.assert_allclose(y[inner], sym * x[inner], rtol=1e-12, atol=1e-12 * abs(sym) + 1e-14)


def test_q_symbol(oracle_lib):
    """Q_h acts on e^{i theta.j} by the symbol of eq. q-operator, beta at the fine eta*."""
    tab = cubic_table(CUBICS)
    n = 12
    vel = homogeneous(n, n, n, 1700.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA_PPW6, 2, tab)
    dims = Hh.dims(0)
    es, _ = pf.eta_star(1700.0, OMEGA_PPW6, H)
    b = [np.polyval(CUBICS[f], es) for f in (5, 6, 7)]
    theta = np.array([0.4, -1.3, 2.2])
    x = plane_wave(dims, theta)
    y = Hh.apply(0, 2, x)
    inner = (slice(2, dims[2] - 1), slice(2, dims[1] - 1), slice(2, dims[0] - 1))
    np.testing.assert_allclose(y[inner], pf.q_symbol(b, theta) * x[inner], rtol=1e-13)


def _sine3(dims):
    Sx, Sy, Sz = (pf.sine_basis(n) for n in dims)
    return np.kron(Sz, np.kron(Sy, Sx))


@pytest.mark.parametrize("level,op", [(0, 0), (0, 1), (1, 1)])
def test_dirichlet_sine_diagonalisation(oracle_lib, table, level, op):
    """With no PML and constant c, the Dirichlet-box operator is diagonal in the
    sine basis with eigenvalues symbol(pi p / N) (on every interior row,
    boundary-adjacent rows included)."""
    nx, ny, nz = 12, 8, 16                      # distinct axes catch transposed strides
    vel = homogeneous(nx, ny, nz, 1800.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA_PPW6, 0, table)
    dims = Hh.dims(level)
    ell = H * 2 ** level
    spl = pf.alpha_functions(table)
    es, kappa = pf.eta_star(1800.0, OMEGA_PPW6, ell)
    a = [float(spl[f](es)) for f in range(5)]
    mu = 1.0 + (0.9j if op == 1 else 0.0)
    thx, thy, thz = (np.pi * np.arange(1, n) / n for n in dims)
    TZ, TY, TX = np.meshgrid(thz, thy, thx, indexing="ij")
    lam = pf.symbol(a, mu * kappa ** 2, ell, np.stack([TX, TY, TZ], -1)).reshape(-1)
    Phi = _sine3(dims)
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(len(lam)) + 1j * rng.standard_normal(len(lam))
    x = np.zeros((dims[2] + 1, dims[1] + 1, dims[0] + 1), complex)
    x[1:-1, 1:-1, 1:-1] = (Phi @ coef).reshape(dims[2] - 1, dims[1] - 1, dims[0] - 1)
    y = Hh.apply(level, op, x)
    expect = (Phi @ (lam * coef)).reshape(dims[2] - 1, dims[1] - 1, dims[0] - 1)
    np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1], expect, rtol=1e-11, atol=1e-11 * np.abs(expect).max())
    assert np.all(y[0] == 0) and np.all(y[:, :, -1] == 0)


@pytest.mark.parametrize("op", [0, 1])
def test_separable_kronecker_pml(oracle_lib, op):
    """Separable tables a4 = (1-2t)^2, a5 = 4t(1-2t), a1 = (1-2m)^3,
    a2 = 6m(1-2m)^2, a3 = 12m^2(1-2m) make the PML stencil a sum of Kronecker
    products: sum_j D_j (x) T (x) T - mu k^2 M (x) M (x) M with T = (t, 1-2t, t),
    M = (m, 1-2m, m), D_j the 1-D stretched second difference."""
    t, m = 0.11, 0.07
    alpha = [(1 - 2 * m) ** 3, 6 * m * (1 - 2 * m) ** 2, 12 * m * m * (1 - 2 * m), (1 - 2 * t) ** 2,
             4 * t * (1 - 2 * t)]
    tab = constant_table(alpha)
    nx, ny, nz, npml = 8, 4, 12, 4
    c = 1600.0
    gmax = 1.119058
    vel = homogeneous(nx, ny, nz, c)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA_PPW6, npml, tab, params=dict(gamma_max=gmax))
    dims = Hh.dims(0)
    mu = 1.0 + (0.9j if op == 1 else 0.0)
    k2 = (OMEGA_PPW6 / c) ** 2

    def tri(n, w):
        return sp.diags([w, 1 - 2 * w, w], [-1, 0, 1], shape=(n - 1, n - 1), dtype=complex)

    D = [sp.csr_matrix(pf.pml_second_difference_1d(n, H, n * H, npml * H, gmax)) for n in dims]
    T = [tri(n, t) for n in dims]
    M = [tri(n, m) for n in dims]
    A = (sp.kron(T[2], sp.kron(T[1], D[0])) + sp.kron(T[2], sp.kron(D[1], T[0])) +
         sp.kron(D[2], sp.kron(T[1], T[0])) - mu * k2 * sp.kron(M[2], sp.kron(M[1], M[0])))
    rng = np.random.default_rng(7)
    shp = (dims[2] - 1, dims[1] - 1, dims[0] - 1)
    xi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    x = np.zeros((dims[2] + 1, dims[1] + 1, dims[0] + 1), complex)
    x[1:-1, 1:-1, 1:-1] = xi
    y = Hh.apply(0, op, x)
    expect = (A @ xi.reshape(-1)).reshape(shp)
    np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1], expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_pml_profile_values(oracle_lib, table):
    """Per-axis 1/xi tables: 1 in the physical region, gamma_max at the outer
    boundary, the cosine profile at half depth, half nodes from averaged gamma."""
    gmax = 1.119058
    npml = 8
    Hh = oracle_lib.Hierarchy(homogeneous(16, 16, 16, 1500.0), H, OMEGA_PPW6, npml, table,
                              params=dict(gamma_max=gmax))
    node, half = Hh.xi_inv(0, 0)
    N = 32
    assert np.allclose(node[npml:N - npml + 1], 1.0, atol=0, rtol=0)
    np.testing.assert_allclose(node[0], 1 / (1 + 1j * gmax), rtol=1e-15)
    np.testing.assert_allclose(node[N], 1 / (1 + 1j * gmax), rtol=1e-15)
    g4 = gmax * (1 - np.cos(np.pi / 4))                # d = L_pml / 2 at node 4
    np.testing.assert_allclose(node[4], 1 / (1 + 1j * g4), rtol=1e-15)
    gam = lambda v: (1 / v - 1).imag                     # noqa: E731
    np.testing.assert_allclose(gam(half[3]), 0.5 * (gam(node[3]) + gam(node[4])), rtol=1e-13)
    # 2h level: same physical thickness (4 coarse layers)
    node2, _ = Hh.xi_inv(1, 0)
    np.testing.assert_allclose(node2[2], node[4], rtol=1e-15)


@pytest.mark.parametrize("variant", [1, 2])
def test_pml_profile_alternative_readings(oracle_lib, table, variant):
    """The two alternative readings of eq. pml-profile / eq. pml-second-difference kept
    for the Green-function study: (1) half-node gamma at the half node's own distance
    instead of the mean of the node values; (2) the profile reaches gamma_max at
    d = L_pml - h and stays there.  Values from the closed forms."""
    gmax, npml, N = 1.119058, 8, 32
    Hh = oracle_lib.Hierarchy(homogeneous(16, 16, 16, 1500.0), H, OMEGA_PPW6, npml, table,
                              params=dict(gamma_max=gmax, pml_variant=variant))
    node, half = Hh.xi_inv(0, 0)
    gam = lambda v: (1 / v - 1).imag                     # noqa: E731
    assert np.allclose(node[npml:N - npml + 1], 1.0, atol=0, rtol=0)
    if variant == 1:
        # half node between nodes 3 and 4: d = 4.5 h of L_pml = 8 h
        np.testing.assert_allclose(gam(half[3]), gmax * (1 - np.cos(np.pi * 4.5 / 16)), rtol=1e-13)
        np.testing.assert_allclose(gam(node[4]), gmax * (1 - np.cos(np.pi / 4)), rtol=1e-13)
        # the physical side of the first PML cell: d = h / 2
        np.testing.assert_allclose(gam(half[npml - 1]), gmax * (1 - np.cos(np.pi * 0.5 / 16)), rtol=1e-13)
    else:
        # L' = 7 h: node 4 has d = 4 h; nodes 1 and 0 (d >= 7 h) carry gamma_max
        np.testing.assert_allclose(gam(node[4]), gmax * (1 - np.cos(np.pi * 4 / 14)), rtol=1e-13)
        np.testing.assert_allclose(gam(node[1]), gmax, rtol=1e-13)
        np.testing.assert_allclose(gam(node[0]), gmax, rtol=1e-13)
        np.testing.assert_allclose(gam(half[3]), 0.5 * (gam(node[3]) + gam(node[4])), rtol=1e-13)


def test_seven_point_reduction(oracle_lib):
    """(a1..a5) = (1, 0, 0, 1, 0) gives the textbook 7-point -Delta_h - k^2."""
    tab = constant_table([1.0, 0.0, 0.0, 1.0, 0.0])
    n = 12
    c = 1700.0
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, c), H, OMEGA_PPW6, 0, tab)
    rng = np.random.default_rng(3)
    x = np.zeros((n + 1,) * 3, complex)
    x[1:-1, 1:-1, 1:-1] = rng.standard_normal((n - 1,) * 3) + 1j * rng.standard_normal((n - 1,) * 3)
    y = Hh.apply(0, 0, x)
    k2 = (OMEGA_PPW6 / c) ** 2
    lap = 6 * x[1:-1, 1:-1, 1:-1] - (x[:-2, 1:-1, 1:-1] + x[2:, 1:-1, 1:-1] + x[1:-1, :-2, 1:-1] +
                                    x[1:-1, 2:, 1:-1] + x[1:-1, 1:-1, :-2] + x[1:-1, 1:-1, 2:])
    np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1], lap / H ** 2 - k2 * x[1:-1, 1:-1, 1:-1], rtol=1e-13,
                               atol=1e-16)


def test_shell_form_outside_pml(oracle_lib, table):
    """Away from the PML the tensor-product rows equal the shell form
    (eq. iofd-shell-form, eq. iofd-shell-coefficients) with the coefficients
    evaluated at the row centre, for variable velocity."""
    nx, ny, nz, npml = 20, 16, 12, 4
    vel = grf_velocity(nx, ny, nz, seed=11, corr_len=4.0)
    Hh = oracle_lib.Hierarchy(vel, H, OMEGA_PPW6, npml, table)
    dims = Hh.dims(0)
    cl = Hh.velocity(0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(cl.shape) + 1j * rng.standard_normal(cl.shape)
    x[0], x[-1], x[:, 0], x[:, -1], x[:, :, 0], x[:, :, -1] = 0, 0, 0, 0, 0, 0
    for op, mu in ((0, 1.0), (1, 1 + 0.9j)):
        y = Hh.apply(0, op, x)
        spl = pf.alpha_functions(table)
        for _ in range(40):
            i = [rng.integers(npml + 1, dims[a] - npml) for a in range(3)]
            es, kappa = pf.eta_star(cl[i[2], i[1], i[0]], OMEGA_PPW6, H)
            a = [float(spl[f](es)) for f in range(5)]
            C = pf.shell_coefficients(a, mu * kappa ** 2)
            acc = 0
            for d in itertools.product((-1, 0, 1), repeat=3):
                acc += C[sum(map(abs, d))] * x[i[2] + d[2], i[1] + d[1], i[0] + d[0]]
            np.testing.assert_allclose(y[i[2], i[1], i[0]], acc / H ** 2, rtol=1e-12)


def test_boundary_values_ignored(oracle_lib, table):
    """Boundary nodes carry u = 0: values stored there are read as zero and
    every operator writes zero on the boundary."""
    n, npml = 12, 2
    Hh = oracle_lib.Hierarchy(grf_velocity(n, n, n, seed=1, corr_len=3.0), H, OMEGA_PPW6, npml, table)
    x = np.zeros(Hh.shape(0), complex)
    x[0], x[-1], x[:, 0], x[:, -1], x[:, :, 0], x[:, :, -1] = 1, 2j, 3, 4, 5j, 6
    for op in (0, 1, 2, 3, 4):
        assert np.all(Hh.apply(0, op, x) == 0)


def test_diagonal(oracle_lib, table):
    """The diagonal operator equals the centre coefficient C0 / ell^2 outside the PML."""
    n = 12
    c = 2100.0
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, c), H, OMEGA_PPW6, 0, table)
    spl = pf.alpha_functions(table)
    for level, op, mu in ((0, 3, 1.0), (1, 4, 1 + 0.9j)):
        ell = H * 2 ** level
        es, kappa = pf.eta_star(c, OMEGA_PPW6, ell)
        a = [float(spl[f](es)) for f in range(5)]
        C0 = pf.shell_coefficients(a, mu * kappa ** 2)[0]
        x = np.ones(Hh.shape(level), complex)
        y = Hh.apply(level, op, x)
        np.testing.assert_allclose(y[1:-1, 1:-1, 1:-1], C0 / ell ** 2, rtol=1e-13)


def test_cube_symmetry(oracle_lib, table):
    """Constant c in a cube with PML: the operator commutes with the 48 axis
    reflections and permutations (catches PML half-node index slips)."""
    n, npml = 8, 4
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, 1500.0), H, OMEGA_PPW6, npml, table)
    rng = np.random.default_rng(9)
    shp = Hh.shape(0)
    x = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    x[0], x[-1], x[:, 0], x[:, -1], x[:, :, 0], x[:, :, -1] = 0, 0, 0, 0, 0, 0
    y = Hh.apply(0, 1, x)
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((False, True), repeat=3):
            def g(v):
                v = np.transpose(v, perm)
                for ax, f in enumerate(flips):
                    if f:
                        v = np.flip(v, ax)
                return v
            np.testing.assert_allclose(Hh.apply(0, 1, g(x)), g(y), rtol=1e-12, atol=1e-12 * np.abs(y).max())


def test_random_table_hermite_against_scipy(oracle_lib):
    """Random (non-derived) tables: shell rows outside the PML match coefficients
    evaluated by scipy's CubicHermiteSpline."""
    tab = random_table(seed=4, K=16)
    n = 12
    c = 1550.0
    Hh = oracle_lib.Hierarchy(homogeneous(n, n, n, c), H, OMEGA_PPW6 * 0.7, 0, tab)
    spl = pf.alpha_functions(tab)
    es, kappa = pf.eta_star(c, OMEGA_PPW6 * 0.7, H)
    a = [float(spl[f](es)) for f in range(5)]
    theta = np.array([0.3, 1.1, -2.0])
    x = plane_wave(Hh.dims(0), theta)
    y = Hh.apply(0, 0, x)
    sym = pf.symbol(a, kappa ** 2, H, theta)
    np.testing.assert_allclose(y[3:-3, 3:-3, 3:-3], sym * x[3:-3, 3:-3, 3:-3], rtol=1e-12)
