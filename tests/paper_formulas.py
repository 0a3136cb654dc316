"""Closed forms printed in the paper, written out in numpy for the CPU pins.

Each function states the passage it transcribes.  These are used to check the
oracle (and through it the GPU library) against the paper:
plane-wave symbols, the Dirichlet sine-basis diagonalisation, grid-transfer
symbols and the Jacobi polynomial.  Hermite evaluation here goes through
scipy's CubicHermiteSpline, a library routine independent of both
implementations.
"""
import numpy as np
from scipy.interpolate import CubicHermiteSpline


def alpha_functions(table):
    """The eight tabulated functions as scipy cubic Hermite splines (Sec. 2.2)."""
    K = table["K"]
    eta = np.linspace(0.0, table["eta_max"], K + 1)
    return [CubicHermiteSpline(eta, table["value"][f], table["slope"][f]) for f in range(8)]


def eta_star(c, omega, ell):
    """eq. iofd-clamped-coordinate: eta* = min(k ell / 2pi, 0.4), kappa = k ell."""
    kappa = omega / c * ell
    return min(kappa / (2 * np.pi), 0.4), kappa


def shell_coefficients(a, kappa2):
    """eq. iofd-shell-coefficients; kappa2 may carry the shift (1 + i sigma) kappa^2."""
    a1, a2, a3, a4, a5 = a
    C0 = 6 * a4 - kappa2 * a1
    C1 = -a4 + a5 - kappa2 * a2 / 6
    C2 = -a5 / 2 + (1 - a4 - a5) / 2 - kappa2 * a3 / 12
    C3 = -0.75 * (1 - a4 - a5) - kappa2 * (1 - a1 - a2 - a3) / 8
    return C0, C1, C2, C3


def symbol(a, kappa2, ell, theta):
    """eq. shifted-iofd-symbol: ell^-2 [C0 + 2 C1 sum z + 4 C2 sum zz + 8 C3 z1 z2 z3], z = cos theta.
    theta has shape (..., 3)."""
    C0, C1, C2, C3 = shell_coefficients(a, kappa2)
    z = np.cos(theta)
    s1 = z[..., 0] + z[..., 1] + z[..., 2]
    s2 = z[..., 0] * z[..., 1] + z[..., 0] * z[..., 2] + z[..., 1] * z[..., 2]
    s3 = z[..., 0] * z[..., 1] * z[..., 2]
    return (C0 + 2 * C1 * s1 + 4 * C2 * s2 + 8 * C3 * s3) / ell ** 2


def q_symbol(b, theta):
    """Symbol of Q_h, eq. q-shell-coefficients and eq. q-operator."""
    b1, b2, b3 = b
    Q0, Q1, Q2, Q3 = b1, b2 / 6, b3 / 12, (1 - b1 - b2 - b3) / 8
    z = np.cos(theta)
    s1 = z[..., 0] + z[..., 1] + z[..., 2]
    s2 = z[..., 0] * z[..., 1] + z[..., 0] * z[..., 2] + z[..., 1] * z[..., 2]
    s3 = z[..., 0] * z[..., 1] * z[..., 2]
    return Q0 + 2 * Q1 * s1 + 4 * Q2 * s2 + 8 * Q3 * s3


def pml_gamma(x, L, Lpml, gamma_max):
    """eq. pml-profile: gamma = gamma_max [1 - cos(pi d / (2 L_pml))], d = distance into the PML."""
    d = np.maximum(0.0, np.maximum(Lpml - x, x - (L - Lpml)))
    return gamma_max * (1 - np.cos(np.pi * d / (2 * Lpml)))


def pml_second_difference_1d(n, ell, L, Lpml, gamma_max):
    """-(D^pml) of eq. pml-second-difference on the interior nodes 1..n-1 of one axis
    (dense (n-1)x(n-1)); half-node gamma averaged before inversion (Sec. 2.2)."""
    x = np.arange(n + 1) * ell
    g = pml_gamma(x, L, Lpml, gamma_max) if Lpml > 0 else np.zeros(n + 1)
    xin = 1.0 / (1 + 1j * g)
    xih = 1.0 / (1 + 1j * 0.5 * (g[:-1] + g[1:]))
    D = np.zeros((n - 1, n - 1), complex)
    for i in range(1, n):
        r = i - 1
        D[r, r] = xin[i] * (xih[i] + xih[i - 1]) / ell ** 2
        if i + 1 <= n - 1:
            D[r, r + 1] = -xin[i] * xih[i] / ell ** 2
        if i - 1 >= 1:
            D[r, r - 1] = -xin[i] * xih[i - 1] / ell ** 2
    return D


def sine_basis(n):
    """phi_p(i) = sin(pi p i / n) on interior nodes i, p = 1..n-1 (columns)."""
    i = np.arange(1, n)[:, None]
    p = np.arange(1, n)[None, :]
    return np.sin(np.pi * p * i / n)


def transfer_symbol(theta):
    """eq. lfa-transfer-symbol: entries prod_j (1 + cos(theta_j + pi p_j)) / 2, p in {0,1}^3."""
    out = {}
    for p in np.ndindex(2, 2, 2):
        out[p] = np.prod([(1 + np.cos(theta[j] + np.pi * p[j])) / 2 for j in range(3)])
    return out


def jacobi_polynomial(bhat, d, omega, nJ):
    """eq. lfa-bottom-inverse: Xi = (omega / d) sum_{j<nJ} s^j, s = 1 - omega bhat / d."""
    s = 1 - omega * bhat / d
    return omega / d * sum(s ** j for j in range(nJ))
