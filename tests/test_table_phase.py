"""Acceptance of the IOFD coefficient table (an input of the method, handed to
both implementations) against the diagnostics the paper prints for its own
table (Sec. 4, "Phase Compatibility of the Physical Grids", and the bounds
stated with eq. shifted-iofd-symbol).

q_l(d; nu) is the normalised numerical wavenumber: the root in [0.9, 1.1] of
the interior symbol a_l(q k l d) (eq. normalized-numerical-wavenumber), found by
50 bisection steps, with k = 2 pi / (nu h), the table evaluated at
eta* = min(k l / 2 pi, 0.4) and the physical k l in the mass term.  The
paper's values at nu = 6 (eq. iofd-phase-matching) are bounds the table must
meet: max|q_h - 1| <= 2.96e-6, max|q_2h - 1| <= 3.27e-4,
max|q_2h - q_h| <= 3.24e-4, and h^2 d_h^0 >= 3.519 for nu in [6, 24],
mass symbol >= 0.489 and a_1 >= 0.588 on [0, 0.4].  Printed values are
compared at their last printed digit.  Hermite evaluation uses scipy.
"""
import itertools

import numpy as np
import pytest

from tests import paper_formulas as pf


def sector_directions(n=3000):
    """Unit directions folded into the symmetry sector d1 >= d2 >= d3 >= 0
    (the symbol is invariant under the 48 cube symmetries), plus the axis,
    face-diagonal and body-diagonal directions."""
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    d = -np.sort(-np.abs(d), axis=1)
    sp = np.array([[1, 0, 0], [1, 1, 0], [1, 1, 1]], float)
    return np.vstack([d, sp / np.linalg.norm(sp, axis=1, keepdims=True)])


def normalised_wavenumber(spl, ratio, nu, dirs):
    """q_l(d; nu) for level spacing l = ratio * h (eq. normalized-numerical-wavenumber)."""
    kappa = 2 * np.pi * ratio / nu
    es = min(kappa / (2 * np.pi), 0.4)
    a = [float(spl[f](es)) for f in range(5)]

    def sym(q):
        return pf.symbol(a, kappa ** 2, 1.0, q[:, None] * kappa * dirs)

    lo = np.full(len(dirs), 0.9)
    hi = np.full(len(dirs), 1.1)
    f_lo = sym(lo)
    assert np.all(np.sign(f_lo) != np.sign(sym(hi))), "root not bracketed in [0.9, 1.1]"
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        f_mid = sym(mid)
        left = np.sign(f_mid) == np.sign(f_lo)
        lo = np.where(left, mid, lo)
        f_lo = np.where(left, f_mid, f_lo)
        hi = np.where(left, hi, mid)
    return 0.5 * (lo + hi)


@pytest.fixture(scope="module")
def spl(table):
    return pf.alpha_functions(table)


def test_phase_matching_at_six_points_per_wavelength(spl):
    dirs = sector_directions()
    qh = normalised_wavenumber(spl, 1, 6.0, dirs)
    q2h = normalised_wavenumber(spl, 2, 6.0, dirs)
    e_h, e_2h, e_x = np.abs(qh - 1).max(), np.abs(q2h - 1).max(), np.abs(q2h - qh).max()
    print(f"max|q_h-1| = {e_h:.3e}, max|q_2h-1| = {e_2h:.3e}, max|q_2h-q_h| = {e_x:.3e}")
    assert e_h <= 2.965e-6
    assert e_2h <= 3.275e-4
    assert e_x <= 3.245e-4


def test_fine_grid_mismatch_shrinks_with_sampling(spl):
    """The fine-coarse mismatch is largest at the shortest wavelength and does
    not grow as the local sampling nu increases over [6, 24]."""
    dirs = sector_directions(800)
    mism = [np.abs(normalised_wavenumber(spl, 2, nu, dirs) - normalised_wavenumber(spl, 1, nu, dirs)).max()
            for nu in (6, 8, 10, 12, 16, 20, 24)]
    assert mism[0] == max(mism)
    assert all(b <= a * 1.05 for a, b in zip(mism, mism[1:])), mism


def test_jacobi_diagonal_and_mass_bounds(spl):
    nus = np.linspace(6, 24, 361)
    d = []
    for nu in nus:
        kappa = 2 * np.pi / nu
        es = min(kappa / (2 * np.pi), 0.4)
        a = [float(spl[f](es)) for f in range(5)]
        d.append(pf.shell_coefficients(a, kappa ** 2)[0])       # h^2 d_h^0 = C_0
    print(f"min h^2 d_h^0 = {min(d):.5f}")
    assert min(d) >= 3.5185
    eta = np.linspace(0, 0.4, 801)
    a1, a2, a3 = (spl[f](eta) for f in range(3))
    assert a1.min() >= 0.5875
    for z in itertools.product((-1.0, 0.0, 1.0), repeat=3):
        s1, s2, s3 = sum(z), z[0] * z[1] + z[0] * z[2] + z[1] * z[2], z[0] * z[1] * z[2]
        m = a1 + a2 / 3 * s1 + a3 / 3 * s2 + (1 - a1 - a2 - a3) * s3
        assert m.min() >= 0.4885, (z, m.min())
