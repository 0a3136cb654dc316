"""Offline derivation of the IOFD coefficient table (alpha_1..alpha_5, beta_1..beta_3).

The paper defines the 27-point operator through five functions alpha_j(s) and
the amplitude correction through three functions beta_j(s), s in [0, 0.4],
each a cubic Hermite interpolant of tabulated optimized values taken from an
external publication (Section 2.2, eq. iofd-shell-form and eq. q-operator).
Those tabulated values are not printed in the paper, so this script derives
an alpha table by the criterion the paper names: directional phase-slowness
optimisation of the interior symbol (eq. shifted-iofd-symbol with sigma = 0).

For each table node eta (kappa = 2*pi*eta) the symbol residual
F(theta) = S(theta; a4, a5) - kappa^2 M(theta; a1, a2, a3) is affine in
a = (a1..a5), so three linear programs are solved in turn:

  1. minimise max_d |F(kappa d)| / |kappa d . grad F(kappa d)| over unit
     directions d in the symmetry sector d1 >= d2 >= d3 >= 0 (this is the
     linearised relative phase error |q - 1|, re-weighted three times);
  2. within 1% of that optimum, maximise the smallest value of the mass
     symbol over the 27 cosine vertices (keeps the shifted operators
     B = L - (1 + i sigma) M well separated from singularity);
  3. within 1% / 0.1% of both optima, stay closest (l1) to the solution at
     the neighbouring node (continuation from eta = 0.2 both ways), which
     selects a smooth branch of the otherwise degenerate optimum.

Constraints: all transverse weights (a4, a5/4, (1-a4-a5)/4) and mass weights
(a1, a2/6, a3/12, (1-a1-a2-a3)/8) nonnegative, plus the two bounds the paper
prints for its table (mass symbol >= 0.489 and a1 >= 0.588 on [0, 0.4]).
Slopes are central differences of the same continuation.

The amplitude correction Q_h (eq. q-operator) enters twice, b = Q f and
u = Q v, so along a direction d the far-field amplitude of the discrete point
response relative to the outgoing Green function is q(kappa d)^2 * 2 kappa /
|grad a(kappa d)| (residue of 1/a at its real pole, with q and a the symbols
of Q_h and P_h).  beta is therefore chosen per node to minimise
max_d |q(kappa d; beta) - s(d)| / s(d), s(d) = sqrt(|grad a(kappa d)| / (2 kappa)),
an LP in beta since q is affine in beta.  Q_h is outside every
preconditioner application (Sec. 2.2), so beta only affects the amplitude of
the reconstructed field, not the solver.

This script is not imported by any runtime code; its output,
iofd_table.json, is an input of the method (like the velocity model) that
the solver library and the oracle both receive.

Run:  python workloads/derive_iofd_table.py   (writes workloads/iofd_table.json)
"""
import json
import os
import numpy as np
from scipy.optimize import linprog

ETA_MAX = 0.4
K = 40                      # intervals; nodes eta_k = k * ETA_MAX / K
MASS_MIN = 0.489
A1_MIN = 0.588


def sector_directions(n=4000):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = np.pi * (1 + 5 ** 0.5) * i
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    d = -np.sort(-np.abs(d), axis=1)
    d = np.unique(np.round(d, 6), axis=0)
    sp = np.array([[1, 0, 0], [1, 1, 0], [1, 1, 1]], float)
    sp /= np.linalg.norm(sp, axis=1, keepdims=True)
    return np.vstack([d, sp])


def affine_parts(theta, kappa):
    """F(theta; a) = const + G @ a for the unshifted interior symbol (h = 1)."""
    z = np.cos(theta)
    s = 2.0 * (1.0 - z)
    z1, z2, z3 = z[:, 0], z[:, 1], z[:, 2]
    P = z1 * z2 * z3
    Sz = z1 + z2 + z3
    Szz = z1 * z2 + z1 * z3 + z2 * z3
    trip = [(s[:, 0], z2, z3), (s[:, 1], z1, z3), (s[:, 2], z1, z2)]
    const = sum(sj * zk * zl for sj, zk, zl in trip) - kappa ** 2 * P
    g4 = sum(sj * (1 - zk * zl) for sj, zk, zl in trip)
    g5 = sum(sj * ((zk + zl) / 2 - zk * zl) for sj, zk, zl in trip)
    k2 = kappa ** 2
    G = np.stack([-k2 * (1 - P), -k2 * (Sz / 3 - P), -k2 * (Szz / 3 - P), g4, g5], 1)
    return const, G


def mass_vertex_rows():
    R, C = [], []
    for z1 in (-1, 0, 1):
        for z2 in (-1, 0, 1):
            for z3 in (-1, 0, 1):
                P = z1 * z2 * z3
                R.append([1 - P, (z1 + z2 + z3) / 3 - P, (z1 * z2 + z1 * z3 + z2 * z3) / 3 - P, 0, 0])
                C.append(P)
    return np.array(R, float), np.array(C, float)


def _lp(obj, A, b, bounds):
    res = linprog(obj, A_ub=np.vstack(A), b_ub=np.concatenate(b), bounds=bounds, method="highs",
                  options=dict(primal_feasibility_tolerance=1e-10, dual_feasibility_tolerance=1e-10))
    if not res.success:
        raise RuntimeError(res.message)
    return res.x


def _weights(eta, dirs, a):
    kappa = 2 * np.pi * eta
    if a is None:
        return np.full(len(dirs), 2 * kappa ** 2)
    eps = 1e-6
    th = kappa * dirs
    c1, G1 = affine_parts(th * (1 + eps), kappa)
    c0, G0 = affine_parts(th * (1 - eps), kappa)
    return np.abs((c1 + G1 @ a - c0 - G0 @ a) / (2 * eps))


def solve_node(eta, dirs, a_prev):
    kappa = 2 * np.pi * eta
    const, G = affine_parts(kappa * dirs, kappa)
    R, C = mass_vertex_rows()
    sum_rows = np.array([[0, 0, 0, 1, 1], [1, 1, 1, 0, 0]], float)
    wbox = [(A1_MIN, 1), (0, 1), (0, 1), (0, 1), (0, 1)]
    a = None
    for _ in range(4):                                     # stage 1, IRLS on the true gradient
        w = _weights(eta, dirs, a)
        cs, Gs = const / w, G / w[:, None]
        rs = 1.0 / np.abs(np.hstack([cs[:, None], Gs])).max()
        cs, Gs = cs * rs, Gs * rs
        n = len(dirs)
        A = [np.hstack([Gs, -np.ones((n, 1))]), np.hstack([-Gs, -np.ones((n, 1))]),
             np.hstack([sum_rows, np.zeros((2, 1))]), np.hstack([-R, np.zeros((len(R), 1))])]
        b = [-cs, cs, np.ones(2), C - MASS_MIN]
        x = _lp(np.r_[np.zeros(5), 1.0], A, b, wbox + [(0, None)])
        a, t = x[:5], x[5]
    tstar = t * 1.01
    # stage 2: maximise the mass-symbol margin
    A = [np.hstack([Gs, np.zeros((n, 1))]), np.hstack([-Gs, np.zeros((n, 1))]),
         np.hstack([sum_rows, np.zeros((2, 1))]), np.hstack([-R, np.ones((len(R), 1))])]
    b = [tstar - cs, tstar + cs, np.ones(2), C]
    x = _lp(np.r_[np.zeros(5), -1.0], A, b, wbox + [(None, None)])
    mstar = x[5] - 1e-3
    if a_prev is None:
        return x[:5]
    # stage 3: continuation tie-break
    Z = np.zeros
    A = [np.hstack([Gs, Z((n, 5))]), np.hstack([-Gs, Z((n, 5))]), np.hstack([sum_rows, Z((2, 5))]),
         np.hstack([-R, Z((len(R), 5))]), np.hstack([np.eye(5), -np.eye(5)]),
         np.hstack([-np.eye(5), -np.eye(5)])]
    b = [tstar - cs, tstar + cs, np.ones(2), C - max(mstar, MASS_MIN), a_prev, -a_prev]
    x = _lp(np.r_[np.zeros(5), np.ones(5)], A, b, wbox + [(0, None)] * 5)
    return x[:5]


def q_affine(theta):
    """Symbol of Q_h: q = 1 + sum_j beta_j g_j(theta) (shell weights of eq. q-shell-coefficients)."""
    z = np.cos(theta)
    Sz = z.sum(1)
    Szz = z[:, 0] * z[:, 1] + z[:, 0] * z[:, 2] + z[:, 1] * z[:, 2]
    P = z.prod(1)
    # Q0 = b1, Q1 = b2/6, Q2 = b3/12, Q3 = (1 - b1 - b2 - b3)/8 ; q = Q0 + 2 Q1 Sz + 4 Q2 Szz + 8 Q3 P
    const = P
    G = np.stack([1 - P, Sz / 3 - P, Szz / 3 - P], 1)
    return const, G


def solve_beta(eta, dirs, a, b_prev=None):
    kappa = 2 * np.pi * eta
    eps = 1e-6
    th = kappa * dirs
    c1, G1 = affine_parts(th * (1 + eps), kappa)
    c0, G0 = affine_parts(th * (1 - eps), kappa)
    radial = np.abs((c1 + G1 @ a - c0 - G0 @ a) / (2 * eps)) / kappa     # d . grad a at the pole
    s = np.sqrt(radial / (2 * kappa))
    const, G = q_affine(th)
    cs, Gs = (const - s) / s, G / s[:, None]
    n = len(dirs)
    A = [np.hstack([Gs, -np.ones((n, 1))]), np.hstack([-Gs, -np.ones((n, 1))])]
    b = [-cs, cs]
    x = _lp(np.r_[np.zeros(3), 1.0], A, b, [(-5, 5)] * 3 + [(0, None)])
    if b_prev is None:
        return x[:3]
    tstar = 1.01 * x[3] + 1e-9
    Z = np.zeros
    A = [np.hstack([Gs, Z((n, 3))]), np.hstack([-Gs, Z((n, 3))]),
         np.hstack([np.eye(3), -np.eye(3)]), np.hstack([-np.eye(3), -np.eye(3)])]
    b = [tstar - cs, tstar + cs, b_prev, -b_prev]
    x = _lp(np.r_[np.zeros(3), np.ones(3)], A, b, [(-5, 5)] * 3 + [(0, None)] * 3)
    return x[:3]


def derive():
    dirs = sector_directions()
    etas = np.linspace(0.0, ETA_MAX, K + 1)
    etas_eval = etas.copy()
    etas_eval[0] = 0.002                   # the eta -> 0 limit is taken at a small positive value
    d_eta = 1e-3
    start = K // 2                          # eta = 0.2
    vals = np.zeros((K + 1, 5))
    slopes = np.zeros((K + 1, 5))
    vals[start] = solve_node(etas_eval[start], dirs, None)
    for k in list(range(start + 1, K + 1)) + list(range(start - 1, -1, -1)):
        prev = vals[k - 1] if k > start else vals[k + 1]
        vals[k] = solve_node(etas_eval[k], dirs, prev)
    for k in range(K + 1):
        lo = max(etas_eval[k] - d_eta, 1e-3)
        hi = min(etas_eval[k] + d_eta, ETA_MAX)
        a_lo = solve_node(lo, dirs, vals[k])
        a_hi = solve_node(hi, dirs, vals[k])
        slopes[k] = (a_hi - a_lo) / (hi - lo)
    slopes[0] = 0.0                         # even function of kappa at kappa = 0
    bvals = np.zeros((K + 1, 3))
    bslopes = np.zeros((K + 1, 3))
    bvals[start] = solve_beta(etas_eval[start], dirs, vals[start])
    for k in list(range(start + 1, K + 1)) + list(range(start - 1, -1, -1)):
        prev = bvals[k - 1] if k > start else bvals[k + 1]
        bvals[k] = solve_beta(etas_eval[k], dirs, vals[k], prev)
    for k in range(K + 1):
        lo = max(etas_eval[k] - d_eta, 1e-3)
        hi = min(etas_eval[k] + d_eta, ETA_MAX)
        bslopes[k] = (solve_beta(hi, dirs, vals[k] + slopes[k] * (hi - etas_eval[k]), bvals[k])
                      - solve_beta(lo, dirs, vals[k] + slopes[k] * (lo - etas_eval[k]), bvals[k])) / (hi - lo)
    bslopes[0] = 0.0
    return etas, vals, slopes, bvals, bslopes


def main():
    etas, av, asl, bv, bs = derive()
    value = np.hstack([av, bv])
    slope = np.hstack([asl, bs])
    out = {
        "description": "IOFD Hermite table: node values and d/d(eta) slopes of alpha1..alpha5, beta1..beta3 "
                       "on uniform nodes eta_k = k*eta_max/K",
        "eta_max": ETA_MAX,
        "K": K,
        "functions": ["alpha1", "alpha2", "alpha3", "alpha4", "alpha5", "beta1", "beta2", "beta3"],
        "value": value.T.round(12).tolist(),
        "slope": slope.T.round(10).tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "iofd_table.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
