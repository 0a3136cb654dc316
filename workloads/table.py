"""Loading and packing of the IOFD coefficient table (node values and slopes).

Packed layout handed to both implementations (``table_flat``): float64 array
of length ``(K+1) * 8 * 2`` ordered ``[node k][function f][value, slope]``,
functions ``alpha1..alpha5, beta1..beta3``, nodes ``eta_k = k * 0.4 / K``.
Slopes are d/d(eta).
"""
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ETA_MAX = 0.4
NFUNC = 8


def load_iofd_table(path=None):
    """Return the derived table as a dict with arrays value[8][K+1], slope[8][K+1]."""
    path = path or os.path.join(_HERE, "iofd_table.json")
    with open(path) as f:
        t = json.load(f)
    return {
        "K": int(t["K"]),
        "eta_max": float(t["eta_max"]),
        "value": np.asarray(t["value"], dtype=np.float64),
        "slope": np.asarray(t["slope"], dtype=np.float64),
    }


def table_flat(table):
    """Pack a table dict into the ``[node][function][value, slope]`` float64 layout."""
    v = np.asarray(table["value"], dtype=np.float64)
    s = np.asarray(table["slope"], dtype=np.float64)
    assert v.shape == s.shape and v.shape[0] == NFUNC
    return np.ascontiguousarray(np.stack([v.T, s.T], axis=-1).reshape(-1))


def random_table(seed, K=40, amplitude=0.05):
    """A seeded smooth perturbation of the derived table (for parity tests only).

    Exercises the Hermite evaluation with nonzero slopes everywhere and a
    non-identity amplitude correction (beta).
    """
    base = load_iofd_table()
    rng = np.random.default_rng(seed)
    Kb = base["K"]
    eta_b = np.linspace(0, ETA_MAX, Kb + 1)
    eta = np.linspace(0, ETA_MAX, K + 1)
    value = np.empty((NFUNC, K + 1))
    slope = np.empty((NFUNC, K + 1))
    for f in range(NFUNC):
        value[f] = np.interp(eta, eta_b, base["value"][f]) + amplitude * rng.standard_normal(K + 1)
        slope[f] = amplitude * 10 * rng.standard_normal(K + 1)
    value[5] = 0.8 + 0.1 * rng.standard_normal(K + 1)     # beta1
    value[6] = 0.15 + 0.05 * rng.standard_normal(K + 1)   # beta2
    value[7] = 0.03 + 0.02 * rng.standard_normal(K + 1)   # beta3
    return {"K": K, "eta_max": ETA_MAX, "value": value, "slope": slope}


def constant_table(alpha, beta=(1.0, 0.0, 0.0), K=4):
    """Table whose functions are constant in eta (all slopes zero)."""
    vals = list(alpha) + list(beta)
    value = np.array([[v] * (K + 1) for v in vals], dtype=np.float64)
    return {"K": K, "eta_max": ETA_MAX, "value": value, "slope": np.zeros_like(value)}
