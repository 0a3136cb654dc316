"""ctypes front end of the FP64 oracle (helm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its binding.

All grid functions are numpy complex128 arrays of shape (Nz+1, Ny+1, Nx+1)
for the level's (Nx, Ny, Nz) intervals.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "helm_oracle.c")

OP_A, OP_B, OP_Q, OP_DIAG_A, OP_DIAG_B = 0, 1, 2, 3, 4

# Fixed solver configuration of the paper's performance table.
DEFAULT_PARAMS = dict(sigma=0.9, omega_h=0.8, omega_2h=0.8, omega_4h=0.2, gamma_max=1.119058,
                      nJ_h=2, nJ_2h=2, nJ_4h=2, m_h=2, c_2h=2, m_2h=10, m_4h=4, m_out=5, pml_variant=0)
_PARAM_ORDER = ["sigma", "omega_h", "omega_2h", "omega_4h", "gamma_max", "nJ_h", "nJ_2h", "nJ_4h",
                "m_h", "c_2h", "m_2h", "m_4h", "m_out", "pml_variant"]


def build(force=False):
    """Compile liboracle.so with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        L.or_create.argtypes = [P, I, I, I, D, D, I, P, I, D, P, ctypes.POINTER(P)]
        L.or_destroy.argtypes = [P]
        L.or_destroy.restype = None
        L.or_dims.argtypes = [P, I, P]
        L.or_level_velocity.argtypes = [P, I, P]
        L.or_level_xi.argtypes = [P, I, I, P, P]
        L.or_apply.argtypes = [P, I, I, P, P]
        L.or_apply_at.argtypes = [P, I, I, P, P, ctypes.c_longlong, P]
        L.or_residual.argtypes = [P, I, I, P, P, P]
        L.or_restrict.argtypes = [P, I, P, P]
        L.or_prolong.argtypes = [P, I, P, P]
        L.or_jacobi.argtypes = [P, I, I, P, I, D, P]
        L.or_gmres.argtypes = [P, I, I, I, D, P, P, I, I]
        for name in ("or_bottom", "or_vcycle", "or_k2h", "or_precond"):
            getattr(L, name).argtypes = [P, P, P]
        L.or_smooth.argtypes = [P, P, P, P]
        L.or_solve.argtypes = [P, P, D, I, P, P, P]
        L.or_apply_t.argtypes = [P, I, I, P, P]
        L.or_apply_dm.argtypes = [P, I, P, P]
        L.or_grad.argtypes = [P, P, P, D, P, P, P]
        _lib = L
    return _lib


def _c(a, dtype=np.complex128):
    return np.ascontiguousarray(a, dtype=dtype)


class Hierarchy:
    """The three grid levels (h, 2h, 4h) of one problem, held by the oracle."""

    def __init__(self, vel_phys, h, omega, n_pml, table, params=None):
        from workloads.table import table_flat
        vel = np.ascontiguousarray(vel_phys, dtype=np.float32)
        nz, ny, nx = (s - 1 for s in vel.shape)
        self.params = dict(DEFAULT_PARAMS)
        if params:
            self.params.update(params)
        pv = np.array([float(self.params[k]) for k in _PARAM_ORDER], dtype=np.float64)
        self._tab = table_flat(table)
        self.K = int(table["K"])
        self.h, self.omega, self.n_pml = float(h), float(omega), int(n_pml)
        self.phys = (nx, ny, nz)
        ptr = ctypes.c_void_p()
        rc = lib().or_create(vel.ctypes.data, nx, ny, nz, self.h, self.omega, self.n_pml,
                             self._tab.ctypes.data, self.K, float(table["eta_max"]), pv.ctypes.data,
                             ctypes.byref(ptr))
        if rc != 0:
            raise ValueError(f"or_create failed ({rc})")
        self._p = ptr

    def close(self):
        if self._p:
            lib().or_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self, level):
        d = np.zeros(3, dtype=np.int32)
        lib().or_dims(self._p, level, d.ctypes.data)
        return tuple(int(v) for v in d)

    def shape(self, level):
        nx, ny, nz = self.dims(level)
        return (nz + 1, ny + 1, nx + 1)

    def zeros(self, level):
        return np.zeros(self.shape(level), dtype=np.complex128)

    def velocity(self, level):
        out = np.zeros(self.shape(level), dtype=np.float64)
        lib().or_level_velocity(self._p, level, out.ctypes.data)
        return out

    def xi_inv(self, level, axis):
        n = self.dims(level)[axis]
        node = np.zeros(n + 1, np.complex128)
        half = np.zeros(n, np.complex128)
        lib().or_level_xi(self._p, level, axis, node.ctypes.data, half.ctypes.data)
        return node, half

    def apply(self, level, op, x):
        x = _c(x)
        y = self.zeros(level)
        rc = lib().or_apply(self._p, level, op, x.ctypes.data, y.ctypes.data)
        assert rc == 0
        return y

    def apply_at(self, level, op, x, flat_nodes):
        x = _c(x)
        nodes = np.ascontiguousarray(flat_nodes, dtype=np.int64)
        y = np.zeros(len(nodes), dtype=np.complex128)
        rc = lib().or_apply_at(self._p, level, op, x.ctypes.data, nodes.ctypes.data, len(nodes), y.ctypes.data)
        assert rc == 0
        return y

    def residual(self, level, op, g, x):
        g, x = _c(g), _c(x)
        r = self.zeros(level)
        assert lib().or_residual(self._p, level, op, g.ctypes.data, x.ctypes.data, r.ctypes.data) == 0
        return r

    def restrict(self, level, fine):
        fine = _c(fine)
        c = self.zeros(level + 1)
        assert lib().or_restrict(self._p, level, fine.ctypes.data, c.ctypes.data) == 0
        return c

    def prolong(self, level, coarse):
        coarse = _c(coarse)
        f = self.zeros(level - 1)
        assert lib().or_prolong(self._p, level, coarse.ctypes.data, f.ctypes.data) == 0
        return f

    def jacobi(self, level, op, g, nJ, wJ):
        g = _c(g)
        y = self.zeros(level)
        assert lib().or_jacobi(self._p, level, op, g.ctypes.data, int(nJ), float(wJ), y.ctypes.data) == 0
        return y

    def gmres(self, level, op, g, x0=None, m=4, cycles=1, nJ=0, wJ=0.0):
        g = _c(g)
        x = self.zeros(level) if x0 is None else _c(x0).copy()
        steps = lib().or_gmres(self._p, level, op, int(nJ), float(wJ), g.ctypes.data, x.ctypes.data, int(m),
                               int(cycles))
        assert steps >= 0
        return x

    def _map(self, name, level, arg):
        arg = _c(arg)
        out = self.zeros(level)
        assert getattr(lib(), name)(self._p, arg.ctypes.data, out.ctypes.data) == 0
        return out

    def bottom(self, q4):
        return self._map("or_bottom", 2, q4)

    def vcycle(self, q2):
        return self._map("or_vcycle", 1, q2)

    def k2h(self, r2):
        return self._map("or_k2h", 1, r2)

    def precond(self, r):
        return self._map("or_precond", 0, r)

    def smooth(self, g, x0=None):
        g = _c(g)
        x0 = self.zeros(0) if x0 is None else _c(x0)
        x = self.zeros(0)
        assert lib().or_smooth(self._p, g.ctypes.data, x0.ctypes.data, x.ctypes.data) == 0
        return x

    def solve(self, f, tol, max_outer=0):
        f = _c(f)
        u = self.zeros(0)
        its = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        st = lib().or_solve(self._p, f.ctypes.data, float(tol), int(max_outer), u.ctypes.data,
                            ctypes.byref(its), ctypes.byref(rel))
        return u, int(its.value), float(rel.value), int(st)

    def apply_t(self, level, op, x):
        """op^T x (op A or B on any level, Q on level 0)."""
        x = _c(x)
        y = self.zeros(level)
        assert lib().or_apply_t(self._p, level, op, x.ctypes.data, y.ctypes.data) == 0
        return y

    def apply_dm(self, op, x):
        """y_i = (d op / d m_i x)_i on the fine level (op A or Q), m = 1/c^2."""
        x = _c(x)
        y = self.zeros(0)
        assert lib().or_apply_dm(self._p, op, x.ctypes.data, y.ctypes.data) == 0
        return y

    def grad(self, f, s, tol):
        """dJ/dm at the physical nodes for the adjoint source s (dJ = Re sum conj(s) du)."""
        f, s = _c(f), _c(s)
        nx, ny, nz = self.phys
        g = np.zeros((nz + 1, ny + 1, nx + 1), dtype=np.float64)
        its = np.zeros(2, dtype=np.int32)
        rel = np.zeros(2, dtype=np.float64)
        st = lib().or_grad(self._p, f.ctypes.data, s.ctypes.data, float(tol), g.ctypes.data, its.ctypes.data,
                           rel.ctypes.data)
        return g, its, rel, int(st)
