"""Python binding of the HIP library (include/helm.h): argument marshalling only.

Every step of the computation runs in libhelm.so on the GPU; PyTorch provides
device memory (torch tensors) and the stream.  Grid functions are torch
complex tensors of shape (Nz+1, Ny+1, Nx+1) on the level's total grid:
complex64 for precision "fp32" and "mixed", complex128 for "fp64".
"""
import ctypes
import json
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhelm.so")
_DEFAULT_TABLE = os.path.join(os.path.dirname(_HERE), "workloads", "iofd_table.json")

HELM_OK, HELM_NOT_CONVERGED = 0, 1
OP_A, OP_B, OP_Q, OP_DIAG_A, OP_DIAG_B = 0, 1, 2, 3, 4
OP_AT, OP_BT, OP_QT, OP_DA, OP_DQ = 5, 6, 7, 8, 9   # transposes and row derivatives in m = 1/c^2
FP64, FP32, MIXED = 0, 1, 2
_PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}

_c_int, _c_double, _c_void_p, _c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class HelmOptions(ctypes.Structure):
    _fields_ = [("struct_size", _c_int), ("precision", _c_int),
                ("sigma", _c_double), ("omega_h", _c_double), ("omega_2h", _c_double), ("omega_4h", _c_double),
                ("gamma_max", _c_double),
                ("nJ_h", _c_int), ("nJ_2h", _c_int), ("nJ_4h", _c_int),
                ("m_h", _c_int), ("c_2h", _c_int), ("m_2h", _c_int), ("m_4h", _c_int), ("m_out", _c_int),
                ("max_outer", _c_int),
                ("iofd_table", _c_void_p), ("iofd_K", _c_int), ("stream", _c_void_p),
                ("tile_tz", _c_int), ("tile_split", _c_int), ("lanes", _c_int), ("pml_variant", _c_int),
                ("batch", _c_int)]


EXPORTED = ["helm_default_options", "helm_workspace_size", "helm_setup", "helm_solve", "helm_solve_checkpoint",
            "helm_grad",
            "helm_grad_workspace_size", "helm_grad_to_velocity", "helm_destroy",
            "helm_last_error", "helm_dims", "helm_apply", "helm_residual", "helm_residual_restrict", "helm_jacobi",
            "helm_restrict",
            "helm_prolong_add", "helm_bottom", "helm_vcycle", "helm_coarse_solve", "helm_smooth", "helm_precond",
            "helm_vec_dots", "helm_vec_orthonormalize", "helm_vec_dots_static", "helm_tiles_save",
            "helm_tiles_load"]

_lib = None


def lib():
    """Load libhelm.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing; build it with `python -m paper_2608_22946_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        P, I, D = _c_void_p, _c_int, _c_double
        L.helm_default_options.argtypes = [ctypes.POINTER(HelmOptions)]
        L.helm_workspace_size.argtypes = [I, I, I, I, ctypes.POINTER(HelmOptions), ctypes.POINTER(_c_size_t)]
        L.helm_setup.argtypes = [P, I, I, I, D, D, I, ctypes.POINTER(HelmOptions), P, _c_size_t, ctypes.POINTER(P)]
        L.helm_solve.argtypes = [P, P, I, D, P, P, P]
        L.helm_solve_checkpoint.argtypes = [P, P, I, D, P, P, P, P]
        L.helm_grad.argtypes = [P, P, P, P, I, D, P, P, _c_size_t, P, P]
        L.helm_grad_workspace_size.argtypes = [P, ctypes.POINTER(_c_size_t)]
        L.helm_grad_to_velocity.argtypes = [P, P, P]
        L.helm_destroy.argtypes = [P]
        L.helm_destroy.restype = None
        L.helm_last_error.argtypes = [P]
        L.helm_last_error.restype = ctypes.c_char_p
        L.helm_dims.argtypes = [P, I, P]
        L.helm_apply.argtypes = [P, I, I, P, P]
        L.helm_residual.argtypes = [P, I, I, P, P, P]
        L.helm_residual_restrict.argtypes = [P, I, I, P, P, P]
        L.helm_jacobi.argtypes = [P, I, I, P, I, D, P]
        L.helm_restrict.argtypes = [P, I, P, P]
        L.helm_prolong_add.argtypes = [P, I, P, P]
        for name in ("helm_bottom", "helm_vcycle", "helm_coarse_solve", "helm_precond"):
            getattr(L, name).argtypes = [P, P, P]
        L.helm_smooth.argtypes = [P, P, P, P]
        L.helm_vec_dots.argtypes = [P, I, I, P, P, P]
        L.helm_vec_orthonormalize.argtypes = [P, I, I, P, P, P]
        L.helm_vec_dots_static.argtypes = [I, ctypes.c_longlong, I, P, P, P, P]
        L.helm_tiles_save.argtypes = [ctypes.c_char_p]
        L.helm_tiles_load.argtypes = [ctypes.c_char_p, P]
        _lib = L
    return _lib


def default_options():
    o = HelmOptions()
    rc = lib().helm_default_options(ctypes.byref(o))
    assert rc == HELM_OK
    return o


def load_table(path=None):
    with open(path or _DEFAULT_TABLE) as f:
        t = json.load(f)
    return {"K": int(t["K"]), "eta_max": float(t["eta_max"]), "value": np.asarray(t["value"], np.float64),
            "slope": np.asarray(t["slope"], np.float64)}


def table_flat(table):
    v = np.asarray(table["value"], np.float64)
    s = np.asarray(table["slope"], np.float64)
    return np.ascontiguousarray(np.stack([v.T, s.T], axis=-1).reshape(-1))


class HelmError(RuntimeError):
    pass


def _check(rc, H=None, allow_not_converged=False):
    if rc == HELM_OK or (allow_not_converged and rc == HELM_NOT_CONVERGED):
        return rc
    msg = lib().helm_last_error(H).decode()
    raise HelmError(f"helm error {rc}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Hierarchy:
    """Operator hierarchy of one problem (helm_setup) and the calls on it."""

    def __init__(self, velocity, h, omega, n_pml, precision="fp32", table=None, device="cuda", **params):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        vel = torch.as_tensor(velocity, dtype=torch.float32).to(self.device).contiguous()
        nz, ny, nx = (s - 1 for s in vel.shape)
        o = default_options()
        if precision not in _PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
        o.precision = _PRECISIONS[precision]
        for k, v in params.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self._tab = table_flat(table if table is not None else load_table())
        o.iofd_K = len(self._tab) // 16 - 1
        o.iofd_table = self._tab.ctypes.data
        o.stream = torch.cuda.current_stream(self.device).cuda_stream
        self.opt = o
        self.precision = precision
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        nbytes = _c_size_t(0)
        _check(lib().helm_workspace_size(nx, ny, nz, int(n_pml), ctypes.byref(o), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        ws_ptr = self.workspace.data_ptr() + off
        self._vel = vel
        hp = _c_void_p()
        _check(lib().helm_setup(_ptr(vel), nx, ny, nz, float(h), float(omega), int(n_pml), ctypes.byref(o),
                                _c_void_p(ws_ptr), nbytes.value, ctypes.byref(hp)))
        self._h = hp
        self.h, self.omega, self.n_pml = float(h), float(omega), int(n_pml)
        self.phys = (nx, ny, nz)

    # -- bookkeeping ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().helm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self, level):
        d = (ctypes.c_int * 3)()
        _check(lib().helm_dims(self._h, level, d), self._h)
        return tuple(d)

    def shape(self, level):
        nx, ny, nz = self.dims(level)
        return (nz + 1, ny + 1, nx + 1)

    def empty(self, level):
        return torch.empty(self.shape(level), dtype=self.cdtype, device=self.device)

    def zeros(self, level):
        return torch.zeros(self.shape(level), dtype=self.cdtype, device=self.device)

    def _vec(self, t, level):
        if t.dtype != self.cdtype or tuple(t.shape) != self.shape(level) or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError(f"expected a contiguous {self.cdtype} tensor of shape {self.shape(level)} on "
                             f"{self.device}")
        return _ptr(t)

    # -- steps of the hot path -------------------------------------------------
    def apply(self, level, op, x, out=None):
        y = self.empty(level) if out is None else out
        _check(lib().helm_apply(self._h, level, op, self._vec(x, level), self._vec(y, level)), self._h)
        return y

    def residual(self, level, op, g, x, out=None):
        r = self.empty(level) if out is None else out
        _check(lib().helm_residual(self._h, level, op, self._vec(g, level), self._vec(x, level),
                                   self._vec(r, level)), self._h)
        return r

    def jacobi(self, level, op, g, nJ, omega, out=None):
        y = self.empty(level) if out is None else out
        _check(lib().helm_jacobi(self._h, level, op, self._vec(g, level), int(nJ), float(omega),
                                 self._vec(y, level)), self._h)
        return y

    def residual_restrict(self, level, op, g, x, out=None):
        """coarse = R (g - op x), level 0 or 1 -> level + 1 (fused)."""
        c = self.empty(level + 1) if out is None else out
        _check(lib().helm_residual_restrict(self._h, level, op, self._vec(g, level), self._vec(x, level),
                                            self._vec(c, level + 1)), self._h)
        return c

    def restrict(self, level, fine, out=None):
        c = self.empty(level + 1) if out is None else out
        _check(lib().helm_restrict(self._h, level, self._vec(fine, level), self._vec(c, level + 1)), self._h)
        return c

    def prolong_add(self, level, coarse, fine):
        _check(lib().helm_prolong_add(self._h, level, self._vec(coarse, level), self._vec(fine, level - 1)),
               self._h)
        return fine

    def bottom(self, q, out=None):
        e = self.empty(2) if out is None else out
        _check(lib().helm_bottom(self._h, self._vec(q, 2), self._vec(e, 2)), self._h)
        return e

    def vcycle(self, q, out=None):
        y = self.empty(1) if out is None else out
        _check(lib().helm_vcycle(self._h, self._vec(q, 1), self._vec(y, 1)), self._h)
        return y

    def coarse_solve(self, r, out=None):
        e = self.empty(1) if out is None else out
        _check(lib().helm_coarse_solve(self._h, self._vec(r, 1), self._vec(e, 1)), self._h)
        return e

    def smooth(self, g, x0=None, out=None):
        x = self.empty(0) if out is None else out
        x0p = self._vec(x0, 0) if x0 is not None else None
        _check(lib().helm_smooth(self._h, self._vec(g, 0), x0p, self._vec(x, 0)), self._h)
        return x

    def precond(self, r, out=None):
        z = self.empty(0) if out is None else out
        _check(lib().helm_precond(self._h, self._vec(r, 0), self._vec(z, 0)), self._h)
        return z

    def vec_dots(self, level, V, w):
        """(conj(V_j) . w for each j, ||w||^2) accumulated in FP64."""
        k = len(V)
        arr = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in V])
        out = np.zeros(2 * (k + 1), np.float64)
        _check(lib().helm_vec_dots(self._h, level, k, arr, self._vec(w, level), out.ctypes.data), self._h)
        c = out[0::2] + 1j * out[1::2]
        return c[:k], c[k].real

    def vec_orthonormalize(self, level, V, w):
        """In place: w <- (w - V h)/||w - V h||; returns (h, ||w - V h||)."""
        k = len(V)
        arr = (ctypes.c_void_p * k)(*[t.data_ptr() for t in V])
        out = np.zeros(2 * (k + 1), np.float64)
        _check(lib().helm_vec_orthonormalize(self._h, level, k, arr, self._vec(w, level), out.ctypes.data), self._h)
        c = out[0::2] + 1j * out[1::2]
        return c[:k], c[k].real

    def grad(self, f, adj_src, tol, v=None):
        """dJ/dm (m = 1/c^2) at the physical nodes for sources f and adjoint sources s
        (dJ = Re sum conj(s) du, u = Q v, A v = Q f); f and s of shape (nrhs, ...) or a
        single grid function; v (optional, complex128, same leading shape): the forward
        solutions from solve_checkpoint, which skips the forward solves.  Returns (float32
        gradient on the physical grid, forward and adjoint preconditioner calls [nrhs, 2],
        true relative residuals [nrhs, 2], rc)."""
        single = f.dim() == 3
        fb = f.unsqueeze(0) if single else f
        sb = adj_src.unsqueeze(0) if single else adj_src
        for t in (fb, sb):
            if t.dtype != self.cdtype or tuple(t.shape[1:]) != self.shape(0) or not t.is_contiguous() \
                    or t.device != self.device:
                raise ValueError("sources must be contiguous with the level-0 shape and precision dtype")
        if fb.shape != sb.shape:
            raise ValueError("f and adj_src must have the same shape")
        vp = None
        if v is not None:
            vb = v.unsqueeze(0) if v.dim() == 3 else v
            if vb.dtype != torch.complex128 or vb.shape != fb.shape or not vb.is_contiguous() or vb.device != self.device:
                raise ValueError("v must be a contiguous complex128 tensor shaped like f")
            vp = _ptr(vb)
        nrhs = fb.shape[0]
        nbytes = _c_size_t(0)
        _check(lib().helm_grad_workspace_size(self._h, ctypes.byref(nbytes)), self._h)
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        nx, ny, nz = self.phys
        g = torch.empty((nz + 1, ny + 1, nx + 1), dtype=torch.float32, device=self.device)
        its = np.zeros((nrhs, 2), np.int32)
        rel = np.zeros((nrhs, 2), np.float64)
        rc = lib().helm_grad(self._h, _ptr(fb), _ptr(sb), vp, nrhs, float(tol), _ptr(g), _c_void_p(ws_ptr),
                             nbytes.value, its.ctypes.data, rel.ctypes.data)
        _check(rc, self._h, allow_not_converged=True)
        return g, its, rel, rc

    def grad_to_velocity(self, grad_m, out=None):
        """dJ/dc from dJ/dm (m = 1/c^2) on the physical nodes, with the hierarchy's velocity."""
        g = torch.empty_like(grad_m) if out is None else out
        _check(lib().helm_grad_to_velocity(self._h, _ptr(grad_m), _ptr(g)), self._h)
        return g

    def solve_checkpoint(self, f, tol, out=None, v_out=None):
        """solve() that also returns the FP64 forward solutions v (A v = Q f) for grad(v=...)."""
        single = f.dim() == 3
        fb = f.unsqueeze(0) if single else f
        if fb.dtype != self.cdtype or tuple(fb.shape[1:]) != self.shape(0) or not fb.is_contiguous():
            raise ValueError("right-hand sides must be contiguous with the level-0 shape and precision dtype")
        nrhs = fb.shape[0]
        u = torch.empty_like(fb) if out is None else out
        v = torch.empty(fb.shape, dtype=torch.complex128, device=self.device) if v_out is None else v_out
        if v.dtype != torch.complex128 or v.shape != fb.shape or not v.is_contiguous():
            raise ValueError("v_out must be a contiguous complex128 tensor shaped like f")
        its = np.zeros(nrhs, np.int32)
        rel = np.zeros(nrhs, np.float64)
        rc = lib().helm_solve_checkpoint(self._h, _ptr(fb), nrhs, float(tol), _ptr(u), _ptr(v), its.ctypes.data,
                                         rel.ctypes.data)
        _check(rc, self._h, allow_not_converged=True)
        if single:
            return u[0], v[0], int(its[0]), float(rel[0]), rc
        return u, v, its, rel, rc

    def solve(self, f, tol, out=None):
        """u = Q v with A v = Q f; f of shape (nrhs, ...) or a single grid function."""
        single = f.dim() == 3
        fb = f.unsqueeze(0) if single else f
        if fb.dtype != self.cdtype or tuple(fb.shape[1:]) != self.shape(0) or not fb.is_contiguous():
            raise ValueError("right-hand sides must be contiguous with the level-0 shape and precision dtype")
        nrhs = fb.shape[0]
        u = torch.empty_like(fb) if out is None else out
        its = np.zeros(nrhs, np.int32)
        rel = np.zeros(nrhs, np.float64)
        rc = lib().helm_solve(self._h, _ptr(fb), nrhs, float(tol), _ptr(u), its.ctypes.data, rel.ctypes.data)
        _check(rc, self._h, allow_not_converged=True)
        if single:
            return u[0], int(its[0]), float(rel[0]), rc
        return u, its, rel, rc


def vec_dots_static(V, w, out=None):
    """helm_vec_dots_static: (conj(V_j) . w, ||w||^2) in FP64 into a device float64 tensor of
    2 (k + 1) entries (complex pairs), enqueued on torch's current stream, with no allocation
    inside the library (its reduction scratch is a static device array)."""
    k = len(V)
    if w.dtype not in (torch.complex64, torch.complex128) or not w.is_contiguous() or w.device.type != "cuda":
        raise ValueError("w must be a contiguous complex64 / complex128 CUDA tensor")
    for v in V:
        if v.dtype != w.dtype or v.numel() != w.numel() or not v.is_contiguous() or v.device != w.device:
            raise ValueError("every V_j must match w in dtype, size and device")
    if out is None:
        out = torch.empty(2 * (k + 1), dtype=torch.float64, device=w.device)
    elif out.dtype != torch.float64 or out.numel() < 2 * (k + 1) or not out.is_contiguous() or out.device != w.device:
        raise ValueError("out must be a contiguous float64 tensor of at least 2 (k + 1) entries on w's device")
    arr = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in V])
    prec = FP64 if w.dtype == torch.complex128 else FP32
    stream = torch.cuda.current_stream(w.device).cuda_stream
    _check(lib().helm_vec_dots_static(prec, w.numel(), k, arr, _ptr(w), _ptr(out), ctypes.c_void_p(stream)))
    return out


def tiles_save(path):
    """helm_tiles_save: write the stencil tile choices timed (or loaded) so far in this process."""
    _check(lib().helm_tiles_save(os.fsencode(path)))


def tiles_load(path):
    """helm_tiles_load: reuse tile choices saved by an earlier process on the same GPU architecture;
    returns the number of entries added or replaced."""
    n = ctypes.c_int(0)
    _check(lib().helm_tiles_load(os.fsencode(path), ctypes.addressof(n)))
    return n.value


class _Solve(torch.autograd.Function):
    """u = Q_h v, A_h(c) v = Q_h f, differentiable in the physical velocity c through helm_grad
    (the incoming gradient g of a real loss L is the adjoint source: dL = Re sum conj(g) du).
    No gradient flows to f."""

    @staticmethod
    def forward(ctx, vel, f, h, omega, n_pml, tol, kwargs):
        hier = Hierarchy(vel.detach(), h, omega, n_pml, device=f.device, **kwargs)
        u, v, its, rel, rc = hier.solve_checkpoint(f, tol)
        ctx.hier, ctx.tol = hier, tol
        ctx.save_for_backward(f, v)          # checkpointed forward solution: no second forward solve
        return u

    @staticmethod
    def backward(ctx, gu):
        f, v = ctx.saved_tensors
        gm, its, rel, rc = ctx.hier.grad(f, gu.to(f.dtype).contiguous(), ctx.tol, v=v)
        gc = ctx.hier.grad_to_velocity(gm)
        return gc, None, None, None, None, None, None


def solve(vel, f, h, omega, n_pml, tol, **kwargs):
    """Differentiable solve: u (same shape as f) for the physical velocity vel (torch float32 tensor
    of shape (nz+1, ny+1, nx+1); gradients flow to it) and the source f on the total grid.  kwargs go
    to Hierarchy (precision, table, lanes, ...)."""
    return _Solve.apply(vel, f, float(h), float(omega), int(n_pml), float(tol), kwargs)
