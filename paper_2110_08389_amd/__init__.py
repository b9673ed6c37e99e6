"""twmg: tweed / wireframe geometric multigrid on MI355X (gfx950).

Thin Python binding of ``libtwmg.so`` (C ABI declared in ``include/twmg.h``).
The binding only marshals arguments: every step of the solver runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.  If the
library has not been built this package raises on import -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtwmg.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EHIP, MG_ENOTCONV, MG_EDIVERGED, MG_EUNSUPPORTED = range(7)
STRETCH = {"uniform": 0, "tanh_wall": 1, "tanh_centre": 2, "sinh_centre": 3, "explicit": 4}
SMOOTHER = {"tweed": 0, "wireframe": 1, "checkerboard": 2, "zebra_x": 3, "zebra_y": 4, "zebra_z": 5,
            "adz": 6, "alt_tw": 7}
PRECISION = {"fp64": 0, "fp32_ir": 1}
MG_INITIAL_GUESS = 1


class mg_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3), ("batch", C.c_int)]


class mg_stretching(C.Structure):
    _fields_ = [("kind", C.c_int * 3), ("param", C.c_double * 3), ("coords", C.POINTER(C.c_double) * 3),
                ("sigma", C.POINTER(C.c_double) * 3)]


class mg_options(C.Structure):
    _fields_ = [("smoother", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int), ("gamma", C.c_int),
                ("precision", C.c_int), ("max_cycles", C.c_int), ("flags", C.c_uint)]


class mg_stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("rel_res", C.c_double), ("res0", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int), ("ms", C.c_double)]


class TwmgError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = capi().mg_strerror(code).decode() if _capi is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})")


_capi = None

# entry points: (name, argtypes, restype)
_SIGS = [
    ("mg_setup", [C.POINTER(mg_grid), C.POINTER(mg_stretching), C.POINTER(mg_options), C.c_void_p,
                  C.POINTER(C.c_void_p)], C.c_int),
    ("mg_destroy", [C.c_void_p], None),
    ("mg_set_stream", [C.c_void_p, C.c_void_p], C.c_int),
    ("mg_set_options", [C.c_void_p, C.POINTER(mg_options)], C.c_int),
    ("mg_workspace_bytes", [C.c_void_p], C.c_size_t),
    ("mg_bind_workspace", [C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    ("mg_levels", [C.c_void_p, C.POINTER(C.c_int)], C.c_int),
    ("mg_level_shape", [C.c_void_p, C.c_int, C.POINTER(C.c_int)], C.c_int),
    ("mg_level_coefs", [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_vcycle", [C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_solve", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(mg_stats)], C.c_int),
    ("mg_solve_adjoint", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(mg_stats)], C.c_int),
    ("mg_bc_grad", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_residual_norm", [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    ("mg_residual_norm_noalloc", [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_smooth", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    ("mg_smooth_f32", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    ("mg_residual", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    ("mg_residual_restrict", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int],
     C.c_int),
    ("mg_prolong_add", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_level_array_len", [C.c_void_p, C.c_int, C.POINTER(C.c_longlong)], C.c_int),
    ("mg_to_layout", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_from_layout", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    ("mg_half_sweep", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int], C.c_int),
    ("mg_strerror", [C.c_int], C.c_char_p),
    # test hooks (include/twmg_debug.h)
    ("mg_debug_table_info", [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)], C.c_int),
    ("mg_debug_setup_host", [C.POINTER(mg_grid), C.POINTER(mg_stretching), C.POINTER(mg_options),
                             C.POINTER(C.c_void_p)], C.c_int),
    ("mg_debug_host_smooth", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    ("mg_debug_host_smooth_layout", [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
]
ENTRY_POINTS = [s[0] for s in _SIGS]


def capi():
    """The loaded C library (ctypes), with argument types declared."""
    global _capi
    if _capi is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libtwmg.so not built ({LIB_PATH}); run __graft_entry__.build() first")
        lib = C.CDLL(LIB_PATH)
        for name, args, res in _SIGS:
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _capi = lib
    return _capi


def _check(rc, what):
    if rc != MG_OK:
        raise TwmgError(rc, what)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Solver:
    """One grid hierarchy (mg_setup) and its solve entry points.

    Arrays are torch tensors on the GPU, full node arrays shaped
    ``(batch, [nz+1,] ny+1, nx+1)`` (the batch axis may be omitted when
    batch = 1), float64 unless an entry point says otherwise.
    """

    def __init__(self, n, L=None, stretch=("uniform", 0.0), smoother="tweed", nu1=2, nu2=2, gamma=1,
                 precision="fp64", max_cycles=200, batch=1, coords=None, sigma=None, device=None, stream=None):
        import torch

        self.torch = torch
        self.dim = len(n)
        self.n = list(n)
        self.batch = batch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        g = mg_grid()
        g.dim = self.dim
        for a in range(self.dim):
            g.n[a] = int(n[a])
            g.L[a] = float(L[a]) if L is not None else 1.0
        g.batch = int(batch)
        st = mg_stretching()
        stretches = stretch if isinstance(stretch, (list, tuple)) and isinstance(stretch[0], (list, tuple)) \
            else [stretch] * self.dim
        self._coord_bufs = []
        for a in range(self.dim):
            kind, par = stretches[a]
            st.kind[a] = STRETCH[kind]
            st.param[a] = float(par)
            if kind == "explicit":
                buf = (C.c_double * (n[a] + 1))(*[float(v) for v in coords[a]])
                self._coord_bufs.append(buf)
                st.coords[a] = C.cast(buf, C.POINTER(C.c_double))
            if sigma is not None and sigma[a] is not None:
                if len(sigma[a]) != n[a]:
                    raise ValueError("sigma: one conductivity per cell on each axis")
                buf = (C.c_double * n[a])(*[float(v) for v in sigma[a]])
                self._coord_bufs.append(buf)
                st.sigma[a] = C.cast(buf, C.POINTER(C.c_double))
        self.opts = mg_options()
        self.opts.smoother = SMOOTHER[smoother]
        self.opts.nu1, self.opts.nu2, self.opts.gamma = int(nu1), int(nu2), int(gamma)
        self.opts.precision = PRECISION[precision]
        self.opts.max_cycles = int(max_cycles)
        self.opts.flags = 0
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.stream = s
            h = C.c_void_p()
            _check(capi().mg_setup(C.byref(g), C.byref(st), C.byref(self.opts), C.c_void_p(s.cuda_stream),
                                   C.byref(h)), "mg_setup")
            self.h = h
            nbytes = capi().mg_workspace_bytes(self.h)
            # torch owns the workspace (256-byte aligned by the caching allocator)
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            _check(capi().mg_bind_workspace(self.h, _ptr(self._ws), nbytes), "mg_bind_workspace")
        nl = C.c_int()
        _check(capi().mg_levels(self.h, C.byref(nl)), "mg_levels")
        self.nlevels = nl.value

    def __del__(self):
        if getattr(self, "h", None) is not None and _capi is not None:
            _capi.mg_destroy(self.h)
            self.h = None

    # -- shapes -------------------------------------------------------------
    def level_n(self, lv=0):
        n = (C.c_int * 3)()
        _check(capi().mg_level_shape(self.h, lv, n), "mg_level_shape")
        return [n[a] for a in range(self.dim)]

    def shape(self, lv=0, batched=None):
        s = tuple(v + 1 for v in reversed(self.level_n(lv)))
        if batched or (batched is None and self.batch > 1):
            s = (self.batch,) + s
        return s

    def zeros(self, lv=0, dtype=None):
        return self.torch.zeros(self.shape(lv), dtype=dtype or self.torch.float64, device=self.device)

    def level_coefs(self, lv, axis):
        import numpy as np

        m = self.level_n(lv)[axis] + 1
        x, lo, hi = np.zeros(m), np.zeros(m), np.zeros(m)
        _check(capi().mg_level_coefs(self.h, lv, axis, x.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                                     hi.ctypes.data_as(C.c_void_p)), "mg_level_coefs")
        return x, lo, hi

    def _arg(self, t, lv=0, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        want = self.shape(lv)
        if t.dtype != dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dtype} tensor on {self.device}")
        if tuple(t.shape) != want and tuple(t.shape) != self.shape(lv, batched=True):
            raise ValueError(f"shape {tuple(t.shape)} != {want}")
        return _ptr(t)

    def set_options(self, **kw):
        for k, v in kw.items():
            if k == "smoother":
                v = SMOOTHER[v]
            if k == "precision":
                v = PRECISION[v]
            setattr(self.opts, k, int(v))
        _check(capi().mg_set_options(self.h, C.byref(self.opts)), "mg_set_options")

    # -- solver ---------------------------------------------------------------
    def solve(self, f, bc=None, tol=1e-10, u=None, history=64):
        """Returns (u, stats-dict).  u is created (zeros) unless given."""
        if u is None:
            u = self.zeros()
        st = mg_stats()
        hist = (C.c_double * max(1, history))()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_cap = history
        rc = capi().mg_solve(self.h, self._arg(u), self._arg(f), self._arg(bc) if bc is not None else C.c_void_p(0),
                             float(tol), C.byref(st))
        if rc not in (MG_OK, MG_ENOTCONV, MG_EDIVERGED):
            _check(rc, "mg_solve")
        return u, dict(cycles=st.cycles, status=st.status, rel_res=st.rel_res, res0=st.res0, ms=st.ms,
                       history=[hist[k] for k in range(min(st.cycles, history))])

    def solve_adjoint(self, w, tol=1e-10, lam=None, history=64):
        if lam is None:
            lam = self.zeros()
        st = mg_stats()
        hist = (C.c_double * max(1, history))()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_cap = history
        rc = capi().mg_solve_adjoint(self.h, self._arg(lam), self._arg(w), float(tol), C.byref(st))
        if rc not in (MG_OK, MG_ENOTCONV, MG_EDIVERGED):
            _check(rc, "mg_solve_adjoint")
        return lam, dict(cycles=st.cycles, status=st.status, rel_res=st.rel_res, res0=st.res0, ms=st.ms,
                         history=[hist[k] for k in range(min(st.cycles, history))])

    def bc_grad(self, lam, w):
        g = self.zeros()
        _check(capi().mg_bc_grad(self.h, self._arg(lam), self._arg(w), self._arg(g)), "mg_bc_grad")
        return g

    def vcycle(self, u, f):
        _check(capi().mg_vcycle(self.h, self._arg(u), self._arg(f)), "mg_vcycle")
        return u

    def residual_norm(self, u, f):
        out = C.c_double()
        _check(capi().mg_residual_norm(self.h, self._arg(u), self._arg(f), C.byref(out)), "mg_residual_norm")
        return out.value

    def residual_norm_noalloc(self, u, f, out):
        """mg_residual_norm_noalloc: enqueues the batch's largest defect norm
        into out[0] (a float64 device tensor); no allocation, no sync."""
        if out.dtype != self.torch.float64 or out.device != self.device or out.numel() < 1:
            raise ValueError("out: a float64 device tensor of at least one element")
        _check(capi().mg_residual_norm_noalloc(self.h, self._arg(u), self._arg(f), _ptr(out)),
               "mg_residual_norm_noalloc")
        return out

    # -- kernel-level entry points ------------------------------------------------
    def smooth(self, u, f, nu=1, lv=0, adjoint=False):
        if u.dtype == self.torch.float32:
            _check(capi().mg_smooth_f32(self.h, lv, self._arg(u, lv, u.dtype), self._arg(f, lv, u.dtype), nu,
                                        int(adjoint)), "mg_smooth_f32")
        else:
            _check(capi().mg_smooth(self.h, lv, self._arg(u, lv), self._arg(f, lv), nu, int(adjoint)), "mg_smooth")
        return u

    def residual(self, u, f, lv=0, adjoint=False):
        d = self.zeros(lv)
        _check(capi().mg_residual(self.h, lv, self._arg(u, lv), self._arg(f, lv), self._arg(d, lv), int(adjoint)),
               "mg_residual")
        return d

    def residual_restrict(self, u, f, lv=0, adjoint=False):
        fc = self.zeros(lv + 1)
        uc = self.torch.full(self.shape(lv + 1), 7.0, dtype=self.torch.float64, device=self.device)
        _check(capi().mg_residual_restrict(self.h, lv, self._arg(u, lv), self._arg(f, lv), self._arg(fc, lv + 1),
                                           self._arg(uc, lv + 1), int(adjoint)), "mg_residual_restrict")
        return fc, uc

    def prolong_add(self, ec, u, lv=0):
        _check(capi().mg_prolong_add(self.h, lv, self._arg(ec, lv + 1), self._arg(u, lv)), "mg_prolong_add")
        return u

    # -- device layout (see mg_level_array_len in include/twmg.h) -------------
    def array_len(self, lv=0):
        n = C.c_longlong()
        _check(capi().mg_level_array_len(self.h, lv, C.byref(n)), "mg_level_array_len")
        return n.value

    def to_layout(self, x, lv=0):
        """Row-major node array(s) of level lv -> a flat tensor in the level's device layout."""
        out = self.torch.zeros(self.batch * self.array_len(lv), dtype=self.torch.float64, device=self.device)
        _check(capi().mg_to_layout(self.h, lv, self._arg(x, lv), _ptr(out)), "mg_to_layout")
        return out

    def from_layout(self, xd, lv=0):
        out = self.zeros(lv)
        if xd.numel() != self.batch * self.array_len(lv) or xd.dtype != self.torch.float64 or xd.device != self.device:
            raise ValueError("from_layout: expected a float64 device tensor of batch * array_len(lv) elements")
        _check(capi().mg_from_layout(self.h, lv, _ptr(xd.contiguous()), _ptr(out)), "mg_from_layout")
        return out

    def half_sweep(self, ud, fd, colour, lv=0, slot=0, adjoint=False):
        """One half-sweep (one colour) on device-layout arrays from to_layout."""
        n = self.batch * self.array_len(lv)
        for t in (ud, fd):
            if t.numel() != n or t.dtype != self.torch.float64 or t.device != self.device or not t.is_contiguous():
                raise ValueError("half_sweep: expected contiguous float64 device tensors in the device layout")
        _check(capi().mg_half_sweep(self.h, lv, _ptr(ud), _ptr(fd), int(slot), int(colour), int(adjoint)),
               "mg_half_sweep")
        return ud


def _autograd():
    import torch

    class MGSolve(torch.autograd.Function):
        """u = A^{-1}(f, g): forward multigrid solve; backward runs the adjoint
        multigrid solve (transposed operator, reversed colour order) and the
        boundary-data gradient.  Gradients: dL/df = lam (zero on boundary
        nodes), dL/dbc = w_B - A_IB^T lam (zero on interior nodes)."""

        @staticmethod
        def forward(ctx, f, bc, solver, tol):
            u, st = solver.solve(f.contiguous(), bc.contiguous(), tol)
            if st["status"] != MG_OK:
                raise TwmgError(st["status"], "MGSolve.forward")
            ctx.solver = solver
            ctx.tol = tol
            return u

        @staticmethod
        def backward(ctx, gu):
            s = ctx.solver
            w = gu.contiguous()
            lam, st = s.solve_adjoint(w, ctx.tol)
            if st["status"] != MG_OK:
                raise TwmgError(st["status"], "MGSolve.backward")
            gbc = s.bc_grad(lam, w)
            return lam, gbc, None, None

    return MGSolve


_MGSolve = None


def mg_solve_autograd(f, bc, solver, tol=1e-10):
    """Differentiable solve: torch.autograd.Function around mg_solve."""
    global _MGSolve
    if _MGSolve is None:
        _MGSolve = _autograd()
    return _MGSolve.apply(f, bc, solver, tol)
