"""twmg oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes + numpy) to the plain FP64 CPU multigrid in
``twmg_oracle.c``.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2110_08389_amd``) and never imports it.

What is here, with the passage of arXiv 2110.08389 each part follows:

* ``coords``            -- Section 5, eq. (tanh) / eq. (tanh_inv), and the sinh
                           centre clustering of the 2049^2 workload.
* ``coefs``             -- Section 2, W/E (S/N, B/T) coefficients of problem (DP).
* ``Hierarchy``         -- Section 4 grid sequence, the smoothers of Section 3
                           (tweed, wireframe, checkerboard, zebra, alternating
                           schemes) and Section 7 (3D tweed; 3D alternating-
                           direction zebra as x, y, z sweeps), the V/W cycle,
                           full/half weighting and bilinear/trilinear transfer.
* ``spectral_radius``   -- Section 5, eq. (Mh2h): rho of the two-grid operator.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "twmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TWEED, WIREFRAME, CHECKER, ZEBRA_X, ZEBRA_Y, ZEBRA_Z, ADZ, ALT_TW = range(8)
UNIFORM, TANH_WALL, TANH_CENTRE, SINH_CENTRE = range(4)
BLK_POINT, BLK_PATH, BLK_SPIDER, BLK_RING = range(4)
SMOOTHERS = {"tweed": TWEED, "wireframe": WIREFRAME, "checkerboard": CHECKER,
             "zebra_x": ZEBRA_X, "zebra_y": ZEBRA_Y, "zebra_z": ZEBRA_Z,
             "adz": ADZ, "alt_tw": ALT_TW}
STRETCH = {"uniform": UNIFORM, "tanh_wall": TANH_WALL, "tanh_centre": TANH_CENTRE,
           "sinh_centre": SINH_CENTRE}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off: no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_coords.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, dp]
        L.orc_coefs.argtypes = [C.c_int, dp, dp, dp]
        L.orc_coefs_sigma.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_create.argtypes = [C.c_int, ip, C.POINTER(dp), C.POINTER(dp), C.c_int, C.c_int, C.c_int]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_nlevels.argtypes = [C.c_void_p]
        L.orc_level_shape.argtypes = [C.c_void_p, C.c_int, ip]
        L.orc_level_coefs.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp, dp]
        L.orc_smooth.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_int, C.c_int, C.c_int]
        L.orc_apply.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_residual.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        L.orc_restrict.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_int]
        L.orc_prolong_add.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_coarse_solve.argtypes = [C.c_void_p, dp, dp]
        L.orc_cycle.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_resnorm.argtypes = [C.c_void_p, dp, dp]
        L.orc_resnorm.restype = C.c_double
        L.orc_solve.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                dp, ip]
        L.orc_direct.argtypes = [C.c_void_p, dp, dp]
        L.orc_twogrid.argtypes = [C.c_void_p, dp, C.c_int, C.c_int]
        L.orc_nblocks.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_block_info.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, ip, ip]
        L.orc_block_points.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, ip]
        L.orc_block_system.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp]
        L.orc_solve_block.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp, dp, C.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int))


def set_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops (same-colour blocks, node
    loops); the results are bitwise identical for every count."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def coords(kind, param: float, n: int, L: float = 1.0) -> np.ndarray:
    """Node coordinates x_0..x_n (Section 5 eq. (tanh), eq. (tanh_inv); sinh)."""
    k = STRETCH[kind] if isinstance(kind, str) else kind
    x = np.zeros(n + 1)
    if lib().orc_coords(k, float(param), n, float(L), _dp(x)) != 0:
        raise ValueError("bad stretching")
    return x


def coefs(x: np.ndarray, sigma=None):
    """Section 2 coefficients (lo = W/S/B, hi = E/N/T) on node coordinates x;
    with sigma (one value per cell) the flux form of problem (CP) with that
    axis-wise conductivity."""
    n = len(x) - 1
    lo = np.zeros(n + 1)
    hi = np.zeros(n + 1)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if sigma is None:
        lib().orc_coefs(n, _dp(x), _dp(lo), _dp(hi))
    else:
        sg = np.ascontiguousarray(sigma, dtype=np.float64)
        assert sg.shape == (n,)
        lib().orc_coefs_sigma(n, _dp(x), _dp(sg), _dp(lo), _dp(hi))
    return lo, hi


class Hierarchy:
    """Multigrid hierarchy on a stretched tensor grid (Section 4).

    ``coords`` is a list of 2 or 3 coordinate arrays (finest level).  Arrays
    passed to the methods are full node arrays shaped ``(nz+1, ny+1, nx+1)``
    (3D) or ``(ny+1, nx+1)`` (2D), row-major with x fastest; the boundary
    entries of ``u`` hold the Dirichlet data.
    """

    def __init__(self, coord_list, smoother="tweed", transpose=False, maxlev=0, sigma=None):
        self.dim = len(coord_list)
        self.n = [len(c) - 1 for c in coord_list]
        self._coords = [np.ascontiguousarray(c, dtype=np.float64) for c in coord_list]
        ptrs = (C.POINTER(C.c_double) * 3)(*[_dp(c) for c in self._coords],
                                           *([None] * (3 - self.dim)))
        # optional axis-wise conductivity: sigma[a] holds one value per cell
        # of axis a (None: 1 on that axis)
        self._sig = [None if sigma is None or sigma[a] is None
                     else np.ascontiguousarray(sigma[a], dtype=np.float64) for a in range(self.dim)]
        for a, sg in enumerate(self._sig):
            if sg is not None and sg.shape != (self.n[a],):
                raise ValueError("sigma: one value per cell on each axis")
        sptrs = (C.POINTER(C.c_double) * 3)(*[_dp(sg) if sg is not None else None for sg in self._sig],
                                            *([None] * (3 - self.dim)))
        n3 = np.array(self.n + [0] * (3 - self.dim), dtype=np.int32)
        sm = SMOOTHERS[smoother] if isinstance(smoother, str) else smoother
        self.smoother = sm
        self.h = lib().orc_create(self.dim, _ip(n3), ptrs, sptrs, sm, int(transpose), int(maxlev))
        if not self.h:
            raise ValueError("oracle: cannot build hierarchy")
        self.nlev = lib().orc_nlevels(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    # -- shapes -----------------------------------------------------------
    def level_n(self, lv):
        n = np.zeros(3, dtype=np.int32)
        lib().orc_level_shape(self.h, lv, _ip(n))
        return [int(v) for v in n[: self.dim]]

    def shape(self, lv=0):
        return tuple(v + 1 for v in reversed(self.level_n(lv)))

    def zeros(self, lv=0):
        return np.zeros(self.shape(lv))

    def level_coefs(self, lv, axis):
        n = self.level_n(lv)[axis]
        x, lo, hi = np.zeros(n + 1), np.zeros(n + 1), np.zeros(n + 1)
        lib().orc_level_coefs(self.h, lv, axis, _dp(x), _dp(lo), _dp(hi))
        return x, lo, hi

    def interior_mask(self, lv=0):
        m = np.ones(self.shape(lv), dtype=bool)
        for ax in range(self.dim):
            sl = [slice(None)] * self.dim
            sl[self.dim - 1 - ax] = 0
            m[tuple(sl)] = False
            sl[self.dim - 1 - ax] = -1
            m[tuple(sl)] = False
        return m

    # -- operations ---------------------------------------------------------
    def apply(self, u, lv=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        lib().orc_apply(self.h, lv, _dp(u), _dp(out))
        return out

    def residual(self, u, f, lv=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        d = np.zeros_like(u)
        lib().orc_residual(self.h, lv, _dp(u), _dp(f), _dp(d))
        return d

    def restrict(self, d, lv=0, half=False):
        d = np.ascontiguousarray(d, dtype=np.float64)
        fc = self.zeros(lv + 1)
        lib().orc_restrict(self.h, lv, _dp(d), _dp(fc), int(half))
        return fc

    def prolong_add(self, ec, uf, lv=0):
        """uf += P ec (in place on a copy; returns it)."""
        ec = np.ascontiguousarray(ec, dtype=np.float64)
        uf = np.array(uf, dtype=np.float64, order="C")
        lib().orc_prolong_add(self.h, lv, _dp(ec), _dp(uf))
        return uf

    def smooth(self, u, f, nu=1, lv=0, dense=False, reverse=False):
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        rc = lib().orc_smooth(self.h, lv, _dp(u), _dp(f), int(nu), int(dense), int(reverse))
        if rc:
            raise RuntimeError(f"oracle smooth failed ({rc})")
        return u

    def coarse_solve(self, u, f):
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().orc_coarse_solve(self.h, _dp(u), _dp(f))
        return u

    def cycle(self, u, f, nu1=2, nu2=2, gamma=1, half=False):
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        rc = lib().orc_cycle(self.h, _dp(u), _dp(f), int(nu1), int(nu2), int(gamma), int(half))
        if rc:
            raise RuntimeError(f"oracle cycle failed ({rc})")
        return u

    def resnorm(self, u, f):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        return lib().orc_resnorm(self.h, _dp(u), _dp(f))

    def solve(self, u, f, nu1=2, nu2=2, gamma=1, tol=1e-10, max_cycles=100):
        """Cycles from the given u until the relative infinity-norm defect < tol.
        Returns (u, cycles, history, status)."""
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        hist = np.zeros(max(1, max_cycles))
        st = C.c_int(0)
        k = lib().orc_solve(self.h, _dp(u), _dp(f), int(nu1), int(nu2), int(gamma), float(tol),
                            int(max_cycles), _dp(hist), C.byref(st))
        return u, int(k), hist[:k].copy(), int(st.value)

    def direct(self, u, f):
        """Banded-LU solve of the finest level (boundary values of u are used)."""
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        if lib().orc_direct(self.h, _dp(u), _dp(f)):
            raise RuntimeError("direct solve failed")
        return u

    def twogrid(self, e, nu, half=False):
        e = np.array(e, dtype=np.float64, order="C")
        if lib().orc_twogrid(self.h, _dp(e), int(nu), int(half)):
            raise RuntimeError("twogrid needs a two-level hierarchy")
        return e

    # -- blocks ---------------------------------------------------------------
    def nblocks(self, lv=0, slot=0):
        return lib().orc_nblocks(self.h, lv, slot)

    def block(self, b, lv=0, slot=0):
        """dict(size, shape, colour, legs, points) of block b (points in solve order)."""
        info = np.zeros(4, dtype=np.int32)
        legs = np.zeros(8, dtype=np.int32)
        lib().orc_block_info(self.h, lv, slot, b, _ip(info), _ip(legs))
        pts = np.zeros(int(info[0]), dtype=np.int32)
        lib().orc_block_points(self.h, lv, slot, b, _ip(pts))
        return dict(size=int(info[0]), shape=int(info[1]), colour=int(info[2]),
                    legs=[int(v) for v in legs[: int(info[3])]], points=pts)

    def blocks(self, lv=0, slot=0):
        return [self.block(b, lv, slot) for b in range(self.nblocks(lv, slot))]

    def block_system(self, b, u, f, lv=0, slot=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.ascontiguousarray(f, dtype=np.float64)
        sz = self.block(b, lv, slot)["size"]
        A = np.zeros((sz, sz))
        r = np.zeros(sz)
        lib().orc_block_system(self.h, lv, slot, b, _dp(u), _dp(f), _dp(A), _dp(r))
        return A, r

    def solve_block(self, b, u, f, lv=0, slot=0, dense=False):
        u = np.array(u, dtype=np.float64, order="C")
        f = np.ascontiguousarray(f, dtype=np.float64)
        if lib().orc_solve_block(self.h, lv, slot, b, _dp(u), _dp(f), int(dense)):
            raise RuntimeError("block solve failed")
        return u


def spectral_radius(coord_list, smoother, nu, half=False, k=6, tol=1e-9):
    """rho(M) for the two-grid operator of Section 5, eq. (Mh2h), computed with
    ARPACK on the oracle's two-grid error propagation (nu1 = nu, nu2 = 0; only
    the sum matters).  The largest-magnitude eigenvalues of a real operator come
    in conjugate pairs, so several are requested and the maximum modulus taken."""
    import scipy.sparse.linalg as sla

    H = Hierarchy(coord_list, smoother, maxlev=2)
    mask = H.interior_mask(0)
    n = int(mask.sum())

    def mv(v):
        e = np.zeros(H.shape(0))
        e[mask] = np.real(v)
        out = H.twogrid(e, nu, half)
        return out[mask]

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
    rng = np.random.default_rng(7)
    vals = sla.eigs(op, k=k, which="LM", tol=tol, ncv=max(2 * k + 1, 30), maxiter=20000,
                    v0=rng.standard_normal(n), return_eigenvectors=False)
    return float(np.max(np.abs(vals)))
