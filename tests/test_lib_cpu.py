"""CPU checks of the HIP library (no GPU needed): the C ABI loads and exports
every declared entry point; the host-side setup (coordinates, coefficients,
block tables) matches the oracle; and the block-relaxation kernel's own
per-lane steps, executed sequentially on the host through the test hook,
reproduce the oracle's block Gauss-Seidel sweep."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2110_08389_amd as pkg
from paper_2110_08389_amd import inputs
from tests.helpers import rel_inf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("twmg.h", "twmg_debug.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", txt))
    return names


def test_exports_every_declared_symbol():
    lib = C.CDLL(pkg.LIB_PATH)
    decl = declared_functions()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert decl == set(pkg.ENTRY_POINTS)
    assert pkg.capi().mg_strerror(pkg.MG_ENOTCONV).decode().startswith("not converged")


def host_handle(n, kind, c, smoother, batch=1, sigma=None):
    lib = pkg.capi()
    g = pkg.mg_grid()
    g.dim = len(n)
    for a in range(len(n)):
        g.n[a] = n[a]
        g.L[a] = 1.0
    g.batch = batch
    st = pkg.mg_stretching()
    bufs = []
    for a in range(len(n)):
        st.kind[a] = pkg.STRETCH[kind]
        st.param[a] = c
        if sigma is not None and sigma[a] is not None:
            buf = np.ascontiguousarray(sigma[a], dtype=np.float64)
            bufs.append(buf)
            st.sigma[a] = buf.ctypes.data_as(C.POINTER(C.c_double))
    o = pkg.mg_options()
    o.smoother = pkg.SMOOTHER[smoother]
    o.nu1 = o.nu2 = 2
    o.gamma = 1
    o.max_cycles = 10
    h = C.c_void_p()
    rc = lib.mg_debug_setup_host(C.byref(g), C.byref(st), C.byref(o), C.byref(h))
    return rc, h


def test_setup_rejects_bad_input():
    assert host_handle([63, 64], "uniform", 0, "tweed")[0] == pkg.MG_EINVAL
    assert host_handle([64, 64], "tanh_wall", -2.0, "tweed")[0] == pkg.MG_EINVAL
    assert host_handle([64, 64, 64], "tanh_wall", 2.0, "wireframe")[0] == pkg.MG_EUNSUPPORTED


def test_setup_rejects_arrays_beyond_32bit_offsets():
    """The kernels address one problem's array with 32-bit offsets: a 1300^3
    grid (1301^3 = 2.2e9 nodes per array, 17.6 GB in FP64, which would fit in
    HBM) is refused at set-up, before any table is built, and so is 1290^3
    (1291^3 = 2.15e9 nodes, just above 2^31 - 1)."""
    assert host_handle([1300, 1300, 1300], "uniform", 0, "checkerboard")[0] == pkg.MG_EUNSUPPORTED
    assert host_handle([1290, 1290, 1290], "uniform", 0, "checkerboard")[0] == pkg.MG_EUNSUPPORTED


@pytest.mark.parametrize("n,kind,c", [([64, 64], "tanh_wall", 3.0), ([96, 48], "sinh_centre", 4.0),
                                      ([32, 16, 24], "tanh_centre", 1.5)])
def test_setup_geometry_matches_oracle(n, kind, c):
    rc, h = host_handle(n, kind, c, "tweed")
    assert rc == 0
    H = O.Hierarchy([O.coords(kind, c, k) for k in n], "tweed")
    nl = C.c_int()
    pkg.capi().mg_levels(h, C.byref(nl))
    assert nl.value == H.nlev
    for lv in range(H.nlev):
        for a in range(len(n)):
            m = H.level_n(lv)[a] + 1
            x, lo, hi = np.zeros(m), np.zeros(m), np.zeros(m)
            pkg.capi().mg_level_coefs(h, lv, a, x.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                                      hi.ctypes.data_as(C.c_void_p))
            xo, loo, hio = H.level_coefs(lv, a)
            assert rel_inf(x, xo) < 1e-15 and rel_inf(lo, loo) < 1e-14 and rel_inf(hi, hio) < 1e-14
    pkg.capi().mg_destroy(h)


EMU_CASES = [([16, 16], "tanh_wall", 2.0, "tweed"), ([64, 64], "tanh_wall", 3.0, "tweed"),
             ([24, 12], "tanh_wall", 2.0, "tweed"), ([12, 40], "tanh_wall", 2.0, "tweed"),
             ([4, 6], "uniform", 0.0, "tweed"),
             ([16, 16], "tanh_centre", 1.5, "wireframe"), ([64, 64], "sinh_centre", 3.0, "wireframe"),
             ([24, 12], "tanh_wall", 2.0, "wireframe"), ([12, 24], "tanh_wall", 2.0, "wireframe"),
             ([6, 4], "uniform", 0.0, "wireframe"),
             ([16, 16], "tanh_wall", 2.0, "zebra_x"), ([16, 20], "tanh_wall", 2.0, "zebra_y"),
             ([16, 16], "tanh_wall", 2.0, "adz"), ([16, 16], "tanh_wall", 2.0, "alt_tw"),
             ([8, 8, 8], "tanh_wall", 2.0, "tweed"), ([16, 16, 16], "tanh_wall", 2.5, "tweed"),
             ([12, 8, 10], "tanh_wall", 2.5, "tweed"), ([4, 4, 4], "uniform", 0.0, "tweed"),
             ([8, 8, 8], "tanh_wall", 2.0, "zebra_z"), ([8, 8, 8], "tanh_wall", 2.5, "adz"),
             ([12, 8, 10], "sinh_centre", 3.0, "adz"), ([512, 512], "tanh_wall", 3.0, "tweed"),
             ([256, 256], "sinh_centre", 4.0, "wireframe")]


@pytest.mark.parametrize("n,kind,c,sm", EMU_CASES)
def test_kernel_steps_on_host_match_oracle(n, kind, c, sm):
    """The device kernel's per-lane steps (chunk elimination, reduced chain /
    spider / ring solve, back substitution), executed on the host over the
    library's own block tables, equal the oracle's sweep (forward and adjoint)."""
    rc, h = host_handle(n, kind, c, sm)
    assert rc == 0
    xs = [O.coords(kind, c, k) for k in n]
    shape = O.Hierarchy(xs, sm, maxlev=1).shape(0)
    u = inputs.normal(shape, 1)
    f = inputs.normal(shape, 2)
    for adj in (0, 1):
        Ho = O.Hierarchy(xs, sm, transpose=bool(adj), maxlev=1)
        ue = u.copy()
        assert pkg.capi().mg_debug_host_smooth(h, 0, ue.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                                               2, adj) == 0
        assert rel_inf(ue, Ho.smooth(u, f, 2)) < 1e-12
    pkg.capi().mg_destroy(h)


@pytest.mark.parametrize("n,kind,c,sm", [([256, 256], "tanh_wall", 3.0, "tweed"), ([256, 128], "tanh_wall", 2.5, "tweed"),
                                        ([256, 256], "sinh_centre", 4.0, "wireframe"),
                                        ([128, 256], "sinh_centre", 3.0, "wireframe"),
                                        ([256, 192], "tanh_wall", 2.0, "zebra_y"), ([256, 256], "tanh_wall", 2.0, "adz"),
                                        ([64, 64, 64], "tanh_wall", 2.5, "tweed"),
                                        ([80, 64, 72], "sinh_centre", 2.0, "tweed")])
def test_kernel_steps_in_device_layout_match_oracle(n, kind, c, sm):
    """The same per-lane steps addressing the level's device layout (lines
    along y stored column-major on the large 2D levels; in 3D from 65^3 nodes
    on, three planes with each line axis fastest) equal the oracle's sweep."""
    rc, h = host_handle(n, kind, c, sm)
    assert rc == 0
    xs = [O.coords(kind, c, k) for k in n]
    shape = O.Hierarchy(xs, sm, maxlev=1).shape(0)
    u = inputs.normal(shape, 3)
    f = inputs.normal(shape, 4)
    for adj in (0, 1):
        Ho = O.Hierarchy(xs, sm, transpose=bool(adj), maxlev=1)
        ue = u.copy()
        assert pkg.capi().mg_debug_host_smooth_layout(h, 0, ue.ctypes.data_as(C.c_void_p),
                                                      f.ctypes.data_as(C.c_void_p), 1, adj) == 0
        assert rel_inf(ue, Ho.smooth(u, f, 1)) < 1e-12
    pkg.capi().mg_destroy(h)


def test_kernel_steps_full_size_wireframe_rings_match_oracle():
    """The 2049^2 centre-clustered grid (sinh, b = 4) of the wireframe
    workload: its outer rings exceed NT/2 chunks, are built without the
    plane cuts and run in NT-lane workgroups that address their points in
    general form -- a path no smaller grid reaches.  The kernel's per-lane
    steps over the level's own tables and device layout equal the oracle's
    relaxation, forward and adjoint."""
    n, kind, c, sm = [2048, 2048], "sinh_centre", 4.0, "wireframe"
    rc, h = host_handle(n, kind, c, sm)
    assert rc == 0
    info = (C.c_int * 6)()
    assert pkg.capi().mg_debug_table_info(h, 0, 0, 0, info) == 0
    assert info[3] > 256  # a workgroup holds a block of more than NT/2 chunks
    xs = [O.coords(kind, c, k) for k in n]
    shape = (n[1] + 1, n[0] + 1)
    u = inputs.normal(shape, 5)
    f = inputs.normal(shape, 6)
    for adj in (0, 1):
        Ho = O.Hierarchy(xs, sm, transpose=bool(adj), maxlev=1)
        ue = u.copy()
        assert pkg.capi().mg_debug_host_smooth_layout(h, 0, ue.ctypes.data_as(C.c_void_p),
                                                      f.ctypes.data_as(C.c_void_p), 1, adj) == 0
        assert rel_inf(ue, Ho.smooth(u, f, 1)) < 1e-12
    pkg.capi().mg_destroy(h)


@pytest.mark.parametrize("n,kind,c,sm,maxchunks", [([4096, 4096], "tanh_wall", 3.0, "tweed", 512),
                                                    ([2048, 2048], "sinh_centre", 4.0, "wireframe", 512),
                                                    ([256, 256, 256], "tanh_wall", 2.5, "tweed", 512),
                                                    ([1024, 1024], "tanh_wall", 2.5, "tweed", 512)])
def test_full_size_tables(n, kind, c, sm, maxchunks):
    """The benchmark grids' block tables fit the kernel (every block in one
    workgroup) and cover every interior point exactly once per sweep."""
    rc, h = host_handle(n, kind, c, sm)
    assert rc == 0
    pts = 0
    for colour in (0, 1):
        info = (C.c_int * 6)()
        assert pkg.capi().mg_debug_table_info(h, 0, 0, colour, info) == 0
        assert info[3] <= maxchunks and info[4] <= 512
        pts += info[5]
    assert pts == int(np.prod([k - 1 for k in n]))
    pkg.capi().mg_destroy(h)



def _sigma(n, seed):
    return np.exp(np.random.default_rng(seed).uniform(-3.0, 3.0, n))


@pytest.mark.parametrize("n,kind,c,sm", [([64, 32], "tanh_wall", 2.5, "tweed"), ([32, 32], "sinh_centre", 3.0, "wireframe"),
                                        ([16, 8, 12], "tanh_wall", 2.0, "adz"), ([256, 256], "tanh_wall", 3.0, "tweed")])
def test_sigma_coefficients_and_sweep_match_oracle(n, kind, c, sm):
    """Axis-wise conductivity (problem (CP) with sigma_aa = s_a(x_a)): the
    library's coefficients on every level (flux form, series-averaged coarse
    cells) and the kernel's per-lane sweep over its tables equal the oracle's."""
    sig = [_sigma(k, 60 + a) for a, k in enumerate(n)]
    rc, h = host_handle(n, kind, c, sm, sigma=sig)
    assert rc == 0
    xs = [O.coords(kind, c, k) for k in n]
    H = O.Hierarchy(xs, sm, sigma=sig)
    nl = C.c_int()
    pkg.capi().mg_levels(h, C.byref(nl))
    assert nl.value == H.nlev
    for lv in range(H.nlev):
        for a in range(len(n)):
            m = H.level_n(lv)[a] + 1
            x, lo, hi = np.zeros(m), np.zeros(m), np.zeros(m)
            pkg.capi().mg_level_coefs(h, lv, a, x.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                                      hi.ctypes.data_as(C.c_void_p))
            xo, loo, hio = H.level_coefs(lv, a)
            assert rel_inf(lo, loo) < 1e-14 and rel_inf(hi, hio) < 1e-14, (lv, a)
    shape = H.shape(0)
    u = inputs.normal(shape, 7)
    f = inputs.normal(shape, 8)
    for adj in (0, 1):
        Ho = O.Hierarchy(xs, sm, transpose=bool(adj), maxlev=1, sigma=sig)
        ue = u.copy()
        assert pkg.capi().mg_debug_host_smooth_layout(h, 0, ue.ctypes.data_as(C.c_void_p),
                                                      f.ctypes.data_as(C.c_void_p), 1, adj) == 0
        assert rel_inf(ue, Ho.smooth(u, f, 1)) < 1e-12
    pkg.capi().mg_destroy(h)


def test_sigma_rejects_nonpositive_values():
    sig = [np.ones(16), np.ones(16)]
    sig[1][3] = 0.0
    assert host_handle([16, 16], "uniform", 0, "tweed", sigma=sig)[0] == pkg.MG_EINVAL
    sig[1][3] = -1.0
    assert host_handle([16, 16], "uniform", 0, "tweed", sigma=sig)[0] == pkg.MG_EINVAL
    sig[1][3] = np.inf
    assert host_handle([16, 16], "uniform", 0, "tweed", sigma=sig)[0] == pkg.MG_EINVAL
