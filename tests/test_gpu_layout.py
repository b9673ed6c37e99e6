"""The split device layout (lines along y stored column-major on the large
levels of the tweed, wireframe and y-zebra smoothers) against the plain
row-major layout of the same library (TWMG_ROW_LAYOUT=1).  The arithmetic is
the same in both; only the addresses differ, so results agree to rounding of
the order of operations (1e-13 relative).  Oracle parity of the split layout
is covered by test_gpu_parity (its grids of 256 cells and up are split)."""
import os

import numpy as np
import pytest

from paper_2110_08389_amd import inputs
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(n, kind, c, sm, row, **kw):
    import paper_2110_08389_amd as pkg

    old = os.environ.get("TWMG_ROW_LAYOUT")
    os.environ["TWMG_ROW_LAYOUT"] = "1" if row else "0"
    try:
        return pkg.Solver(n, stretch=(kind, c), smoother=sm, device=torch.device("cuda", 0), **kw)
    finally:
        if old is None:
            del os.environ["TWMG_ROW_LAYOUT"]
        else:
            os.environ["TWMG_ROW_LAYOUT"] = old


CASES = [([512, 512], "tanh_wall", 3.0, "tweed", {}),
         ([512, 256], "tanh_wall", 2.5, "tweed", {}),
         ([256, 512], "tanh_wall", 2.5, "tweed", {"gamma": 2}),
         ([512, 512], "sinh_centre", 4.0, "wireframe", {"gamma": 2}),
         ([256, 384], "sinh_centre", 3.0, "wireframe", {}),
         ([512, 256], "tanh_wall", 2.0, "zebra_y", {}),
         ([256, 256], "tanh_wall", 3.0, "tweed", {"batch": 3}),
         ([64, 64, 64], "tanh_wall", 2.5, "tweed", {}),
         ([128, 64, 96], "sinh_centre", 2.0, "tweed", {"batch": 2})]


@pytest.mark.parametrize("n,kind,c,sm,kw", CASES)
def test_split_layout_matches_row_layout(n, kind, c, sm, kw):
    a = make(n, kind, c, sm, False, **kw)
    b = make(n, kind, c, sm, True, **kw)
    shape = tuple(a.shape())
    f = torch.tensor(inputs.uniform(shape, 21), device=a.device)
    g = torch.tensor(inputs.uniform(shape, 22), device=a.device)
    # one smoothing pass, one cycle, a full solve and an adjoint solve
    sa, sb = a.smooth(g.clone(), f, nu=2), b.smooth(g.clone(), f, nu=2)
    torch.cuda.synchronize()
    assert rel_inf(sa.cpu().numpy(), sb.cpu().numpy()) < 1e-13
    ua, ub = g.clone(), g.clone()
    a.vcycle(ua, f)
    b.vcycle(ub, f)
    torch.cuda.synchronize()
    assert rel_inf(ua.cpu().numpy(), ub.cpu().numpy()) < 1e-13
    xa, ta = a.solve(f, tol=1e-10)
    xb, tb = b.solve(f, tol=1e-10)
    assert ta["status"] == tb["status"] and ta["cycles"] == tb["cycles"]
    assert rel_inf(xa.cpu().numpy(), xb.cpu().numpy()) < 1e-12
    la, qa = a.solve_adjoint(f, tol=1e-6)
    lb, qb = b.solve_adjoint(f, tol=1e-6)
    assert qa["cycles"] == qb["cycles"]
    assert rel_inf(la.cpu().numpy(), lb.cpu().numpy()) < 1e-12


def test_split_layout_dirichlet_and_refinement():
    n = [512, 512]
    a = make(n, "tanh_wall", 3.0, "tweed", False, precision="fp32_ir")
    b = make(n, "tanh_wall", 3.0, "tweed", True, precision="fp32_ir")
    shape = tuple(a.shape())
    f = torch.tensor(inputs.normal(shape, 23), device=a.device)
    bc = torch.tensor(inputs.normal(shape, 24), device=a.device)
    xa, ta = a.solve(f, bc, tol=1e-10)
    xb, tb = b.solve(f, bc, tol=1e-10)
    assert ta["status"] == 0 and tb["status"] == 0 and ta["cycles"] == tb["cycles"]
    assert rel_inf(xa.cpu().numpy(), xb.cpu().numpy()) < 1e-9
    # the boundary values are the Dirichlet data
    m = np.zeros(shape, bool)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
    assert np.array_equal(xa.cpu().numpy()[m], bc.cpu().numpy()[m])


def test_split_layout_transfer_operators():
    n = [512, 512]
    a = make(n, "tanh_wall", 3.0, "tweed", False)
    b = make(n, "tanh_wall", 3.0, "tweed", True)
    shape = tuple(a.shape())
    u = torch.tensor(inputs.normal(shape, 25), device=a.device)
    f = torch.tensor(inputs.normal(shape, 26), device=a.device)
    for adj in (False, True):
        assert rel_inf(a.residual(u, f, adjoint=adj).cpu().numpy(), b.residual(u, f, adjoint=adj).cpu().numpy()) < 1e-14
        fa, ua = a.residual_restrict(u, f, adjoint=adj)
        fb, ub = b.residual_restrict(u, f, adjoint=adj)
        assert rel_inf(fa.cpu().numpy(), fb.cpu().numpy()) < 1e-14
        assert np.array_equal(ua.cpu().numpy(), ub.cpu().numpy())
    ec = torch.tensor(inputs.normal(tuple(a.shape(1)), 27), device=a.device)
    pa = a.prolong_add(ec, u.clone())
    pb = b.prolong_add(ec, u.clone())
    assert rel_inf(pa.cpu().numpy(), pb.cpu().numpy()) < 1e-15


@pytest.mark.parametrize("n,kind,c,sm,slots", [([512, 512], "tanh_wall", 3.0, "tweed", 1),
                                               ([256, 256], "sinh_centre", 4.0, "wireframe", 1),
                                               ([256, 128], "tanh_wall", 2.0, "zebra_y", 1),
                                               ([128, 128], "tanh_wall", 2.0, "adz", 2),
                                               ([64, 64], "tanh_wall", 2.0, "alt_tw", 2),
                                               ([64, 64, 64], "tanh_wall", 2.5, "tweed", 1)])
def test_half_sweeps_in_device_layout(n, kind, c, sm, slots):
    """Half-sweeps on device-layout arrays, in the smoother's order, give what
    mg_smooth gives; the layout conversions are exact inverses."""
    s = make(n, kind, c, sm, False)
    shape = tuple(s.shape())
    u = torch.tensor(inputs.normal(shape, 31), device=s.device)
    f = torch.tensor(inputs.normal(shape, 32), device=s.device)
    assert torch.equal(s.from_layout(s.to_layout(u)), u)
    for adj in (False, True):
        ref = s.smooth(u.clone(), f, nu=1, adjoint=adj)
        ud, fd = s.to_layout(u), s.to_layout(f)
        order = [(sl, c_) for sl in range(slots) for c_ in (0, 1)]
        if adj:
            order = order[::-1]
        for sl, c_ in order:
            s.half_sweep(ud, fd, c_, slot=sl, adjoint=adj)
        assert torch.equal(s.from_layout(ud), ref)
