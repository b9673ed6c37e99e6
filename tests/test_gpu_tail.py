"""The coarse-level kernel (the coarsest levels run in LDS by one workgroup per
problem) against the per-level kernels of the same library: with
TWMG_NO_TAIL=1 every level uses the per-level launches.  Both paths evaluate
the same per-point formulas, so cycles agree to rounding (1e-13 relative);
the oracle parity of both paths is covered by test_gpu_parity.  Inside the
coarse-level kernel the sub-cycle of the largest level with at most 256
unknowns runs as its precomputed affine map (TWMG_NO_TAIL_MAP=1 runs its
operations instead); the map is exact up to rounding, so the same bound
holds in FP64.  In FP32 cycles the map's sums (up to 450 terms) round
differently from the operations they replace, by FP32 amounts: a refined
solve takes the same cycles to the same solution, and its FP64 residual
history agrees to 1e-3 relative."""
import os

import numpy as np
import pytest

from paper_2110_08389_amd import inputs
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(n, kind, c, sm, notail, nomap=False, **kw):
    import paper_2110_08389_amd as pkg

    saved = {k: os.environ.get(k) for k in ("TWMG_NO_TAIL", "TWMG_NO_TAIL_MAP")}
    os.environ["TWMG_NO_TAIL"] = "1" if notail else "0"
    os.environ["TWMG_NO_TAIL_MAP"] = "1" if nomap else "0"
    try:
        return pkg.Solver(n, stretch=(kind, c), smoother=sm, device=torch.device("cuda", 0), **kw)
    finally:
        for k, v in saved.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


CASES = [([64, 64], "tanh_wall", 3.0, "tweed", {}),
         ([512, 512], "tanh_wall", 3.0, "tweed", {}),
         ([256, 128], "tanh_wall", 2.5, "tweed", {"gamma": 2}),
         ([256, 256], "sinh_centre", 4.0, "wireframe", {"gamma": 2}),
         ([128, 128], "tanh_wall", 2.0, "checkerboard", {}),
         ([128, 128], "tanh_wall", 2.0, "adz", {}),
         ([128, 128], "tanh_wall", 2.0, "alt_tw", {}),
         ([96, 96], "tanh_wall", 2.0, "tweed", {"nu1": 1, "nu2": 3}),
         ([64, 64, 64], "tanh_wall", 2.5, "tweed", {}),
         ([32, 48, 32], "tanh_wall", 2.0, "zebra_z", {}),
         ([64, 64, 64], "tanh_wall", 2.5, "adz", {}),
         ([256, 256], "tanh_wall", 3.0, "tweed", {"batch": 3})]


@pytest.mark.parametrize("n,kind,c,sm,kw", CASES)
def test_tail_matches_per_level_kernels(n, kind, c, sm, kw):
    a = make(n, kind, c, sm, False, **kw)
    b = make(n, kind, c, sm, True, **kw)
    shape = tuple(a.shape())
    f = torch.tensor(inputs.uniform(shape, 11), device=a.device)
    g = torch.tensor(inputs.uniform(shape, 12), device=a.device)
    ua, ub = g.clone(), g.clone()
    for _ in range(3):
        a.vcycle(ua, f)
        b.vcycle(ub, f)
    torch.cuda.synchronize()
    assert rel_inf(ua.cpu().numpy(), ub.cpu().numpy()) < 1e-13
    # adjoint cycles (colour order reversed, transposed operator): a loose
    # tolerance stops the solve after a few cycles
    la, sa = a.solve_adjoint(f, tol=1e-3)
    lb, sb = b.solve_adjoint(f, tol=1e-3)
    assert sa["cycles"] == sb["cycles"]
    torch.cuda.synchronize()
    assert rel_inf(la.cpu().numpy(), lb.cpu().numpy()) < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_tail_full_solve(prec):
    n = [256, 256]
    a = make(n, "tanh_wall", 3.0, "tweed", False, precision=prec)
    b = make(n, "tanh_wall", 3.0, "tweed", True, precision=prec)
    f = torch.tensor(inputs.uniform(tuple(a.shape()), 1001), device=a.device)
    ua, sa = a.solve(f, tol=1e-10)
    ub, sb = b.solve(f, tol=1e-10)
    assert sa["status"] == 0 and sb["status"] == 0 and sa["cycles"] == sb["cycles"]
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_inf(ua.cpu().numpy(), ub.cpu().numpy()) < tol
    np.testing.assert_allclose(sa["history"], sb["history"], rtol=1e-6 if prec == "fp64" else 1e-3, atol=1e-12)


def test_tail_follows_option_changes():
    """The operation lists are rebuilt when the cycle options change."""
    n = [128, 128]
    a = make(n, "tanh_wall", 2.0, "tweed", False)
    b = make(n, "tanh_wall", 2.0, "tweed", True)
    f = torch.tensor(inputs.uniform(tuple(a.shape()), 13), device=a.device)
    for opts in ({"gamma": 2}, {"nu1": 3, "nu2": 0}, {"smoother": "checkerboard"}, {"gamma": 1, "nu1": 2, "nu2": 2}):
        a.set_options(**opts)
        b.set_options(**opts)
        ua, ub = torch.zeros_like(f), torch.zeros_like(f)
        a.vcycle(ua, f)
        b.vcycle(ub, f)
        torch.cuda.synchronize()
        assert rel_inf(ua.cpu().numpy(), ub.cpu().numpy()) < 1e-13, opts


@pytest.mark.parametrize("n,kind,c,sm,kw", [([256, 256], "sinh_centre", 4.0, "wireframe", {"gamma": 2}),
                                            ([64, 64], "tanh_wall", 3.0, "tweed", {}),
                                            ([32, 32, 32], "tanh_wall", 2.5, "tweed", {"gamma": 2})])
def test_tail_map_matches_its_operations(n, kind, c, sm, kw):
    """The sub-cycle map against the operations it replaces; with gamma = 2
    the mapped level is also entered with a nonzero u (second visit)."""
    a = make(n, kind, c, sm, False, **kw)
    b = make(n, kind, c, sm, False, nomap=True, **kw)
    shape = tuple(a.shape())
    f = torch.tensor(inputs.uniform(shape, 14), device=a.device)
    ua, ub = torch.zeros_like(f), torch.zeros_like(f)
    for _ in range(3):
        a.vcycle(ua, f)
        b.vcycle(ub, f)
    torch.cuda.synchronize()
    assert rel_inf(ua.cpu().numpy(), ub.cpu().numpy()) < 1e-13
