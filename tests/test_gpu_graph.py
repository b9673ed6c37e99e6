"""The solve loop's steps replayed from a captured HIP graph against the same
steps launched one by one (TWMG_NO_GRAPH=1).  A graph runs the same kernels
on the same arrays in the same order, so every solve must agree bit for bit:
the iterates, the cycle count and the residual history.  Each case replays
the graph several times, with other work of the library and of torch, and
host synchronisations, between the replays, and changes what a capture
depends on (the direction, the options) so that it is captured again."""
import os

import numpy as np
import pytest

from paper_2110_08389_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make(n, kind, c, sm, eager, **kw):
    import paper_2110_08389_amd as pkg

    saved = os.environ.get("TWMG_NO_GRAPH")
    os.environ["TWMG_NO_GRAPH"] = "1" if eager else "0"
    try:
        return pkg.Solver(n, stretch=(kind, c), smoother=sm, device=torch.device("cuda", 0), **kw)
    finally:
        if saved is None:
            del os.environ["TWMG_NO_GRAPH"]
        else:
            os.environ["TWMG_NO_GRAPH"] = saved


def same(a, b):
    return np.array_equal(a.cpu().numpy(), b.cpu().numpy())


# every case's finest level uses a split layout, whose solves run on the
# workspace's own arrays and are therefore captured
CASES = [([512, 512], "tanh_wall", 3.0, "tweed", {}, 1e-10),
         ([256, 256], "sinh_centre", 4.0, "wireframe", {"gamma": 2}, 1e-10),
         ([512, 512], "tanh_wall", 3.0, "tweed", {"precision": "fp32_ir"}, 1e-10),
         ([64, 64, 64], "tanh_wall", 2.5, "tweed", {}, 1e-8),
         ([256, 256], "tanh_wall", 3.0, "tweed", {"batch": 3}, 1e-10)]


@pytest.mark.parametrize("n,kind,c,sm,kw,tol", CASES)
def test_graph_replays_match_eager_launches(n, kind, c, sm, kw, tol):
    e = make(n, kind, c, sm, True, **kw)
    g = make(n, kind, c, sm, False, **kw)
    shape = tuple(e.shape())
    for seed in (31, 32, 33):
        f = torch.tensor(inputs.uniform(shape, seed), device=e.device)
        ue, se = e.solve(f, tol=tol)
        ug, sg = g.solve(f, tol=tol)
        torch.cuda.synchronize()
        assert se["status"] == 0 and sg["status"] == 0
        assert se["cycles"] == sg["cycles"] and se["history"] == sg["history"]
        assert same(ue, ug)
        # other work between replays: the library's own kernels, torch's, a
        # host synchronisation
        r = g.residual_norm(ug, f)
        w = (ug * 2.0).sum()
        torch.cuda.synchronize()
        assert np.isfinite(r) and np.isfinite(float(w))
    # the adjoint direction takes its own capture, then the forward one again
    w = torch.tensor(inputs.normal(shape, 34), device=e.device)
    le, qe = e.solve_adjoint(w, tol=1e-8)
    lg, qg = g.solve_adjoint(w, tol=1e-8)
    torch.cuda.synchronize()
    assert qe["cycles"] == qg["cycles"] and same(le, lg)
    ue, se = e.solve(f, tol=tol)
    ug, sg = g.solve(f, tol=tol)
    torch.cuda.synchronize()
    assert se["cycles"] == sg["cycles"] and same(ue, ug)


def test_graph_follows_option_changes():
    n = [512, 512]
    e = make(n, "tanh_wall", 3.0, "tweed", True)
    g = make(n, "tanh_wall", 3.0, "tweed", False)
    shape = tuple(e.shape())
    f = torch.tensor(inputs.uniform(shape, 35), device=e.device)
    for opts in ({}, {"nu1": 1, "nu2": 3}, {"precision": "fp32_ir"}, {"nu1": 2, "nu2": 2, "precision": "fp64"}):
        if opts:
            e.set_options(**opts)
            g.set_options(**opts)
        for _ in range(2):
            ue, se = e.solve(f, tol=1e-10)
            ug, sg = g.solve(f, tol=1e-10)
            torch.cuda.synchronize()
            assert se["cycles"] == sg["cycles"] and se["history"] == sg["history"], opts
            assert same(ue, ug), opts
