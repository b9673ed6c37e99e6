"""GPU parity at the full size of the timed workload: the 2D Poisson problem on
4097^2 nodes, tanh wall clustering with g = 3 on both axes (Section 5.1),
tweed V(2,2) cycles in FP64, with the solver set up exactly as the benchmark
sets it up.  The oracle finishes one relaxation of this grid in about 2 s and
one V-cycle in about 10 s, so the comparison is element by element over the
whole array, at the tolerances of the smaller parity cases (1e-12 relative in
the max-norm).  At this size the finest level's black colour holds a block of
512 chunks (the centre cross), which runs as a 512-lane workgroup in a launch
of its own beside the other black workgroups.
"""
import numpy as np
import pytest

import oracle as O
from paper_2110_08389_amd import inputs
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_CELLS = 4096
STRETCH = ("tanh_wall", 3.0)


def dev():
    return torch.device("cuda", 0)


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def N(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solver():
    import paper_2110_08389_amd as pkg

    return pkg.Solver([N_CELLS, N_CELLS], stretch=STRETCH, smoother="tweed", nu1=2, nu2=2, gamma=1,
                      precision="fp64", max_cycles=100, device=dev())


@pytest.fixture(scope="module")
def problem():
    x = O.coords(STRETCH[0], STRETCH[1], N_CELLS)
    H = O.Hierarchy([x, x], "tweed")
    shape = H.shape(0)
    u0 = inputs.normal(shape, 31)
    u0[~H.interior_mask()] = 0.0
    f = inputs.uniform(shape, 32)
    return H, u0, f


def test_fullsize_relaxation(problem):
    H, u0, f = problem
    s = solver()
    ug = N(s.smooth(T(u0), T(f), nu=1))
    uo = H.smooth(u0, f, 1)
    assert rel_inf(ug, uo) < 1e-12, rel_inf(ug, uo)
    del s


def test_fullsize_adjoint_relaxation(problem):
    H, u0, f = problem
    x = O.coords(STRETCH[0], STRETCH[1], N_CELLS)
    Ht = O.Hierarchy([x, x], "tweed", transpose=True, maxlev=1)
    s = solver()
    ug = N(s.smooth(T(u0), T(f), nu=1, adjoint=True))
    uo = Ht.smooth(u0, f, 1)
    assert rel_inf(ug, uo) < 1e-12, rel_inf(ug, uo)
    del s


def test_fullsize_vcycle(problem):
    H, u0, f = problem
    s = solver()
    ug = T(u0)
    s.vcycle(ug, T(f))
    uo = H.cycle(u0, f)
    assert rel_inf(N(ug), uo) < 1e-12, rel_inf(N(ug), uo)
    del s
