"""The allocation-free defect norm (mg_residual_norm_noalloc) against
mg_residual_norm, through the C ABI: two calls in a row on the same GPU, the
second on a smaller grid and batch, each equal to the allocating entry
point's value (the maximum is exact whatever the partial split)."""
import ctypes as C

import numpy as np
import pytest

from paper_2110_08389_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_norm_matches_allocating_entry_point():
    import paper_2110_08389_amd as pkg

    dev = torch.device("cuda", 0)
    lib = pkg.capi()
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
    cases = [([1024, 1024], 3, "tanh_wall", 3.0, "tweed"), ([96, 64], 2, "sinh_centre", 2.0, "wireframe"),
             ([32, 32, 16], 1, "tanh_wall", 2.5, "tweed")]
    for k, (n, B, kind, c, sm) in enumerate(cases):
        s = pkg.Solver(n, stretch=(kind, c), smoother=sm, batch=B, device=dev)
        shape = s.shape(0, batched=True)
        u = torch.tensor(inputs.normal(shape, 300 + k), device=dev)
        f = torch.tensor(inputs.normal(shape, 400 + k), device=dev)
        want = C.c_double()
        assert lib.mg_residual_norm(s.h, C.c_void_p(u.data_ptr()), C.c_void_p(f.data_ptr()), C.byref(want)) == 0
        assert lib.mg_residual_norm_noalloc(s.h, C.c_void_p(u.data_ptr()), C.c_void_p(f.data_ptr()),
                                            C.c_void_p(out.data_ptr())) == 0
        torch.cuda.synchronize()
        got = out[0].item()
        assert got == want.value, (n, B, got, want.value)
        assert out[1].item() == -1.0  # nothing past out[0] is written
        # the same call again on the same inputs gives the same bits
        s.residual_norm_noalloc(u, f, out)
        torch.cuda.synchronize()
        assert out[0].item() == want.value
        del s


def test_noalloc_norm_rejects_bad_arguments():
    import paper_2110_08389_amd as pkg

    dev = torch.device("cuda", 0)
    lib = pkg.capi()
    s = pkg.Solver([16, 16], stretch=("uniform", 0.0), smoother="tweed", device=dev)
    u = s.zeros()
    assert lib.mg_residual_norm_noalloc(s.h, C.c_void_p(u.data_ptr()), C.c_void_p(u.data_ptr()),
                                        C.c_void_p(0)) == pkg.MG_EINVAL
    assert lib.mg_residual_norm_noalloc(None, C.c_void_p(u.data_ptr()), C.c_void_p(u.data_ptr()),
                                        C.c_void_p(u.data_ptr())) == pkg.MG_EINVAL
    # a batch beyond the device array's 16384 partial slots is refused
    sb = pkg.Solver([2, 2], stretch=("uniform", 0.0), smoother="tweed", batch=16385, device=dev)
    ub = sb.zeros()
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    assert lib.mg_residual_norm_noalloc(sb.h, C.c_void_p(ub.data_ptr()), C.c_void_p(ub.data_ptr()),
                                        C.c_void_p(out.data_ptr())) == pkg.MG_EINVAL
