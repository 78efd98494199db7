"""The allocation-free residual entry point against homg_residual.

homg_residual_noalloc runs the residual and norm kernels of homg_residual
with their partial sums in the library's static device workspace instead of
a handle's.  Called through the C ABI, it must give the same r and relative
residual bit for bit, on two calls in a row (the second on a smaller grid,
so stale partial sums of the first would show), in 2D and 3D; grids past
the workspace limit are refused before any device work."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def B(torch_cuda):
    import paper_1108_2045_amd as P
    return P


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def noalloc(B, torch, f, u, r):
    L = B.lib()
    rel = ctypes.c_double()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.homg_residual_noalloc(f.dim(), f.shape[0], ctypes.c_void_p(f.data_ptr()),
                                 ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                 ctypes.byref(rel), s)
    assert st == 0, L.homg_last_error(None)
    return rel.value


@pytest.mark.parametrize("d,sizes", [(2, (1025, 257)), (3, (129, 33))])
def test_noalloc_residual_equals_handle_residual(B, torch_cuda, d, sizes):
    torch = torch_cuda
    rng = np.random.default_rng(77 + d)
    for n in sizes:
        say("noalloc residual d=%d n=%d" % (d, n))
        f = dev(torch, W.uniform(d, n, seed=70 + n))
        un = np.zeros((n,) * d)
        un[(slice(1, -1),) * d] = rng.standard_normal((n - 2,) * d)
        u = dev(torch, un)
        # boundary entries of r are left as they are: start both from the
        # same non-zero fill, so a write there would show
        r1 = torch.full((n,) * d, 7.0, dtype=torch.float64, device="cuda")
        r2 = torch.full((n,) * d, 7.0, dtype=torch.float64, device="cuda")
        rel_na = noalloc(B, torch, f, u, r1)
        s = B.Solver(d, n)
        rel_h = s.residual(f, u, r2)
        torch.cuda.synchronize()
        assert torch.equal(r1, r2)
        assert rel_na == rel_h, (rel_na, rel_h)
        # the binding's wrapper takes the same path
        r3 = torch.full_like(r1, 7.0)
        assert B.residual_noalloc(f, u, r3) == rel_h
        assert torch.equal(r3, r2)


def test_noalloc_rejects_bad_sizes(B, torch_cuda):
    torch = torch_cuda
    L = B.lib()
    t = torch.zeros(9, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(t.data_ptr())
    rel = ctypes.c_double()
    assert L.homg_residual_noalloc(2, 10, p, p, p, ctypes.byref(rel), None) == 1   # not 2^k + 1
    assert L.homg_residual_noalloc(4, 9, p, p, p, ctypes.byref(rel), None) == 1    # bad ndim
    assert L.homg_residual_noalloc(2, 65537, p, p, p, ctypes.byref(rel), None) == 2  # too large
    assert L.homg_residual_noalloc(3, 2049, p, p, p, ctypes.byref(rel), None) == 2
    assert L.homg_residual_noalloc(2, 9, p, p, None, ctypes.byref(rel), None) == 1  # r required
