"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/homg.h declares, and
reject bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "homg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(homg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("homg_create", "homg_solve", "homg_residual", "homg_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1108_2045_amd import homg as B
    L = B.load_library()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_version_string():
    from paper_1108_2045_amd import homg as B
    assert "gfx950" in B.load_library().homg_version().decode()


@pytest.mark.parametrize("ndim,n,levels,stencil,status", [
    (4, 9, 0, 0, 1),      # bad ndim
    (2, 10, 0, 0, 1),     # side not 2^k + 1
    (2, 2, 0, 0, 1),      # too small
    (2, 9, 4, 0, 1),      # levels > k
    (2, 9, -1, 0, 1),     # negative levels
    (3, 9, 0, 0, 2),      # 2D stencil on a 3D grid
    (2, 9, 0, 1, 2),      # 3D stencil on a 2D grid
    (2, 9, 0, 7, 1),      # unknown stencil
])
def test_create_rejects_bad_arguments_before_device_work(ndim, n, levels, stencil, status):
    from paper_1108_2045_amd import homg as B
    L = B.load_library()
    opt = B.Options()
    L.homg_options_init(ctypes.byref(opt))
    dims = (ctypes.c_int64 * 4)(n, n, n, n)
    h = ctypes.c_void_p()
    st = L.homg_create(ctypes.byref(h), ndim, dims, levels, stencil, ctypes.byref(opt))
    assert st == status
    assert not h.value
    assert L.homg_last_error(None)


def test_create_rejects_bad_options():
    from paper_1108_2045_amd import homg as B
    L = B.load_library()
    dims = (ctypes.c_int64 * 2)(9, 9)
    h = ctypes.c_void_p()
    for field, value in (("omega", 1.5), ("precision", 9), ("temporal_block", -1), ("struct_size", 3)):
        opt = B.Options()
        L.homg_options_init(ctypes.byref(opt))
        setattr(opt, field, value)
        assert L.homg_create(ctypes.byref(h), 2, dims, 0, 0, ctypes.byref(opt)) == 1, field
    opt = B.Options()
    L.homg_options_init(ctypes.byref(opt))
    bad = (ctypes.c_int * 4)(5, 2, 0, 1)  # level 5 on a 9^2 grid (k = 3)
    opt.schedule = bad
    opt.schedule_len = 2
    assert L.homg_create(ctypes.byref(h), 2, dims, 0, 0, ctypes.byref(opt)) == 1


def test_calls_reject_null_handle():
    from paper_1108_2045_amd import homg as B
    L = B.load_library()
    assert L.homg_destroy(None) == 0
    info = B.Info()
    assert L.homg_solve(None, None, None, 1e-10, None, ctypes.byref(info)) == 1
    assert L.homg_residual(None, None, None, None, None, None) == 1


# ------------------------------------------------- argument shapes (binding)
#
# The C ABI takes raw device pointers and cannot see array sizes, so the
# binding checks every array's shape against the handle before any call.
# These objects are built without a device: the checks must fire first.

def _solver(ndim, n):
    from paper_1108_2045_amd import homg as B
    s = B.Solver.__new__(B.Solver)
    s._h, s.ndim, s.n, s.max_cycles, s.precision = None, ndim, n, 10, "fp64"
    return s


def _t(*shape, dtype=None):
    import torch
    return torch.zeros(shape, dtype=dtype or torch.float64)


@pytest.mark.parametrize("ndim,n", [(2, 33), (3, 17)])
def test_solver_rejects_wrong_shapes(ndim, n):
    s = _solver(ndim, n)
    good, small = _t(*([n] * ndim)), _t(*([n - 1] * ndim))
    flat = _t(n ** ndim)
    with pytest.raises(ValueError, match="shape"):
        s.solve(small, good)
    with pytest.raises(ValueError, match="shape"):
        s.solve(good, small)
    with pytest.raises(ValueError, match="shape"):
        s.solve_cycles(good, flat, 1)
    with pytest.raises(ValueError, match="shape"):
        s.residual(good, good, small)
    with pytest.raises(ValueError, match="shape"):
        s.set_coefficient(small)
    with pytest.raises(ValueError, match="shape"):
        s.step_cycle(good, small)
    nc = (n - 1) // 2 + 1
    with pytest.raises(ValueError, match="shape"):
        s.step_restrict(0, good, good)          # coarse array of the fine side
    with pytest.raises(ValueError, match="shape"):
        s.step_restrict(1, good, _t(*([(nc - 1) // 2 + 1] * ndim)))
    with pytest.raises(ValueError, match="shape"):
        s.step_sweeps(1, 1, good, good, good)   # level-1 residual of the fine side
    with pytest.raises(ValueError, match="level"):
        s.step_sweeps(9, 1, good, good, good)
    with pytest.raises(ValueError, match="shape"):
        s.smoother_gate([good, small], 2)
    # right shapes pass the shape check and stop at the device check
    with pytest.raises(ValueError, match="GPU"):
        s.solve(good, good)
    with pytest.raises(ValueError, match="GPU"):
        s.step_sweeps(1, 1, good, _t(*([nc] * ndim)), good)


def test_batch_and_learned_calls_reject_wrong_shapes():
    import torch
    from paper_1108_2045_amd import homg as B
    b = B.BatchSolver.__new__(B.BatchSolver)
    b._h, b.sides = None, [9, 17]
    fs = [_t(9, 9), _t(17, 17)]
    with pytest.raises(ValueError, match="shape"):
        b.solve(fs, [_t(9, 9), _t(9, 9)])
    with pytest.raises(ValueError, match="shape"):
        b.tune([_t(9, 9), _t(16, 16)], fs)
    with pytest.raises(ValueError, match="one f and one u"):
        b.solve(fs, fs[:1])
    f32 = torch.float32
    x = _t(17, 17, dtype=f32)
    w = _t(B.SMOOTHER_WEIGHTS, dtype=f32)
    with pytest.raises(ValueError, match="shape"):
        B.learn_forward(x, _t(9, 9, dtype=f32), None, w, 0.1, x)
    with pytest.raises(ValueError, match="shape"):
        B.learn_forward(x, x, None, w, 0.1, _t(17, 16, dtype=f32))
    with pytest.raises(ValueError, match="square"):
        B.learn_grad(_t(17, 9, dtype=f32), x, None, x, w, 0.1)
    with pytest.raises(ValueError, match="shape"):
        B.learn_grad(x, x, _t(16, 16, dtype=f32), x, w, 0.1)
    with pytest.raises(ValueError, match="shape"):
        B.learn_adam(w, w, _t(10, dtype=f32), _t(B.SMOOTHER_WEIGHTS), 1, 1e-3, w)
    with pytest.raises(ValueError):
        B.learn_forward(x, x, None, _t(575, dtype=f32), 0.1, x)


@pytest.mark.parametrize("ndim,n,prec,stencil,status", [
    (2, 129, 0, 0, 1),    # not a power of two
    (2, 2, 0, 0, 1),      # too small
    (3, 64, 0, 1, 2),     # 3D
    (2, 64, 1, 0, 2),     # FP32
    (2, 64, 0, 2, 2),     # diffusion stencil
])
def test_pow2_layout_rejects_unsupported(ndim, n, prec, stencil, status):
    from paper_1108_2045_amd import homg as B
    L = B.load_library()
    opt = B.Options()
    L.homg_options_init(ctypes.byref(opt))
    opt.grid_layout = 1
    opt.precision = prec
    dims = (ctypes.c_int64 * 3)(n, n, n)
    h = ctypes.c_void_p()
    assert L.homg_create(ctypes.byref(h), ndim, dims, 0, stencil, ctypes.byref(opt)) == status
    assert not h.value
    opt.grid_layout = 7
    assert L.homg_create(ctypes.byref(h), 2, dims, 0, 0, ctypes.byref(opt)) == 1
