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
