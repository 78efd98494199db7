"""FP64 CPU oracle of the power-of-two grid strategy (Sec. 3 of
arXiv:1108.2045) for the 2D Poisson problem.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product.  The
per-node arithmetic is in ``pow2_oracle.c`` (see its header for the reading
of Sec. 3: four quadrants, level marks measured from each quadrant's
external corner up to the points just outside it, relaxation at every mark,
interpolation only from the node's own quadrant, one nested restriction
sequence per quadrant).  This module strings the steps together exactly as
``oracle/homg.py`` does for the nested 2^k + 1 grids: the restrictions of
the residual, the MFMG schedule of whole-grid iterations (Sec. 2, Fig. 1),
the update and the restart on the residual equation.
"""
import ctypes

import numpy as np

from . import homg as _O

_lib = None


def _bind(L):
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_p2_family_base.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    L.oracle_p2_family_base.restype = None
    L.oracle_p2_restrict.argtypes = [ctypes.c_int, dp, dp]
    L.oracle_p2_restrict.restype = None
    L.oracle_p2_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(dp), dp, dp]
    L.oracle_p2_sweep.restype = None
    L.oracle_p2_marks.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.oracle_p2_marks.restype = None
    L.oracle_p2_prolong.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    L.oracle_p2_prolong.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _bind(_O.lib())  # builds liboracle.so if needed; the Sec. 3 functions live in it too
    return _lib


def use_library(path):
    """Point the Sec. 3 functions at another build of them (None: the
    oracle's own library); the planted-mistake tests use this."""
    global _lib
    _lib = _bind(ctypes.CDLL(path)) if path else None


def _p(x):
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def check_side(N):
    """N must be 2^k with k >= 2; returns k (the number of levels)."""
    k = N.bit_length() - 1
    if N < 4 or (1 << k) != N:
        raise ValueError("side must be a power of two >= 4, got %d" % N)
    return k


def default_schedule(levels, max_i):
    return _O.default_schedule(levels, max_i)


def families(r0, levels):
    """fam[m][q]: the level-m restriction of quadrant q = 2 sy + sx (m >= 1);
    fam[0] = [r0]."""
    N = r0.shape[0]
    L = lib()
    out = [[np.ascontiguousarray(r0)]]
    base = []
    for q in range(4):
        F = np.empty((N, N))
        L.oracle_p2_family_base(N, q & 1, q >> 1, _p(np.ascontiguousarray(r0)), _p(F))
        base.append(F)
    cur = base
    for m in range(1, levels):
        nxt = []
        for F in cur:
            s = F.shape[0] // 2
            C = np.empty((s, s))
            L.oracle_p2_restrict(F.shape[0], _p(F), _p(C))
            nxt.append(C)
        out.append(nxt)
        cur = nxt
    return out


def sweep(N, m, omega, fam_m, e_old):
    arr = (ctypes.POINTER(ctypes.c_double) * 4)(*[_p(a) for a in (list(fam_m) + [fam_m[0]] * 4)[:4]])
    e_new = np.empty((N, N))
    lib().oracle_p2_sweep(N, m, omega, arr, _p(np.ascontiguousarray(e_old)), _p(e_new))
    return e_new


def marks(N, m):
    out = np.empty((N, N), dtype=np.int32)
    lib().oracle_p2_marks(N, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def prolong(N, m, e):
    out = np.empty((N, N))
    lib().oracle_p2_prolong(N, m, _p(np.ascontiguousarray(e)), _p(out))
    return out


def mfmg_cycle(N, r0, schedule, omega, keep_states=False):
    """One MFMG cycle on A e = r0 from e = 0 (Sec. 2 steps, Sec. 3 layout)."""
    levels = 1 + max(m for m, _ in schedule)
    fam = families(r0, levels)
    e = np.zeros((N, N))
    states = []
    for m, iters in schedule:
        for _ in range(iters):
            e = sweep(N, m, omega, fam[m], e)
            if keep_states:
                states.append(e.copy())
    return (e, states) if keep_states else e


def solve(N, f, u0=None, *, tol=1e-10, max_cycles=100, omega=0.8, max_i=4, schedule=None,
          fixed_cycles=None):
    """HOMG on the power-of-two grid with the residual restart; returns
    (u, relres history)."""
    k = check_side(N)
    if schedule is None:
        schedule = default_schedule(k, max_i)
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.zeros((N, N)) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    fn = np.sqrt(_O.norm2_interior(2, N, f))
    denom = fn if fn > 0 else 1.0
    r, s = _O.residual(2, N, f, u)
    hist = [np.sqrt(s) / denom]
    ncyc = fixed_cycles if fixed_cycles is not None else max_cycles
    for _ in range(ncyc):
        if fixed_cycles is None and hist[-1] <= tol:
            break
        e = mfmg_cycle(N, r, schedule, omega)
        u += e
        r, s = _O.residual(2, N, f, u)
        hist.append(np.sqrt(s) / denom)
    return u, hist
