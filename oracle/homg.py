"""FP64 CPU oracle of the high occupancy multigrid (HOMG), arXiv:1108.2045.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product library.  The
per-node arithmetic lives in ``homg_oracle.c`` (plain loops, IEEE double);
this module strings those steps together in the order of Sec. 2 of the paper:

  * the level schedule of the modified full multigrid cycle (MFMG, Sec. 2
    and Fig. 1): two iterations on the coarsest level, doubling on every finer
    level, capped at MaxI;
  * one MFMG cycle on the residual equation A e = r, starting from e = 0,
    with the restricted right-hand sides P_m r computed first (Sec. 2, the
    restrictions as nested partial reductions);
  * the outer restart on the residual equation until the target accuracy
    (Sec. 2, last paragraph; Sec. 4).

Readings taken where the paper is silent or garbled are listed in the
project's design notes; the ones that shape this file are: the schedule is
monotone from the coarsest level to level 0; the Jacobi weight defaults to
4/5 in 2D and 6/7 in 3D; the coarsest level is the 3^d lattice with one
interior unknown; every cycle solves A e = r from e = 0; the relative
residual is ||f - A u||_2 / ||f||_2 over interior nodes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def load_library(path):
    """ctypes handle on an oracle library with its argument types set."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_residual.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    L.oracle_residual.restype = ctypes.c_double
    L.oracle_norm2_interior.argtypes = [ctypes.c_int, ctypes.c_int, dp]
    L.oracle_norm2_interior.restype = ctypes.c_double
    L.oracle_restrict.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    L.oracle_restrict.restype = None
    L.oracle_interpolate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.oracle_interpolate.restype = ctypes.c_double
    L.oracle_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               dp, dp, dp, dp]
    L.oracle_sweep.restype = None
    L.oracle_add.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    L.oracle_add.restype = None
    L.oracle_prolong.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    L.oracle_prolong.restype = None
    return L


def lib():
    """Load (building first if needed) the oracle's shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = load_library(_LIB_PATH)
    return _lib


def _p(x):
    if x is None:
        return None
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid(d, n):
    return (n,) * d


def check_side(n):
    """n must be 2^k + 1 with k >= 1; returns k."""
    k = (n - 1).bit_length() - 1
    if n < 3 or (1 << k) + 1 != n:
        raise ValueError("side must be 2^k + 1, got %d" % n)
    return k


def default_omega(d):
    """Damped-Jacobi weight: 4/5 in 2D, 6/7 in 3D (the paper states none)."""
    return 4.0 / 5.0 if d == 2 else 6.0 / 7.0


def default_schedule(levels, max_i):
    """MFMG schedule (Sec. 2, Fig. 1): levels M = levels-1 down to 0; two
    iterations on the coarsest, doubling per finer level, capped at MaxI."""
    M = levels - 1
    return [(m, min(2 ** (M - m + 1), max_i)) for m in range(M, -1, -1)]


# ---------------------------------------------------------------- steps --

def residual(d, n, f, u, a=None):
    """r = f - A u on interior nodes, 0 on the boundary; returns (r, sum r^2)."""
    r = np.empty(_grid(d, n))
    s = lib().oracle_residual(d, n, _p(a), _p(f), _p(u), _p(r))
    return r, s


def norm2_interior(d, n, f):
    return lib().oracle_norm2_interior(d, n, _p(f))


def restrict(d, rf):
    """One full-weighting step: side nf -> (nf-1)/2 + 1."""
    nf = rf.shape[0]
    nc = (nf - 1) // 2 + 1
    rc = np.empty(_grid(d, nc))
    lib().oracle_restrict(d, nf, _p(np.ascontiguousarray(rf)), _p(rc))
    return rc


def pyramid(d, r0, levels):
    """[r_0, r_1 = P r_0, ..., r_M]: the restricted right-hand sides of all
    levels (Sec. 2, nested partial reductions)."""
    out = [np.ascontiguousarray(r0)]
    for _ in range(1, levels):
        out.append(restrict(d, out[-1]))
    return out


def interpolate(d, n, m, e, idx):
    """S_m(e) at one node idx = (j, i) or (k, j, i)."""
    if d == 2:
        k, j, i = 0, idx[0], idx[1]
    else:
        k, j, i = idx
    return lib().oracle_interpolate(d, n, m, _p(e), k, j, i)


def prolong(d, n, m, e):
    """S_m(e) at every node of the grid."""
    out = np.empty(_grid(d, n))
    lib().oracle_prolong(d, n, m, _p(np.ascontiguousarray(e)), _p(out))
    return out


def sweep(d, n, m, omega, rm, e_old, a=None):
    """One whole-grid relax+interpolate iteration at level m; returns e_new."""
    e_new = np.empty(_grid(d, n))
    lib().oracle_sweep(d, n, m, omega, _p(a), _p(np.ascontiguousarray(rm)),
                       _p(np.ascontiguousarray(e_old)), _p(e_new))
    return e_new


# ---------------------------------------------------------------- cycle --

def mfmg_cycle(d, n, r0, schedule, omega, a=None, levels=None, keep_states=False):
    """One MFMG cycle on A e = r0 from e = 0 (Sec. 2, HOMG steps (a)-(c)).

    Returns e after the last iteration; with keep_states also the list of
    every whole-grid iterate (e after iteration 1, 2, ...)."""
    if levels is None:
        levels = 1 + max(m for m, _ in schedule)
    rs = pyramid(d, r0, levels)
    e = np.zeros(_grid(d, n))
    states = []
    for m, iters in schedule:
        for _ in range(iters):
            e = sweep(d, n, m, omega, rs[m], e, a)
            if keep_states:
                states.append(e.copy())
    return (e, states) if keep_states else e


def solve(d, n, f, u0=None, *, tol=1e-10, max_cycles=100, omega=None, max_i=4,
          levels=None, schedule=None, a=None, fixed_cycles=None):
    """HOMG with the residual-equation restart (Sec. 2 last paragraph).

    Returns (u, history) where history[c] is the relative residual after
    cycle c (history[0] is that of u0).  Stops at the first cycle with
    relres <= tol, or after exactly ``fixed_cycles`` cycles if given."""
    k = check_side(n)
    if levels is None:
        levels = k
    if omega is None:
        omega = default_omega(d)
    if schedule is None:
        schedule = default_schedule(levels, max_i)
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.zeros(_grid(d, n)) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    fn = np.sqrt(norm2_interior(d, n, f))
    denom = fn if fn > 0 else 1.0
    r, s = residual(d, n, f, u, a)
    hist = [np.sqrt(s) / denom]
    ncyc = fixed_cycles if fixed_cycles is not None else max_cycles
    for _ in range(ncyc):
        if fixed_cycles is None and hist[-1] <= tol:
            break
        e = mfmg_cycle(d, n, r, schedule, omega, a, levels)
        lib().oracle_add(d, n, _p(u), _p(e))
        r, s = residual(d, n, f, u, a)
        hist.append(np.sqrt(s) / denom)
    return u, hist
