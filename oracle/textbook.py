"""Textbook multigrid and dense assembly of A: the independent half of the oracle.

TEST INFRASTRUCTURE ONLY.  Written separately from ``homg_oracle.c`` (numpy
slicing on per-level compact grids instead of per-node loops on one array)
so that the HOMG oracle can be pinned to the discrete solution u* = A^-1 f
by code that shares nothing with it:

  * ``assemble_dense``: A as an explicit matrix on the interior nodes,
    Kronecker sums of the 1D second difference for the Laplacian, face by
    face for -div(a grad) (Sec. 2, the system A u = f);
  * ``vcycle_solve``: the classic correction-scheme V(nu1, nu2) cycle of
    Sec. 2 (pre-smoothing, restriction of the residual, coarse residual
    equation, interpolation and correction, post-smoothing) with damped
    Jacobi, full weighting, linear interpolation and rediscretised coarse
    operators (the standard choices the paper names).
"""
import numpy as np

# ------------------------------------------------------------ operators --


def _inner(d):
    return (slice(1, -1),) * d


def _shift(d, axis, s, n):
    sl = [slice(1, -1)] * d
    sl[axis] = slice(1 + s, n - 1 + s)
    return tuple(sl)


def face_coef(am, d, axis, s):
    """Harmonic mean of the nodal coefficient across the face in direction
    (axis, s) for every interior node; 1 if am is None."""
    if am is None:
        return 1.0
    n = am.shape[0]
    c = am[_inner(d)]
    q = am[_shift(d, axis, s, n)]
    return 2.0 * c * q / (c + q)


def apply_A(u, hm, am=None):
    """(A u) on interior nodes of a compact grid with spacing hm; 0 on the
    boundary."""
    d = u.ndim
    n = u.shape[0]
    out = np.zeros_like(u)
    inn = _inner(d)
    for axis in range(d):
        for s in (-1, 1):
            out[inn] += face_coef(am, d, axis, s) * (u[inn] - u[_shift(d, axis, s, n)])
    return out / (hm * hm)


def diag_A(shape, hm, am=None):
    d = len(shape)
    dg = np.zeros(tuple(s - 2 for s in shape))
    for axis in range(d):
        for s in (-1, 1):
            dg = dg + face_coef(am, d, axis, s)
    return dg / (hm * hm)


def fw_restrict(rf):
    """Full weighting, tensor product of (1/4)[1 2 1]; boundary 0."""
    d = rf.ndim
    nf = rf.shape[0]
    nc = (nf - 1) // 2 + 1
    rc = np.zeros((nc,) * d)
    w1 = {-1: 0.25, 0: 0.5, 1: 0.25}
    inn = _inner(d)
    for offs in np.ndindex(*(3,) * d):
        o = [x - 1 for x in offs]
        w = np.prod([w1[x] for x in o])
        sl = tuple(slice(2 + x, nf - 2 + x, 2) for x in o)
        rc[inn] += w * rf[sl]
    return rc


def lin_interp(ec):
    """Linear interpolation coarse -> fine, one axis at a time."""
    d = ec.ndim
    out = ec
    for axis in range(d):
        nc = out.shape[axis]
        nf = 2 * nc - 1
        shape = list(out.shape)
        shape[axis] = nf
        f = np.zeros(shape)
        ev = [slice(None)] * d
        ev[axis] = slice(0, nf, 2)
        f[tuple(ev)] = out
        od = [slice(None)] * d
        od[axis] = slice(1, nf, 2)
        lo = [slice(None)] * d
        lo[axis] = slice(0, nc - 1)
        hi = [slice(None)] * d
        hi[axis] = slice(1, nc)
        f[tuple(od)] = 0.5 * (out[tuple(lo)] + out[tuple(hi)])
        out = f
    return out


# ------------------------------------------------------------ assembly --


def _lap1d(nint):
    return 2.0 * np.eye(nint) - np.eye(nint, k=1) - np.eye(nint, k=-1)


def assemble_dense(d, n, a=None):
    """A on the (n-2)^d interior unknowns, C order, x fastest."""
    h = 1.0 / (n - 1)
    nint = n - 2
    if a is None:
        T = _lap1d(nint)
        I = np.eye(nint)
        if d == 2:
            A = np.kron(I, T) + np.kron(T, I)
        else:
            A = np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)
        return A / (h * h)
    # face by face: each interior face (p, q) adds its coefficient to the
    # diagonal of both ends and subtracts it from the coupling; faces to a
    # boundary node only touch the diagonal of the interior end.
    N = nint ** d
    A = np.zeros((N, N))

    def uid(idx):
        if any(x == 0 or x == n - 1 for x in idx):
            return -1
        lin = 0
        for x in idx:
            lin = lin * nint + (x - 1)
        return lin

    for idx in np.ndindex(*(n,) * d):
        for axis in range(d):
            q = list(idx)
            q[axis] += 1
            if q[axis] >= n:
                continue
            q = tuple(q)
            c = 2.0 * a[idx] * a[q] / (a[idx] + a[q])
            ip, iq = uid(idx), uid(q)
            if ip >= 0:
                A[ip, ip] += c
            if iq >= 0:
                A[iq, iq] += c
            if ip >= 0 and iq >= 0:
                A[ip, iq] -= c
                A[iq, ip] -= c
    return A / (h * h)


def dense_solve(d, n, f, a=None, boundary=None):
    """u* = A^-1 f by LU (numpy.linalg.solve) with zero Dirichlet data."""
    A = assemble_dense(d, n, a)
    rhs = np.ascontiguousarray(f[_inner(d)]).reshape(-1)
    u = np.zeros((n,) * d)
    u[_inner(d)] = np.linalg.solve(A, rhs).reshape((n - 2,) * d)
    return u


def laplace_eigenvalue(d, n, ks):
    """Eigenvalue of the discrete -Laplacian for the mode prod sin(k_i pi x_i)."""
    h = 1.0 / (n - 1)
    return (4.0 / (h * h)) * sum(np.sin(k * np.pi * h / 2.0) ** 2 for k in ks)


def sine_mode(d, n, ks):
    x = np.linspace(0.0, 1.0, n)
    out = np.ones((n,) * d)
    for axis, k in enumerate(ks):
        shape = [1] * d
        shape[axis] = n
        out = out * np.sin(k * np.pi * x).reshape(shape)
    return out


# ------------------------------------------------------------ V-cycle --


class VCycle:
    """Classic V(nu1, nu2) correction scheme on compact grids (Sec. 2)."""

    def __init__(self, d, n, a=None, omega=None, nu1=2, nu2=2):
        self.d, self.n = d, n
        self.omega = omega if omega is not None else (0.8 if d == 2 else 6.0 / 7.0)
        self.nu1, self.nu2 = nu1, nu2
        k = (n - 1).bit_length() - 1
        self.L = k  # levels; coarsest side 3
        self.sides = [(n - 1) // (1 << m) + 1 for m in range(self.L)]
        self.h = [(1 << m) / (n - 1) for m in range(self.L)]
        if a is None:
            self.a = [None] * self.L
        else:
            self.a = [np.ascontiguousarray(a[(slice(None, None, 1 << m),) * d]) for m in range(self.L)]
        self.dg = [diag_A((s,) * d, hm, am) for s, hm, am in zip(self.sides, self.h, self.a)]

    def smooth(self, m, u, r, iters):
        inn = _inner(self.d)
        for _ in range(iters):
            res = r - apply_A(u, self.h[m], self.a[m])
            u[inn] += self.omega * res[inn] / self.dg[m]
        return u

    def vcycle(self, m, u, r):
        if m == self.L - 1:
            # exact solve of the coarsest system
            s = self.sides[m]
            if self.a[m] is None:
                A = assemble_dense(self.d, s) * (1.0 / (s - 1)) ** 2 / self.h[m] ** 2
            else:
                A = assemble_dense(self.d, s, self.a[m]) * (1.0 / (s - 1)) ** 2 / self.h[m] ** 2
            u = np.zeros_like(u)
            inn = _inner(self.d)
            u[inn] = np.linalg.solve(A, r[inn].reshape(-1)).reshape(u[inn].shape)
            return u
        u = self.smooth(m, u, r, self.nu1)
        res = r - apply_A(u, self.h[m], self.a[m])
        rc = fw_restrict(res)
        ec = self.vcycle(m + 1, np.zeros_like(rc), rc)
        u = u + lin_interp(ec)
        return self.smooth(m, u, r, self.nu2)

    def solve(self, f, tol=1e-13, max_cycles=200):
        d = self.d
        f = np.array(f, dtype=np.float64)
        bd = np.ones(f.shape, dtype=bool)
        bd[_inner(d)] = False
        f[bd] = 0.0
        u = np.zeros_like(f)
        fn = np.linalg.norm(f[_inner(d)])
        hist = [1.0]
        for _ in range(max_cycles):
            u = self.vcycle(0, u, f)
            rel = np.linalg.norm((f - apply_A(u, self.h[0], self.a[0]))[_inner(d)]) / fn
            hist.append(rel)
            if rel <= tol or (len(hist) > 3 and rel >= 0.9 * hist[-2]):
                break
        return u, hist
