"""Seeded synthetic inputs for the HOMG workloads (no method arithmetic here).

The one module that both the oracle-side tests and the GPU-side tests and
benchmark use: it only draws and shapes inputs.  Every array is FP64,
C-ordered with x fastest, generated on the host with numpy's PCG64
(``numpy.random.default_rng(seed)``); boundary entries of f are set to 0
(the solver ignores them).

Workloads (sizes and distributions of the problems the method is run on):
  sine2d     2D, side 129, f = 2 pi^2 sin(pi x) sin(pi y)      (u = sin sin)
  uniform    any d, side n, f ~ U[-1, 1]
  normal     any d, side n, f ~ N(0, 1)
  batch2d    count problems, sides drawn from {65,129,257,513,1025}, each f ~ U[-1,1]
  grf2d      2D, side n, a = exp(g), g a Gaussian random field (sigma 1,
             squared-exponential covariance, correlation length 0.1),
             f ~ U[-1, 1]
  poly2d     the paper's polynomial test problem (Sec. 4), -Laplacian form
"""
import numpy as np

BATCH_SIDES = (65, 129, 257, 513, 1025)


def _zero_boundary(f):
    d = f.ndim
    for axis in range(d):
        sl = [slice(None)] * d
        sl[axis] = 0
        f[tuple(sl)] = 0.0
        sl[axis] = -1
        f[tuple(sl)] = 0.0
    return f


def coords(n):
    return np.linspace(0.0, 1.0, n)


def sine2d(n=129):
    x = coords(n)
    f = 2.0 * np.pi ** 2 * np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    return _zero_boundary(np.ascontiguousarray(f))


def sine2d_exact(n=129):
    x = coords(n)
    return np.outer(np.sin(np.pi * x), np.sin(np.pi * x))


def poly2d(n):
    """Sec. 4 test problem, negated for -Laplace u = f: returns (f, u)."""
    x = coords(n)
    X2, X1 = np.meshgrid(x, x, indexing="ij")  # X2 varies along rows (y), X1 along x
    u = -(X1 ** 2) * X2 ** 2 * (1 - X1 ** 2) * (1 - X2 ** 2)
    lap = -2.0 * (X2 ** 2 * (1 - 6 * X1 ** 2) * (1 - X2 ** 2) + X1 ** 2 * (1 - 6 * X2 ** 2) * (1 - X1 ** 2))
    return _zero_boundary(np.ascontiguousarray(-lap)), np.ascontiguousarray(u)


def uniform(d, n, seed=0):
    rng = np.random.default_rng(seed)
    return _zero_boundary(rng.uniform(-1.0, 1.0, (n,) * d))


def normal(d, n, seed=0):
    rng = np.random.default_rng(seed)
    return _zero_boundary(rng.standard_normal((n,) * d))


def batch2d(count=512, seed=0, sides=BATCH_SIDES):
    rng = np.random.default_rng(seed)
    ss = rng.choice(np.array(sides), count)
    fs = [_zero_boundary(rng.uniform(-1.0, 1.0, (int(s), int(s)))) for s in ss]
    return [int(s) for s in ss], fs


def grf2d(n, seed=0, sigma=1.0, corr=0.1):
    """Stationary Gaussian field on the n x n nodes of the unit square:
    seeded white noise on a periodic 2(n-1) grid convolved (by FFT) with a
    Gaussian kernel whose self-convolution is the squared-exponential
    covariance exp(-r^2 / (2 corr^2)), cropped to n x n and standardised."""
    rng = np.random.default_rng(seed)
    P = 2 * (n - 1)
    h = 1.0 / (n - 1)
    w = rng.standard_normal((P, P))
    x = np.fft.fftfreq(P, d=1.0 / P) * h  # signed periodic distance
    X, Y = np.meshgrid(x, x, indexing="ij")
    ker = np.exp(-(X ** 2 + Y ** 2) / (corr ** 2))  # width corr/sqrt(2)
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * np.fft.fft2(ker)))[:n, :n]
    g = (g - g.mean()) / g.std() * sigma
    return np.ascontiguousarray(g)


def grf_problem(n=1025, seed=0):
    """(a, f) for the variable-coefficient diffusion problem."""
    g = grf2d(n, seed)
    a = np.exp(g)
    rng = np.random.default_rng(seed + 1_000_003)
    f = _zero_boundary(rng.uniform(-1.0, 1.0, (n, n)))
    return np.ascontiguousarray(a), f
