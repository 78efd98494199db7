"""FP64 CPU oracle of the learned smoother that replaces damped Jacobi at the
lattice nodes of the HOMG fused task.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product library, with
which it shares no code.

The paper has no learned component: its lattice nodes relax with damped
Jacobi, the explicit Euler step of the heat equation (Sec. 2).  This module
defines the replacement used for the variable-coefficient diffusion
problem, in plain numpy on the compact level-m lattice (side nm, spacing
h_l = 2^m h; nodes ordered with x fastest, rows = y):

features (per interior lattice node p, zero on the boundary)
    face coefficients a_W, a_E, a_S, a_N: harmonic means of the nodal
    coefficient of p and of its lattice neighbour (1 for the Laplacian);
    rho = (h_l^2 r_m(p) - sum_q a_pq (x_p - x_q)) / sum_q a_pq, the
    Jacobi-scaled local residual (damped Jacobi is x + omega rho);
    X_0 = rho, X_1 = rho (a_E - a_W)/(a_E + a_W), X_2 = rho (a_N - a_S)/(a_N + a_S).
network N (bias-free, so N(c X) = c N(X) for c > 0)
    P_c(p) = sum_ci sum_k W1[c, ci, k] X_ci(p + o_k)     c = 0..15 (interior p)
    H_c = max(P_c, 0) on interior nodes, 0 on the boundary
    y(p) = sum_c sum_k W2[c, k] H_c(p + o_k)             (interior p)
    with the 3x3 offsets o_k = (dy, dx), k = 3 (dy + 1) + (dx + 1), taken
    as a correlation (no kernel flip) and zero outside the lattice.  On the
    whole grid this is a 3x3 convolution dilated by l = 2^m.
update
    x'(p) = x(p) + y(p) at interior lattice nodes.  In the whole-grid task
    every other interior node still interpolates the previous iterate and
    boundary nodes stay 0 (Sec. 2, fused relaxation and interpolation).
loss (training)
    L = E(delta - y) / E(delta), E(v) = v^T A_m v = sum_p v_p (A_m v)_p with
    (A_m v)_p = sum_q a_pq (v_p - v_q), where delta = x* - x is the error
    of the iterate against the exact solution x* of the level system
    A_m x* = h_l^2 r_m.  L is the energy-norm error left by one smoothing
    step, relative to the error before it.

Weights are a flat vector of 576 values: W1[c][ci][k] at 27 c + 9 ci + k,
then W2[c][k] at 432 + 9 c + k.  The GPU stores them in BF16; the oracle
takes whatever values it is given (tests pass the BF16-rounded ones).
"""
import numpy as np

from . import homg as O

C_IN = 3
HID = 16
NW1 = HID * C_IN * 9
NW = NW1 + HID * 9
OFFS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def split(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NW,)
    return w[:NW1].reshape(HID, C_IN, 9), w[NW1:].reshape(HID, 9)


def join(W1, W2):
    return np.concatenate([np.asarray(W1, np.float64).ravel(), np.asarray(W2, np.float64).ravel()])


def shifted(v, dy, dx):
    """v(p + (dy, dx)) for every node p of a 2D array, 0 where that lies outside."""
    n0, n1 = v.shape
    out = np.zeros_like(v)
    ys, yd = (slice(dy, n0), slice(0, n0 - dy)) if dy >= 0 else (slice(0, n0 + dy), slice(-dy, n0))
    xs, xd = (slice(dx, n1), slice(0, n1 - dx)) if dx >= 0 else (slice(0, n1 + dx), slice(-dx, n1))
    out[yd, xd] = v[ys, xs]
    return out


def interior_mask(nm):
    m = np.zeros((nm, nm))
    m[1:-1, 1:-1] = 1.0
    return m


def faces(am, nm):
    """Face coefficients (W, E, S, N) at the interior nodes, shape (nm-2)^2
    each; ones for the constant-coefficient operator."""
    if am is None:
        one = np.ones((nm - 2, nm - 2))
        return one, one, one, one
    c = am[1:-1, 1:-1]

    def hm(q):
        return 2.0 * c * q / (c + q)
    return hm(am[1:-1, :-2]), hm(am[1:-1, 2:]), hm(am[:-2, 1:-1]), hm(am[2:, 1:-1])


def apply_level(v, am):
    """(A_m v)_p = sum_q a_pq (v_p - v_q) at interior nodes (unscaled level
    operator, the neighbours in the order W, E, S, N), 0 on the boundary."""
    nm = v.shape[0]
    aW, aE, aS, aN = faces(am, nm)
    c = v[1:-1, 1:-1]
    out = np.zeros_like(v)
    out[1:-1, 1:-1] = (aW * (c - v[1:-1, :-2]) + aE * (c - v[1:-1, 2:])
                       + aS * (c - v[:-2, 1:-1]) + aN * (c - v[2:, 1:-1]))
    return out


def features(x, rm, am, hl):
    """The three input channels at every lattice node (zero on the boundary)."""
    nm = x.shape[0]
    aW, aE, aS, aN = faces(am, nm)
    sum_a = ((aW + aE) + aS) + aN
    flux = apply_level(x, am)[1:-1, 1:-1]
    rho = (hl * hl * rm[1:-1, 1:-1] - flux) / sum_a
    X = np.zeros((C_IN, nm, nm))
    X[0, 1:-1, 1:-1] = rho
    X[1, 1:-1, 1:-1] = rho * (aE - aW) / (aE + aW)
    X[2, 1:-1, 1:-1] = rho * (aN - aS) / (aN + aS)
    return X


def forward(X, w):
    """(P, H, y): pre-activations, hidden channels, output (all (.., nm, nm))."""
    W1, W2 = split(w)
    nm = X.shape[-1]
    mask = interior_mask(nm)
    P = np.zeros((HID, nm, nm))
    for c in range(HID):
        for ci in range(C_IN):
            for k, (dy, dx) in enumerate(OFFS):
                P[c] += W1[c, ci, k] * shifted(X[ci], dy, dx)
    P *= mask
    H = np.maximum(P, 0.0) * mask
    y = np.zeros((nm, nm))
    for c in range(HID):
        for k, (dy, dx) in enumerate(OFFS):
            y += W2[c, k] * shifted(H[c], dy, dx)
    return P, H, y * mask


def smooth_step(x, rm, am, hl, w):
    """One learned relaxation of every interior node of the compact lattice."""
    _, _, y = forward(features(x, rm, am, hl), w)
    return x + y


def energy(v, am):
    """E(v) = v^T A_m v (v zero on the boundary)."""
    return float(np.sum(v * apply_level(v, am)))


def loss(x, rm, am, hl, delta, w):
    """Energy of the error left by one learned step relative to delta's."""
    _, _, y = forward(features(x, rm, am, hl), w)
    return energy(delta - y, am) / energy(delta, am)


def loss_and_grad(x, rm, am, hl, delta, w):
    """L and dL/dw by the chain rule through the network (features do not
    depend on w):  g = dL/dy = -2 A_m (delta - y) / E(delta) on interior
    nodes; dW2[c,k] = sum_p g(p) H_c(p + o_k); dH_c(q) = sum_k W2[c,k]
    g(q - o_k) on interior q; dP = dH where P > 0; dW1[c,ci,k] = sum_q
    dP_c(q) X_ci(q + o_k)."""
    X = features(x, rm, am, hl)
    P, H, y = forward(X, w)
    W1, W2 = split(w)
    nm = x.shape[0]
    mask = interior_mask(nm)
    E0 = energy(delta, am)
    z = delta - y
    L = energy(z, am) / E0
    g = -2.0 * apply_level(z, am) / E0 * mask
    dW2 = np.zeros((HID, 9))
    dW1 = np.zeros((HID, C_IN, 9))
    for c in range(HID):
        dH = np.zeros((nm, nm))
        for k, (dy, dx) in enumerate(OFFS):
            dW2[c, k] = np.sum(g * shifted(H[c], dy, dx))
            dH += W2[c, k] * shifted(g, -dy, -dx)
        dP = dH * mask * (P[c] > 0)
        for ci in range(C_IN):
            for k, (dy, dx) in enumerate(OFFS):
                dW1[c, ci, k] = np.sum(dP * shifted(X[ci], dy, dx))
    return L, join(dW1, dW2)


def jacobi_weights(omega):
    """A weight set whose network is exactly omega * rho: two hidden channels
    with centre taps +1 and -1 on rho, combined with +omega and -omega
    (omega ReLU(rho) - omega ReLU(-rho) = omega rho)."""
    W1 = np.zeros((HID, C_IN, 9))
    W2 = np.zeros((HID, 9))
    W1[0, 0, 4], W1[1, 0, 4] = 1.0, -1.0
    W2[0, 4], W2[1, 4] = omega, -omega
    return join(W1, W2)


def to_bf16(v):
    """Round FP64 values to the nearest BF16 value (ties to even), via FP32
    (FP64 -> FP32 round to nearest, then keep the top 16 bits of the FP32
    pattern with round-to-nearest-even on the dropped half)."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the master weights theta
    with gradient g; t is the 1-based step count.  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------- whole-grid task --

def lattice_coefficient(a, m):
    """The nodal coefficient on the level-m lattice (compact)."""
    if a is None:
        return None
    l = 1 << m
    return np.ascontiguousarray(a[::l, ::l])


def sweep(n, m, rm, e_old, w, a=None):
    """One whole-grid HOMG iteration at level m with the learned relaxation
    (2D): interior lattice nodes take x + y, every other node the multilinear
    interpolant of the previous iterate's lattice (the fused task of Sec. 2,
    interpolations delayed one iteration), boundary nodes 0."""
    l = 1 << m
    hl = l / (n - 1.0)
    e_new = O.prolong(2, n, m, e_old)
    x = np.ascontiguousarray(e_old[::l, ::l])
    xn = smooth_step(x, rm, lattice_coefficient(a, m), hl, w)
    e_new[::l, ::l][1:-1, 1:-1] = xn[1:-1, 1:-1]
    e_new[0, :] = e_new[-1, :] = 0.0
    e_new[:, 0] = e_new[:, -1] = 0.0
    return e_new


def mfmg_cycle(n, r0, schedule, w, a=None, levels=None):
    """One MFMG cycle on A e = r0 from e = 0 with the learned relaxation."""
    if levels is None:
        levels = 1 + max(m for m, _ in schedule)
    rs = O.pyramid(2, r0, levels)
    e = np.zeros((n, n))
    for m, iters in schedule:
        for _ in range(iters):
            e = sweep(n, m, rs[m], e, w, a)
    return e


def solve(n, f, w, a=None, *, tol=1e-10, max_cycles=100, max_i=4, fixed_cycles=None):
    """HOMG with the learned relaxation and the residual-equation restart;
    returns (u, history) as oracle.homg.solve does."""
    k = O.check_side(n)
    schedule = O.default_schedule(k, max_i)
    u = np.zeros((n, n))
    fn = np.sqrt(O.norm2_interior(2, n, f))
    denom = fn if fn > 0 else 1.0
    r, s = O.residual(2, n, f, u, a)
    hist = [np.sqrt(s) / denom]
    ncyc = fixed_cycles if fixed_cycles is not None else max_cycles
    for _ in range(ncyc):
        if fixed_cycles is None and hist[-1] <= tol:
            break
        u = u + mfmg_cycle(n, r, schedule, w, a, k)
        r, s = O.residual(2, n, f, u, a)
        hist.append(np.sqrt(s) / denom)
    return u, hist
