"""Pins of the learned-smoother oracle (oracle/learned.py) to facts that do
not come from it: the HOMG oracle's damped Jacobi (C code), a library
correlation (scipy.signal.correlate2d), a dense matrix assembled face by
face, central finite differences of the loss, torch's Adam and torch's
BF16 conversion.  All CPU."""
import numpy as np
import pytest
import scipy.signal
import torch

import workloads as W
from oracle import homg as O
from oracle import learned as L
from oracle import textbook as T


def rand_interior(rng, nm):
    x = np.zeros((nm, nm))
    x[1:-1, 1:-1] = rng.standard_normal((nm - 2, nm - 2))
    return x


def rand_weights(rng, scale=0.3):
    return rng.standard_normal(L.NW) * scale


def grf_coef(nm, seed):
    a, _ = W.grf_problem(nm, seed=seed)
    return a


# ------------------------------------------------------------ forward --

@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("m", [0, 1, 3])
def test_jacobi_weights_reproduce_the_homg_sweep(var, m):
    """With the Jacobi-equivalent weights the learned whole-grid iteration is
    the HOMG oracle's damped-Jacobi iteration (C code, whole grid)."""
    n = 65
    rng = np.random.default_rng(10 + m)
    a = grf_coef(n, 3) if var else None
    l = 1 << m
    nm = (n - 1) // l + 1
    e = rand_interior(rng, n)
    rm = rand_interior(rng, nm)
    omega = 0.8
    got = L.sweep(n, m, rm, e, L.jacobi_weights(omega), a)
    want = O.sweep(2, n, m, omega, rm, e, a)
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_jacobi_weights_reproduce_a_whole_solve():
    n = 33
    a, f = W.grf_problem(n, seed=5)
    u1, h1 = L.solve(n, f, L.jacobi_weights(0.8), a, fixed_cycles=4)
    u2, h2 = O.solve(2, n, f, a=a, fixed_cycles=4)
    assert np.linalg.norm(u1 - u2) <= 1e-12 * np.linalg.norm(u2)
    np.testing.assert_allclose(h1, h2, rtol=1e-9)


@pytest.mark.parametrize("nm", [5, 9, 17])
def test_forward_matches_library_correlation(nm):
    """The network against scipy's 2D correlation (zero fill outside): catches
    a flipped kernel, swapped channels or a wrong weight layout."""
    rng = np.random.default_rng(nm)
    X = np.zeros((L.C_IN, nm, nm))
    X[:, 1:-1, 1:-1] = rng.standard_normal((L.C_IN, nm - 2, nm - 2))
    w = rand_weights(rng)
    W1 = w[:L.NW1].reshape(L.HID, L.C_IN, 3, 3)   # [c][ci][dy+1][dx+1]
    W2 = w[L.NW1:].reshape(L.HID, 3, 3)
    inner = np.zeros((nm, nm))
    inner[1:-1, 1:-1] = 1.0
    H = np.zeros((L.HID, nm, nm))
    for c in range(L.HID):
        pre = sum(scipy.signal.correlate2d(X[ci], W1[c, ci], mode="same", boundary="fill")
                  for ci in range(L.C_IN))
        H[c] = np.maximum(pre, 0.0) * inner
    y = sum(scipy.signal.correlate2d(H[c], W2[c], mode="same", boundary="fill")
            for c in range(L.HID)) * inner
    _, Hg, yg = L.forward(X, w)
    assert np.max(np.abs(Hg - H)) <= 1e-13 * np.max(np.abs(H))
    assert np.max(np.abs(yg - y)) <= 1e-13 * np.max(np.abs(y))


def test_single_tap_moves_the_right_way():
    """A single +x tap of W1 on channel 0 and the centre tap of W2: y(p) =
    ReLU(rho(p + x)) -- the correlation reads the neighbour at +x."""
    nm = 9
    X = np.zeros((L.C_IN, nm, nm))
    X[0, 4, 5] = 2.0
    W1 = np.zeros((L.HID, L.C_IN, 9))
    W2 = np.zeros((L.HID, 9))
    W1[3, 0, 5] = 1.0   # k = 3 (dy + 1) + (dx + 1) = 3*1 + 2: (dy, dx) = (0, +1)
    W2[3, 4] = 1.0
    _, _, y = L.forward(X, L.join(W1, W2))
    assert y[4, 4] == 2.0 and np.count_nonzero(y) == 1


def test_scale_equivariance_and_boundary():
    rng = np.random.default_rng(4)
    nm = 17
    a = grf_coef(nm, 7)
    x, rm = rand_interior(rng, nm), rand_interior(rng, nm)
    w = rand_weights(rng)
    X = L.features(x, rm, a, 1 / 16)
    _, _, y = L.forward(X, w)
    _, _, y3 = L.forward(3.5 * X, w)
    assert np.max(np.abs(y3 - 3.5 * y)) <= 1e-13 * np.max(np.abs(y3))
    assert not np.any(y[0]) and not np.any(y[-1]) and not np.any(y[:, 0]) and not np.any(y[:, -1])
    # constant coefficient: the anisotropy channels vanish
    Xc = L.features(x, rm, None, 1 / 16)
    assert not np.any(Xc[1]) and not np.any(Xc[2])


def test_features_against_dense_operator():
    """rho = D^-1 (h_l^2 r - A_m x) with A_m and its diagonal from the dense
    face-by-face assembly."""
    rng = np.random.default_rng(6)
    nm = 9
    a = grf_coef(nm, 8)
    hl = 0.25
    x, rm = rand_interior(rng, nm), rand_interior(rng, nm)
    A = T.assemble_dense(2, nm, a) * (1.0 / (nm - 1)) ** 2   # unscaled level operator
    xi = x[1:-1, 1:-1].reshape(-1)
    rho = (hl * hl * rm[1:-1, 1:-1].reshape(-1) - A @ xi) / np.diag(A)
    X = L.features(x, rm, a, hl)
    assert np.max(np.abs(X[0, 1:-1, 1:-1].reshape(-1) - rho)) <= 1e-13 * np.max(np.abs(rho))
    # anisotropy channels: (a_E - a_W) / (a_E + a_W) from the dense couplings
    i, j = 3, 4
    p = (j - 1) * (nm - 2) + (i - 1)
    aE, aW = -A[p, p + 1], -A[p, p - 1]
    aN, aS = -A[p, p + (nm - 2)], -A[p, p - (nm - 2)]
    assert X[1, j, i] == pytest.approx(X[0, j, i] * (aE - aW) / (aE + aW), rel=1e-13)
    assert X[2, j, i] == pytest.approx(X[0, j, i] * (aN - aS) / (aN + aS), rel=1e-13)


# ------------------------------------------------------------ loss --

def test_energy_against_dense_matrix():
    rng = np.random.default_rng(9)
    nm = 9
    a = grf_coef(nm, 9)
    v = rand_interior(rng, nm)
    A = T.assemble_dense(2, nm, a) * (1.0 / (nm - 1)) ** 2
    vi = v[1:-1, 1:-1].reshape(-1)
    assert L.energy(v, a) == pytest.approx(vi @ A @ vi, rel=1e-13)


def test_loss_of_jacobi_is_its_energy_contraction():
    """With the Jacobi weights, L = E((I - omega D^-1 A) delta) / E(delta),
    computed with the dense matrix; zero weights give L = 1."""
    rng = np.random.default_rng(11)
    nm, hl = 9, 0.125
    a = grf_coef(nm, 10)
    A = T.assemble_dense(2, nm, a) * (1.0 / (nm - 1)) ** 2
    x, xs = rand_interior(rng, nm), rand_interior(rng, nm)
    rm = np.zeros((nm, nm))
    rm[1:-1, 1:-1] = (A @ xs[1:-1, 1:-1].reshape(-1)).reshape(nm - 2, nm - 2) / hl ** 2
    delta = (xs - x)[1:-1, 1:-1].reshape(-1)
    after = delta - 0.8 * (A @ delta) / np.diag(A)
    want = (after @ A @ after) / (delta @ A @ delta)
    d2 = np.zeros((nm, nm))
    d2[1:-1, 1:-1] = delta.reshape(nm - 2, nm - 2)
    assert L.loss(x, rm, a, hl, d2, L.jacobi_weights(0.8)) == pytest.approx(want, rel=1e-12)
    assert L.loss(x, rm, a, hl, d2, np.zeros(L.NW)) == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("var", [False, True])
def test_gradient_against_central_differences(var):
    rng = np.random.default_rng(12)
    nm, hl = 9, 0.125
    a = grf_coef(nm, 12) if var else None
    x, rm, delta = rand_interior(rng, nm), rand_interior(rng, nm), rand_interior(rng, nm)
    w = rand_weights(rng)
    Lv, g = L.loss_and_grad(x, rm, a, hl, delta, w)
    assert Lv == pytest.approx(L.loss(x, rm, a, hl, delta, w), rel=1e-14)
    eps = 1e-6
    idx = list(rng.choice(L.NW1, 40, replace=False)) + list(L.NW1 + rng.choice(L.NW - L.NW1, 30, replace=False))
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (L.loss(x, rm, a, hl, delta, wp) - L.loss(x, rm, a, hl, delta, wm)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) * np.max(np.abs(g)), (i, fd, g[i])


# ------------------------------------------------------------ optimiser, rounding --

def test_adam_matches_torch():
    rng = np.random.default_rng(13)
    theta0 = rng.standard_normal(L.NW)
    grads = [rng.standard_normal(L.NW) for _ in range(5)]
    p = torch.nn.Parameter(torch.tensor(theta0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    theta, m, v = theta0.copy(), np.zeros(L.NW), np.zeros(L.NW)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        theta, m, v = L.adam_step(theta, g, m, v, t, 1e-2)
        np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(14)
    v = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.8, -0.8, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 0.0]])
    want = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(L.to_bf16(v), want)
    assert L.to_bf16(np.array([0.8]))[0] == 0.80078125
