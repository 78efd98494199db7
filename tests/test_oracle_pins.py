"""Pins of the FP64 CPU oracle to facts the paper and the mathematics fix.

Each test checks the oracle (oracle/homg_oracle.c via oracle.homg) against
something that is not the oracle: closed forms, an independently assembled
dense matrix solved by LU, exact invariants of the operators, an
independently coded compact-lattice cascade, and the qualitative claims of
Sec. 4.  A plausible mistake (dropped term, wrong sign, wrong stride or
index, transposed operand, interpolation from the wrong iterate) fails at
least one of them.
"""
import numpy as np
import pytest

import workloads as W
from oracle import homg as O
from oracle import textbook as T


def inner(d):
    return (slice(1, -1),) * d


def rand_interior(rng, d, n):
    x = np.zeros((n,) * d)
    x[inner(d)] = rng.standard_normal((n - 2,) * d)
    return x


def A_apply(d, n, x, a=None):
    """A x through the oracle's residual with f = 0 (r = -A x)."""
    r, _ = O.residual(d, n, np.zeros((n,) * d), np.ascontiguousarray(x), a)
    return -r


# ---------------------------------------------------------------- operator --

@pytest.mark.parametrize("d,n", [(2, 17), (2, 33), (3, 9), (3, 17)])
@pytest.mark.parametrize("var", [False, True])
def test_A_symmetric(d, n, var):
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((n,) * d)) if var else None
    x, y = rand_interior(rng, d, n), rand_interior(rng, d, n)
    lhs = np.vdot(A_apply(d, n, x, a), y)
    rhs = np.vdot(x, A_apply(d, n, y, a))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


@pytest.mark.parametrize("d,n,ks", [(2, 33, (1, 1)), (2, 33, (3, 7)), (2, 65, (31, 2)),
                                    (3, 17, (1, 2, 3)), (3, 17, (15, 1, 8))])
def test_A_eigenpairs(d, n, ks):
    v = T.sine_mode(d, n, ks)
    lam = T.laplace_eigenvalue(d, n, ks)
    Av = A_apply(d, n, v)
    assert np.max(np.abs(Av[inner(d)] - lam * v[inner(d)])) <= 1e-10 * lam


@pytest.mark.parametrize("d,n", [(2, 9), (2, 17), (3, 9)])
def test_residual_matches_dense_assembly(d, n):
    rng = np.random.default_rng(2)
    a = np.exp(rng.standard_normal((n,) * d))
    u = rand_interior(rng, d, n)
    f = rng.standard_normal((n,) * d)
    for coef in (None, a):
        A = T.assemble_dense(d, n, coef)
        r, s = O.residual(d, n, f, u, coef)
        want = f[inner(d)].reshape(-1) - A @ u[inner(d)].reshape(-1)
        np.testing.assert_allclose(r[inner(d)].reshape(-1), want, rtol=0, atol=1e-11 * np.abs(A).max())
        assert np.all(r[0] == 0) and np.all(r[-1] == 0)
        assert s == pytest.approx(np.sum(want ** 2), rel=1e-12)


# ------------------------------------------------------ discrete solution --

@pytest.mark.parametrize("d,n", [(2, 9), (2, 17), (3, 9), (3, 17)])
def test_homg_converges_to_dense_lu(d, n):
    f = W.uniform(d, n, seed=3)
    ustar = T.dense_solve(d, n, f)
    u, hist = O.solve(d, n, f, tol=1e-14, max_cycles=60)
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(u - ustar)) <= 1e-12 * np.max(np.abs(ustar))


@pytest.mark.parametrize("n", [9, 17])
def test_homg_variable_coefficient_converges_to_dense_lu(n):
    a, f = W.grf_problem(n, seed=4)
    ustar = T.dense_solve(2, n, f, a)
    u, hist = O.solve(2, n, f, a=a, tol=1e-14, max_cycles=80)
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(u - ustar)) <= 1e-11 * np.max(np.abs(ustar))


def test_sine_problem_closed_form():
    """-Lap u = 2 pi^2 sin sin: the discrete solution is the same mode scaled
    by 2 pi^2 / lambda_h, lambda_h = (8/h^2) sin^2(pi h / 2), and its error
    against sin sin is pi^2 h^2 / 12 to leading order."""
    n = 129
    h = 1.0 / (n - 1)
    f = W.sine2d(n)
    u, hist = O.solve(2, n, f, tol=1e-12, max_cycles=60)
    lam = T.laplace_eigenvalue(2, n, (1, 1))
    uh = (2 * np.pi ** 2 / lam) * W.sine2d_exact(n)
    # rigorous a-posteriori bound ||u - u*||_2 <= ||r||_2 / lambda_min
    r, s = O.residual(2, n, f, u)
    assert np.linalg.norm(u - uh) <= np.sqrt(s) / lam * (1 + 1e-6) + 1e-14
    assert np.linalg.norm(u - uh) / np.linalg.norm(uh) <= 1e-11
    rel = 2 * np.pi ** 2 / lam - 1
    assert rel == pytest.approx(np.pi ** 2 * h ** 2 / 12, rel=1e-3)


def test_textbook_vcycle_second_order():
    """The independent textbook V-cycle converges to the discrete solution,
    whose error against the manufactured continuous solution falls as h^2."""
    errs = []
    for n in (33, 65, 129):
        f = W.sine2d(n)
        vc = T.VCycle(2, n)
        u, hist = vc.solve(f, tol=1e-13)
        assert hist[-1] <= 1e-12
        errs.append(np.max(np.abs(u - W.sine2d_exact(n))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - 2.0) < 0.02 for r in rates), rates


@pytest.mark.parametrize("d,n", [(2, 65), (3, 17)])
def test_homg_within_rigorous_bound_of_textbook(d, n):
    f = W.uniform(d, n, seed=5)
    ustar, vh = T.VCycle(d, n).solve(f, tol=1e-14)
    assert vh[-1] <= 1e-13
    h = 1.0 / (n - 1)
    lam_min = (4 * d / h ** 2) * np.sin(np.pi * h / 2) ** 2
    for cycles in (1, 3, 8):
        u, hist = O.solve(d, n, f, fixed_cycles=cycles)
        r, s = O.residual(d, n, f, u)
        assert np.linalg.norm(u - ustar) <= np.sqrt(s) / lam_min * (1 + 1e-9) + 1e-15


# ------------------------------------------------- restriction, interpolation --

@pytest.mark.parametrize("d,nf,ks", [(2, 33, (1, 1)), (2, 33, (5, 11)), (3, 17, (3, 1, 5)), (3, 17, (7, 7, 2))])
def test_full_weighting_of_sine_mode(d, nf, ks):
    """FW maps the fine mode prod sin(k pi x) to prod cos^2(k pi h/2) times the
    same mode on the coarse nodes (exact for modes vanishing on the boundary)."""
    hf = 1.0 / (nf - 1)
    v = T.sine_mode(d, nf, ks)
    rc = O.restrict(d, v)
    nc = (nf - 1) // 2 + 1
    want = np.prod([np.cos(k * np.pi * hf / 2) ** 2 for k in ks]) * T.sine_mode(d, nc, ks)
    assert np.max(np.abs(rc - want)) <= 1e-14


@pytest.mark.parametrize("d,nf", [(2, 17), (3, 9)])
def test_full_weighting_adjoint_of_interpolation(d, nf):
    """<FW x, y>_coarse = 2^-d <x, S y>_fine."""
    rng = np.random.default_rng(6)
    nc = (nf - 1) // 2 + 1
    x = rand_interior(rng, d, nf)
    y = rand_interior(rng, d, nc)
    yfine = np.zeros((nf,) * d)
    yfine[(slice(None, None, 2),) * d] = y
    Sy = O.prolong(d, nf, 1, yfine)
    lhs = np.vdot(O.restrict(d, x), y)
    rhs = np.vdot(x, Sy) / 2 ** d
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_full_weighting_matches_textbook_and_constants():
    rng = np.random.default_rng(7)
    for d, n in ((2, 33), (3, 17)):
        x = rand_interior(rng, d, n)
        np.testing.assert_allclose(O.restrict(d, x), T.fw_restrict(x), rtol=0, atol=1e-15)
        c = np.zeros((n,) * d)
        c[inner(d)] = 1.0
        rc = O.restrict(d, c)
        # coarse nodes whose stencil avoids the fine boundary see the constant
        assert np.allclose(rc[(slice(2, -2),) * d], 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,n,m", [(2, 33, 1), (2, 33, 3), (2, 65, 5), (3, 17, 1), (3, 17, 2), (3, 17, 3)])
def test_interpolation_reproduces_multilinear(d, n, m):
    x = np.linspace(0, 1, n)
    grids = np.meshgrid(*([x] * d), indexing="ij")
    rng = np.random.default_rng(8)
    c = rng.standard_normal(2 ** d)
    g = np.zeros((n,) * d)
    for b in range(2 ** d):
        term = np.full((n,) * d, c[b])
        for axis in range(d):
            if (b >> axis) & 1:
                term = term * grids[axis]
        g = g + term
    e = np.zeros((n,) * d)
    lat = (slice(None, None, 1 << m),) * d
    e[lat] = g[lat]
    out = O.prolong(d, n, m, e)
    assert np.max(np.abs(out - g)) <= 1e-13


def test_interpolation_equals_composed_linear_interpolation():
    """Direct multilinear interpolation from level m equals m one-level
    linear interpolations (the textbook prolongation) applied in turn."""
    rng = np.random.default_rng(9)
    for d, n, m in ((2, 65, 4), (3, 17, 3)):
        l = 1 << m
        nc = (n - 1) // l + 1
        ec = rand_interior(rng, d, nc)
        want = ec
        for _ in range(m):
            want = T.lin_interp(want)
        e = np.zeros((n,) * d)
        e[(slice(None, None, l),) * d] = ec
        assert np.max(np.abs(O.prolong(d, n, m, e) - want)) <= 1e-14


# -------------------------------------------------------------- relaxation --

@pytest.mark.parametrize("d,n,m,ks", [(2, 65, 0, (3, 5)), (2, 65, 2, (1, 6)), (3, 17, 0, (2, 3, 5)), (3, 33, 2, (1, 2, 3))])
def test_jacobi_damps_eigenmode_by_its_factor(d, n, m, ks):
    """With zero right-hand side the level-m relaxation multiplies a lattice
    eigenmode by 1 - omega (1 - (1/d) sum cos(k_i pi h_l))."""
    l = 1 << m
    h = 1.0 / (n - 1)
    omega = O.default_omega(d)
    v = T.sine_mode(d, n, ks)
    nm = (n - 1) // l + 1
    e_new = O.sweep(d, n, m, omega, np.zeros((nm,) * d), v)
    g = 1 - omega * (1 - np.mean([np.cos(k * np.pi * h * l) for k in ks]))
    lat = (slice(l, -1, l),) * d
    np.testing.assert_allclose(e_new[lat], g * v[lat], rtol=0, atol=1e-13)


@pytest.mark.parametrize("d,n,m", [(2, 33, 1), (2, 33, 2), (3, 17, 1)])
@pytest.mark.parametrize("var", [False, True])
def test_level_relaxation_fixed_point_is_level_system(d, n, m, var):
    """Iterating level-m sweeps with a fixed r_m drives the lattice values to
    the solution of the level-m system (spacing h_l = 2^m h) by LU."""
    rng = np.random.default_rng(10)
    l = 1 << m
    nm = (n - 1) // l + 1
    a = np.exp(rng.standard_normal((n,) * d)) if var else None
    rm = rand_interior(rng, d, nm)
    # the level-m system: A on the compact grid with the lattice coefficients
    am = None if a is None else np.ascontiguousarray(a[(slice(None, None, l),) * d])
    Am = T.assemble_dense(d, nm, am)  # compact side nm has spacing 1/(nm-1) = h_l
    want = np.linalg.solve(Am, rm[inner(d)].reshape(-1)).reshape((nm - 2,) * d)
    e = np.zeros((n,) * d)
    for _ in range(3000):
        e = O.sweep(d, n, m, O.default_omega(d), rm, e, a)
    got = e[(slice(l, -1, l),) * d]
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


# ----------------------------------------------------- the fused HOMG cycle --

def compact_cascade(d, n, r0, schedule, omega):
    """Independent formulation of one MFMG cycle: at each level, Jacobi on the
    compact lattice grid, then the whole grid is S_m (composed one-level
    linear interpolations) of the second-to-last lattice iterate with the
    last iterate on the interior lattice (the one-iteration delay)."""
    levels = 1 + max(m for m, _ in schedule)
    h = 1.0 / (n - 1)
    rs = [r0]
    for _ in range(1, levels):
        rs.append(T.fw_restrict(rs[-1]))
    E = np.zeros((n,) * d)
    for m, iters in schedule:
        l = 1 << m
        lat = (slice(None, None, l),) * d
        x = E[lat].copy()
        hm = l * h
        dg = T.diag_A(x.shape, hm)
        prev = x
        for _ in range(iters):
            prev = x
            x = x.copy()
            x[inner(d)] = prev[inner(d)] + omega * (rs[m] - T.apply_A(prev, hm))[inner(d)] / dg
        E = prev
        for _ in range(m):
            E = T.lin_interp(E)
        Elat = E[lat]
        Elat[inner(d)] = x[inner(d)]
        E[lat] = Elat
    return E


@pytest.mark.parametrize("d,n,max_i", [(2, 33, 4), (2, 65, 2), (2, 65, 32), (3, 17, 4), (3, 33, 8)])
def test_lattice_independence_identity(d, n, max_i):
    f = W.uniform(d, n, seed=11)
    k = O.check_side(n)
    sched = O.default_schedule(k, max_i)
    omega = O.default_omega(d)
    r0, _ = O.residual(d, n, f, np.zeros_like(f))
    e = O.mfmg_cycle(d, n, r0, sched, omega)
    want = compact_cascade(d, n, r0, sched, omega)
    assert np.max(np.abs(e - want)) <= 1e-13 * np.max(np.abs(want))


def test_fig3_spike_then_pyramid():
    """Sec. 4, Fig. 3: iteration 1 is a spike (only the middle node relaxes,
    interpolations have null sources); iteration 2 has the relaxation stalled
    and the interpolated nodes forming the pyramid of the zero mode."""
    n = 129
    f, _ = W.poly2d(n)
    omega = O.default_omega(2)
    k = O.check_side(n)
    sched = O.default_schedule(k, 2)
    r0, _ = O.residual(2, n, f, np.zeros_like(f))
    _, states = O.mfmg_cycle(2, n, r0, sched, omega, keep_states=True)
    # restricted source at the single coarsest unknown, by the textbook FW
    rM = r0
    for _ in range(k - 1):
        rM = T.fw_restrict(rM)
    hM = 0.5
    c = n // 2
    e1 = states[0]
    spike = (omega / 4) * hM ** 2 * rM[1, 1]
    assert e1[c, c] == pytest.approx(spike, rel=1e-14)
    e1z = e1.copy()
    e1z[c, c] = 0.0
    assert np.all(e1z == 0.0)
    e2 = states[1]
    x = np.linspace(0, 1, n)
    hat = 1 - 2 * np.abs(x - 0.5)
    pyr = spike * np.outer(hat, hat)
    pyr[c, c] = e2[c, c]
    assert np.max(np.abs(e2 - pyr)) <= 1e-15 * abs(spike) * 10
    # the centre takes its second Jacobi value: neighbours at +-64 are boundary
    assert e2[c, c] == pytest.approx(spike + (omega / 4) * (hM ** 2 * rM[1, 1] - 4 * spike), rel=1e-13)
    # iteration 3 is the first iteration of the next finer level: its 3x3
    # interior lattice relaxes, so the values at +-32 change from the pyramid
    assert len(states) == sum(it for _, it in sched)


def test_default_schedule_counts():
    assert O.default_schedule(7, 4) == [(6, 2), (5, 4), (4, 4), (3, 4), (2, 4), (1, 4), (0, 4)]
    assert O.default_schedule(7, 2) == [(m, 2) for m in range(6, -1, -1)]
    # sweeps per cycle of the workloads at MaxI = 4 and 32
    for levels, s4, s32 in ((7, 26, 126), (12, 46, 286), (8, 30, 158), (9, 34, 190), (10, 38, 222)):
        assert sum(i for _, i in O.default_schedule(levels, 4)) == s4
        assert sum(i for _, i in O.default_schedule(levels, 32)) == s32


# ------------------------------------------------- outer iteration, Sec. 4 --

def test_contraction_independent_of_resolution():
    """Sec. 4: cycles with the same MaxI descend over the same convergence
    path for different resolutions (h-independent contraction)."""
    rates = []
    for n in (33, 65, 129, 257):
        f = W.uniform(2, n, seed=12)
        _, hist = O.solve(2, n, f, fixed_cycles=6)
        rates.append((hist[6] / hist[2]) ** 0.25)
    assert max(rates) < 0.3
    assert max(rates) - min(rates) < 0.03, rates


def test_linear_work_cycles_to_tolerance_flat_in_n():
    cyc = []
    for n in (33, 65, 129, 257):
        _, hist = O.solve(2, n, W.uniform(2, n, seed=13), tol=1e-10)
        cyc.append(len(hist) - 1)
    assert max(cyc) - min(cyc) <= 3, cyc


def test_larger_maxi_reaches_lower_error():
    """Sec. 4: one MFMG cycle on the polynomial problem; the normalised L1
    error is (nearly) the same across resolutions and lower for larger MaxI."""
    res = {}
    for max_i in (4, 32):
        errs = []
        for n in (65, 129, 257):
            f, uex = W.poly2d(n)
            u, _ = O.solve(2, n, f, max_i=max_i, fixed_cycles=1)
            errs.append(np.sum(np.abs(uex - u)) / np.sum(np.abs(uex)))
        res[max_i] = errs
        assert max(errs) - min(errs) < 0.02, errs
    assert max(res[32]) < min(res[4])


def test_variable_coefficient_contraction():
    """-div(a grad) with a = exp(GRF): HOMG still converges to 1e-10; the
    measured per-cycle contraction is slower than for the Laplacian and grows
    with MaxI decreasing (measured, not fixed by the paper)."""
    a, f = W.grf_problem(129, seed=14)
    rates = {}
    for max_i in (4, 32):
        _, hist = O.solve(2, 129, f, a=a, tol=1e-10, max_cycles=100, max_i=max_i)
        assert hist[-1] <= 1e-10
        rates[max_i] = (hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2))
    assert rates[32] < rates[4] < 0.9, rates
