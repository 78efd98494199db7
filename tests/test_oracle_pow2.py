"""Pins of the power-of-two grid oracle (Sec. 3; oracle/pow2_oracle.c).

Each pin checks the oracle against something fixed outside it:
  * the discrete solution by dense LU on 8^2, 16^2 and 32^2 grids;
  * bilinear functions, which the subdomain-local interpolation must
    reproduce exactly, and the absence of cross-subdomain reads;
  * the closed form of full weighting on a sine mode, seen from each
    quadrant's corner (weights, offsets and the mirroring of every family);
  * the closed-form eigenvalue damping of damped Jacobi at level m for
    marks whose stencil stays inside one quadrant's lattice;
  * the zero mode: every quadrant has one interior point at the coarsest
    level (the point just outside it), and the first two iterations of a
    cycle give four spikes, then four pyramids (Sec. 4, Fig. 3 text: only
    the middle points relax);
  * the mirror symmetries of the square;
  * planted mistakes in a copy of the C source, each caught by a pin.
"""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import homg as O
from oracle import pow2 as P2
from oracle import textbook as T

OMEGA = 0.8


def rand_f(N, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((N, N))
    f[1:-1, 1:-1] = rng.uniform(-1, 1, (N - 2, N - 2))
    return f


@pytest.mark.parametrize("N", [8, 16, 32])
def test_converges_to_dense_lu(N):
    f = rand_f(N, 3 + N)
    u, hist = P2.solve(N, f, tol=1e-13, max_cycles=80)
    assert hist[-1] <= 1e-13
    us = T.dense_solve(2, N, f)
    assert np.linalg.norm(u - us) <= 1e-11 * np.linalg.norm(us)


def test_contraction_like_nested_grids():
    """The per-cycle contraction stays h-independent and of the size the
    nested 2^k + 1 grids give (no slowdown from the four subdomains)."""
    rates = []
    for N in (16, 32, 64, 128):
        _, hist = P2.solve(N, rand_f(N, 5), fixed_cycles=8)
        rates.append((hist[8] / hist[3]) ** 0.2)
    assert max(rates) < 0.32, rates
    assert max(rates) - min(rates) < 0.08, rates


@pytest.mark.parametrize("N,m", [(16, 1), (16, 3), (64, 2), (64, 5)])
def test_interpolation_reproduces_bilinear(N, m):
    x = np.arange(N) / (N - 1)
    rng = np.random.default_rng(N + m)
    c = rng.standard_normal(4)
    g = c[0] + c[1] * x[None, :] + c[2] * x[:, None] + c[3] * np.outer(x, x)
    out = P2.prolong(N, m, np.ascontiguousarray(g))
    assert np.max(np.abs(out - g)) <= 1e-13 * np.max(np.abs(g))


@pytest.mark.parametrize("N,m", [(16, 2), (64, 3)])
def test_no_cross_subdomain_interpolation(N, m):
    """Changing the marks of one quadrant changes the interpolated values
    of that quadrant's nodes only."""
    rng = np.random.default_rng(7)
    e = rng.standard_normal((N, N))
    mk = P2.marks(N, m)
    base = P2.prolong(N, m, e)
    jj, ii = np.indices((N, N))
    owner = (ii >= N // 2).astype(int) + 2 * (jj >= N // 2).astype(int)
    for q in range(4):
        e2 = e.copy()
        e2[mk == 1 + q] += 1.0
        diff = P2.prolong(N, m, e2) != base
        assert diff.any()
        assert np.all(owner[diff] == q)


def test_marks_reach_just_outside_their_subdomain():
    N = 64
    k = P2.check_side(N)
    for m in range(1, k):
        mk = P2.marks(N, m)
        l = 1 << m
        for q in range(4):
            sx, sy = q & 1, q >> 1
            jj, ii = np.nonzero(mk == 1 + q)
            ax = ii if sx == 0 else N - 1 - ii
            ay = jj if sy == 0 else N - 1 - jj
            assert ax.max() == N // 2 and ay.max() == N // 2
            assert np.all(ax % l == 0) and np.all(ay % l == 0)
            assert len(ii) == (N // (2 * l) + 1) ** 2
    # coarsest level: one interior point per quadrant, the four central nodes
    mk = P2.marks(N, k - 1)
    inner = mk[1:-1, 1:-1]
    jj, ii = np.nonzero(inner)
    pts = sorted(zip(jj + 1, ii + 1))
    assert pts == [(N // 2 - 1, N // 2 - 1), (N // 2 - 1, N // 2), (N // 2, N // 2 - 1), (N // 2, N // 2)]


@pytest.mark.parametrize("N,ks", [(32, (1, 1)), (64, (3, 2)), (64, (5, 7))])
def test_family_restriction_of_sine_mode(N, ks):
    """Full weighting maps sin(k pi x) to cos^2(k pi h_j / 2) sin(k pi x) at
    every interior node; seen from each corner, every family level j holds
    the mode (mirrored) times the product of those factors."""
    x = np.arange(N) / (N - 1)
    h = 1.0 / (N - 1)
    r0 = np.outer(np.sin(ks[1] * np.pi * x), np.sin(ks[0] * np.pi * x))
    r0[0, :] = r0[-1, :] = 0.0
    r0[:, 0] = r0[:, -1] = 0.0
    k = P2.check_side(N)
    fam = P2.families(r0, k)
    for j in range(1, k):
        fac = 1.0
        for t in range(j):
            hj = h * (1 << t)
            fac *= np.cos(ks[0] * np.pi * hj / 2) ** 2 * np.cos(ks[1] * np.pi * hj / 2) ** 2
        s = N >> j
        A = np.arange(s) << j
        for q in range(4):
            sx, sy = q & 1, q >> 1
            gi = A if sx == 0 else N - 1 - A
            gj = A if sy == 0 else N - 1 - A
            want = fac * r0[np.ix_(gj, gi)]
            got = fam[j][q]
            assert np.max(np.abs(got[1:, 1:] - want[1:, 1:])) <= 1e-13, (j, q)
            assert np.all(got[0, :] == 0) and np.all(got[:, 0] == 0)


def test_level_relaxation_damps_eigenmode():
    """At a level-m mark whose neighbours at distance l are marks of the same
    quadrant, with zero source, damped Jacobi multiplies a lattice eigenmode
    by 1 - omega (1 - (cos(k1 pi h_l) + cos(k2 pi h_l)) / 2)."""
    N, m = 64, 2
    l = 1 << m
    x = np.arange(N) / (N - 1)
    hl = l / (N - 1)
    ks = (3, 5)
    e = np.outer(np.sin(ks[1] * np.pi * x), np.sin(ks[0] * np.pi * x))
    zero = [np.zeros((N >> m, N >> m))] * 4
    out = P2.sweep(N, m, OMEGA, zero, e)
    fac = 1 - OMEGA * (1 - 0.5 * (np.cos(ks[0] * np.pi * hl) + np.cos(ks[1] * np.pi * hl)))
    mk = P2.marks(N, m)
    checked = 0
    for j in range(l, N // 2 - l, l):
        for i in range(l, N // 2 - l, l):
            assert mk[j, i] == 1
            assert out[j, i] == pytest.approx(fac * e[j, i], abs=1e-13)
            checked += 1
    assert checked > 20


def test_fig3_four_spikes_then_four_pyramids():
    N = 64
    k = P2.check_side(N)
    M = k - 1
    f, _ = W.poly2d(N)  # the Sec. 4 source on the power-of-two grid
    r0, _ = O.residual(2, N, f, np.zeros_like(f))
    sched = P2.default_schedule(k, 2)
    _, states = P2.mfmg_cycle(N, r0, sched, OMEGA, keep_states=True)
    fam = P2.families(r0, k)
    hM = (N // 2) / (N - 1)
    e1, e2 = states[0], states[1]
    centre = {0: (N // 2, N // 2), 1: (N // 2, N // 2 - 1), 2: (N // 2 - 1, N // 2), 3: (N // 2 - 1, N // 2 - 1)}
    nz = np.argwhere(e1 != 0)
    assert sorted(map(tuple, nz)) == sorted(centre.values())
    for q, (j, i) in centre.items():
        assert e1[j, i] == pytest.approx((OMEGA / 4) * hM ** 2 * fam[M][q][1, 1], rel=1e-14)
        # relaxations stall: the neighbours at distance N/2 are boundary or outside
        assert e2[j, i] == pytest.approx(e1[j, i] + (OMEGA / 4) * (hM ** 2 * fam[M][q][1, 1] - 4 * e1[j, i]),
                                         rel=1e-13)
    # every other node is the bilinear pyramid of its own quadrant's centre
    x = np.arange(N)
    for q, (cj, ci) in centre.items():
        sx, sy = q & 1, q >> 1
        wx = (x if sx == 0 else N - 1 - x) / (N // 2)
        wy = (x if sy == 0 else N - 1 - x) / (N // 2)
        ii = np.nonzero((x >= N // 2) == bool(sx))[0]
        jj = np.nonzero((x >= N // 2) == bool(sy))[0]
        pyr = e1[cj, ci] * np.outer(wy[jj], wx[ii])
        got = e2[np.ix_(jj, ii)].copy()
        mk = P2.marks(N, M)[np.ix_(jj, ii)]
        sel = mk == 0
        assert np.max(np.abs(got[sel] - pyr[sel])) <= 1e-14 * abs(e1[cj, ci])
    assert np.all(e2[1:-1, 1:-1] != 0)  # the zero mode covers the whole square


def test_mirror_symmetry():
    N = 32
    f = rand_f(N, 11)
    u, _ = P2.solve(N, f, fixed_cycles=3)
    for flip in (lambda a: a[:, ::-1], lambda a: a[::-1, :], lambda a: a.T):
        uf, _ = P2.solve(N, np.ascontiguousarray(flip(f)), fixed_cycles=3)
        assert np.max(np.abs(uf - flip(u))) <= 1e-12 * np.max(np.abs(u))


# ------------------------------------------------- planted mistakes

SRC = os.path.join(os.path.dirname(O.__file__), "pow2_oracle.c")
SRC_NESTED = os.path.join(os.path.dirname(O.__file__), "homg_oracle.c")

MUTANTS = {
    "no_just_outside_marks": ("if (a % l == 0 && a <= N / 2) return s;", "if (a % l == 0 && a < N / 2) return s;"),
    "cross_domain_interp": ("const int sx = i >= N / 2, sy = j >= N / 2;", "const int sx = 0, sy = 0;"),
    "family_not_mirrored": ("F[at(N, b, a)] = r0[at(N, local_of(N, sy, b), local_of(N, sx, a))];",
                            "F[at(N, b, a)] = r0[at(N, b, a)];"),
    "relax_stride_one": ("double nb = ev(N, e_old, j, i - l) + ev(N, e_old, j, i + l) + ev(N, e_old, j - l, i) +\n"
                         "                        ev(N, e_old, j + l, i);",
                         "double nb = ev(N, e_old, j, i - 1) + ev(N, e_old, j, i + 1) + ev(N, e_old, j - 1, i) +\n"
                         "                        ev(N, e_old, j + 1, i);"),
    "restrict_weight": ("double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.5 : 0.25);",
                        "double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.25 : 0.5);"),
    "restrict_offset": ("s += w * F[at(nf, 2 * B + oy, 2 * A + ox)];", "s += w * F[at(nf, 2 * B + oy, 2 * A + 2 * ox)];"),
    "interp_weight": ("double w = (bx ? tx : 1.0 - tx) * (by ? ty : 1.0 - ty);",
                      "double w = (bx ? 1.0 - tx : tx) * (by ? ty : 1.0 - ty);"),
}


def _pins():
    yield lambda: test_converges_to_dense_lu(16)
    yield lambda: test_interpolation_reproduces_bilinear(16, 2)
    yield lambda: test_no_cross_subdomain_interpolation(16, 2)
    yield lambda: test_family_restriction_of_sine_mode(32, (1, 1))
    yield test_level_relaxation_damps_eigenmode
    yield test_fig3_four_spikes_then_four_pyramids
    yield test_marks_reach_just_outside_their_subdomain


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / ("libmut_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    SRC_NESTED, str(mut), "-o", str(so), "-lm"], check=True)
    P2.use_library(str(so))
    try:
        failed = 0
        for pin in _pins():
            try:
                pin()
            except AssertionError:
                failed += 1
        assert failed >= 1, "no pin caught " + name
    finally:
        P2.use_library(None)
