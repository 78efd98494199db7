"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Element by element on the same seeded inputs.  Tolerances, derived from the
arithmetic:
  * FP64 kernels: a few ulp per node formula; single steps within
    1e-12 * max|expected|, whole solves within 1e-11 relative in u at the
    same cycle count (the benchmark spec's bound).
  * FP32 steps: within 1e-5 * max|expected| (a few FP32 ulp, 2^-24 each).
  * BF16 steps: inputs are made exactly representable in BF16; the GPU
    rounds its FP32 result to BF16 and the expectation is the FP64 result
    rounded to BF16, so the two may sit one BF16 ulp apart (at most 2^-7
    relative): within 2^-7 * |expected| + 1e-5 * max|expected| per node.
  * Residual history: within 1e-6 relative plus the rounding floor of the
    residual itself, 16 eps || |A| |u| ||_2 / ||f||_2, since two correct
    FP64 residuals of nearly the same u differ by that much.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import homg as O

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def B(torch_cuda):
    import paper_1108_2045_amd as P
    return P


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rand_interior(rng, d, n):
    x = np.zeros((n,) * d)
    x[(slice(1, -1),) * d] = rng.standard_normal((n - 2,) * d)
    return x


def representable(torch, x, prec):
    """Round test inputs so the GPU's conversion to `prec` is exact."""
    if prec == "fp64":
        return x
    dt = torch.float32 if prec == "fp32" else torch.bfloat16
    return torch.from_numpy(x).to(dt).to(torch.float64).numpy()


def step_tol(prec, want):
    mx = np.max(np.abs(want)) if want.size else 0.0
    if prec == "fp64":
        return 1e-12 * mx + 1e-300
    if prec == "fp32":
        return 1e-5 * mx + 1e-300
    return 2.0 ** -7 * np.abs(want) + 1e-5 * mx + 1e-300


def abs_A_u(d, n, u):
    """|A| |u|: (2d|u_p| + sum |u_q|) / h^2 on interior nodes."""
    h = 1.0 / (n - 1)
    au = np.abs(u)
    inn = (slice(1, -1),) * d
    out = 2 * d * au[inn]
    for axis in range(d):
        for s in (-1, 1):
            sl = [slice(1, -1)] * d
            sl[axis] = slice(1 + s, n - 1 + s)
            out = out + au[tuple(sl)]
    return out / (h * h)


def assert_u_close(ug, uo, bound=1e-11):
    """u parity at equal cycle counts: relative 2-norm AND element by element,
    max |u_gpu - u_oracle| <= bound * max |u_oracle|."""
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    assert rel <= bound, rel
    worst = np.max(np.abs(ug - uo))
    assert worst <= bound * np.max(np.abs(uo)), (worst, np.max(np.abs(uo)))


def relres_floor(d, n, u, f):
    fn = np.linalg.norm(f[(slice(1, -1),) * d])
    return 16 * EPS * np.linalg.norm(abs_A_u(d, n, u)) / (fn if fn > 0 else 1.0)


# ------------------------------------------------------------- single steps

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d,n", [(2, 257), (2, 1025), (3, 33), (3, 129)])
def test_step_restrict(B, torch_cuda, d, n, prec):
    torch = torch_cuda
    rng = np.random.default_rng(100 + n + d)
    k = O.check_side(n)
    s = B.Solver(d, n, precision=prec)
    for level in sorted({0, 1, k - 2}):
        nf = (n - 1) // (1 << level) + 1
        nc = (nf - 1) // 2 + 1
        say("restrict d=%d n=%d level=%d prec=%s" % (d, n, level, prec))
        rf = representable(torch, rand_interior(rng, d, nf), prec)
        out = torch.zeros((nc,) * d, dtype=torch.float64, device="cuda")
        s.step_restrict(level, dev(torch, rf), out)
        torch.cuda.synchronize()
        want = O.restrict(d, rf)
        got = host(out)
        inn = (slice(1, -1),) * d
        tol = np.broadcast_to(step_tol(prec, want), want.shape)
        assert np.all(np.abs(got[inn] - want[inn]) <= tol[inn])


@pytest.mark.parametrize("blocked", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d,n", [(2, 257), (2, 1025), (3, 33), (3, 65)])
def test_step_sweeps_every_level(B, torch_cuda, d, n, prec, blocked):
    torch = torch_cuda
    rng = np.random.default_rng(200 + n + d)
    k = O.check_side(n)
    s = B.Solver(d, n, precision=prec, temporal_block=blocked)
    omega = O.default_omega(d)
    for level in range(k):
        nm = (n - 1) // (1 << level) + 1
        for iters in (1, 3):
            say("sweeps d=%d n=%d level=%d iters=%d prec=%s blocked=%d" % (d, n, level, iters, prec, blocked))
            e0 = representable(torch, rand_interior(rng, d, n), prec)
            rm = representable(torch, rand_interior(rng, d, nm), prec)
            out = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
            s.step_sweeps(level, iters, dev(torch, e0), dev(torch, rm), out)
            torch.cuda.synchronize()
            want = e0
            for _ in range(iters):
                want = O.sweep(d, n, level, omega, rm, want)
                if prec != "fp64":
                    # the GPU stores every iterate in the working precision
                    want = representable(torch, want, prec)
            got = host(out)
            tol = step_tol(prec, want)
            if iters > 1 and prec == "fp32":
                tol = tol * 4
            if iters > 1 and prec == "bf16":
                # a one-ulp difference in an intermediate BF16 rounding propagates
                tol = 2.0 ** -7 * iters * np.max(np.abs(want))
            assert np.all(np.abs(got - want) <= tol), (level, iters, np.max(np.abs(got - want)))


def round_to(torch, x, prec):
    """FP64 values rounded as the library rounds to its storage type (to FP32,
    then for BF16 to BF16, round to nearest even)."""
    t = torch.from_numpy(np.ascontiguousarray(x)).to(torch.float32)
    if prec == "bf16":
        t = t.to(torch.bfloat16)
    return t.to(torch.float64).numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d,n", [(2, 65), (2, 257), (3, 17), (3, 33)])
def test_coarsest_level_is_fp64_in_reduced_precision(B, torch_cuda, d, n, prec):
    """In FP32/BF16 cycles the coarsest level computes in FP64: the
    restriction onto it is the FP64 oracle's restriction of the stored
    values (to FP64 rounding, not the storage type's), and its iterations
    match the FP64 oracle's, rounded once to the storage type at the end.
    (Iterating in the storage type would round after every iteration and
    miss the lattice values by an ulp or more on most draws.)"""
    torch = torch_cuda
    k = O.check_side(n)
    M = k - 1
    s = B.Solver(d, n, precision=prec)
    omega = O.default_omega(d)
    nf = (n - 1) // (1 << (M - 1)) + 1
    for seed in range(12):
        rng = np.random.default_rng(900 + 31 * n + seed)
        say("coarsest FP64 d=%d n=%d prec=%s seed=%d" % (d, n, prec, seed))
        # restriction M-1 -> M of values stored in the storage type
        rf = representable(torch, rand_interior(rng, d, nf), prec)
        out = torch.zeros((3,) * d, dtype=torch.float64, device="cuda")
        s.step_restrict(M - 1, dev(torch, rf), out)
        want = O.restrict(d, rf)
        assert np.max(np.abs(host(out) - want)) <= 1e-14 * np.max(np.abs(want))
        # iterations at level M from a stored e and an FP64 right-hand side
        e0 = representable(torch, rand_interior(rng, d, n), prec)
        rm = rand_interior(rng, d, 3)
        for iters in (1, 2, 3):
            got = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
            s.step_sweeps(M, iters, dev(torch, e0), dev(torch, rm), got)
            x = e0
            for _ in range(iters):
                x = O.sweep(d, n, M, omega, rm, x)
            c = (n // 2,) * d
            g = host(got)
            assert g[c] == round_to(torch, x[c], prec), (iters, g[c], x[c])


@pytest.mark.parametrize("d,n,max_i", [(2, 129, 4), (2, 513, 2), (2, 257, 32), (3, 33, 4), (3, 65, 8)])
def test_step_cycle_fp64(B, torch_cuda, d, n, max_i):
    torch = torch_cuda
    say("cycle d=%d n=%d max_i=%d" % (d, n, max_i))
    rng = np.random.default_rng(300 + n)
    r0 = rand_interior(rng, d, n)
    s = B.Solver(d, n, max_i=max_i)
    acc = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    s.step_cycle(dev(torch, r0), acc)
    torch.cuda.synchronize()
    k = O.check_side(n)
    want = O.mfmg_cycle(d, n, r0, O.default_schedule(k, max_i), O.default_omega(d))
    got = host(acc)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d,n,max_i,var", [(2, 1025, 4, False), (2, 257, 32, False), (2, 129, 4, True),
                                           (3, 129, 4, False), (3, 65, 8, False)])
def test_level_blocked_path_is_bitwise_identical(B, torch_cuda, d, n, max_i, var, prec):
    """The level-blocked path (compact-lattice iterations, one whole-grid pass
    per level), the chained path (the whole grid written only before level 0)
    and the one-launch-per-iteration path give the same bits."""
    torch = torch_cuda
    if var and prec != "fp64":
        pytest.skip("variable coefficient covered in FP64")
    say("blocked vs per-iteration d=%d n=%d max_i=%d var=%s prec=%s" % (d, n, max_i, var, prec))
    f = dev(torch, W.uniform(d, n, seed=17))
    a = None
    if var:
        a_np, _ = W.grf_problem(n, seed=17)
        a = dev(torch, a_np)
    outs = []
    for blocked in (0, 1, 2):
        s = B.Solver(d, n, max_i=max_i, precision=prec, temporal_block=blocked,
                     stencil=B.DIFFUSION_5PT_2D if var else None)
        if var:
            s.set_coefficient(a)
        u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
        s.solve_cycles(f, u, 3)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def test_schedule_matches_oracle(B, torch_cuda):
    for d, n, max_i in ((2, 129, 4), (2, 4097, 4), (3, 257, 32), (2, 1025, 2)):
        k = O.check_side(n)
        if d == 3 and n > 257:
            continue
        s = B.Solver(d, n, max_i=max_i)
        assert s.schedule() == O.default_schedule(k, max_i)


# ------------------------------------------------------------- whole solves

def solve_and_compare(B, torch, d, n, f, *, a=None, max_i=4, tol=1e-10, schedule=None, levels=0,
                      stencil=None):
    say("solve d=%d n=%d max_i=%d levels=%d var=%s" % (d, n, max_i, levels, a is not None))
    s = B.Solver(d, n, max_i=max_i, schedule=schedule, levels=levels, stencil=stencil)
    if a is not None:
        s.set_coefficient(dev(torch, a))
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=tol)
    torch.cuda.synchronize()
    ug = host(u)
    lv = levels if levels else None
    uo, ho = O.solve(d, n, f, a=a, max_i=max_i, fixed_cycles=res["cycles"], schedule=schedule, levels=lv)
    # u parity at the same cycle count
    assert_u_close(ug, uo)
    # residual history
    floor = relres_floor(d, n, uo, f)
    hg = np.array(res["history"])
    assert len(hg) == len(ho)
    assert np.all(np.abs(hg - np.array(ho)) <= 1e-6 * np.array(ho) + floor), (hg, ho, floor)
    # final residual recomputed by the oracle from the GPU's u
    _, s2 = O.residual(d, n, f, ug, a)
    fn = np.sqrt(O.norm2_interior(d, n, f))
    assert np.sqrt(s2) / fn <= tol * (1 + 1e-6) + floor
    assert res["converged"]
    return ug, res


def test_sine_problem_129_fp64(B, torch_cuda):
    """2D -Lap u = 2 pi^2 sin sin on 129^2, omega 4/5, down to the 3x3 lattice."""
    torch = torch_cuda
    n = 129
    f = W.sine2d(n)
    ug, res = solve_and_compare(B, torch, 2, n, f)
    from oracle import textbook as T
    lam = T.laplace_eigenvalue(2, n, (1, 1))
    uh = (2 * np.pi ** 2 / lam) * W.sine2d_exact(n)
    assert np.linalg.norm(ug - uh) / np.linalg.norm(uh) <= 1e-9
    assert res["final_relres"] <= 1e-10


@pytest.mark.parametrize("d,n,seed,max_i", [(2, 257, 1, 4), (2, 1025, 2, 4), (2, 513, 3, 32),
                                            (3, 33, 4, 4), (3, 65, 5, 4), (3, 129, 6, 8)])
def test_uniform_solves_fp64(B, torch_cuda, d, n, seed, max_i):
    solve_and_compare(B, torch_cuda, d, n, W.uniform(d, n, seed=seed), max_i=max_i)


def test_normal_source_and_partial_levels(B, torch_cuda):
    f = W.normal(3, 65, seed=7)
    solve_and_compare(B, torch_cuda, 3, 65, f, levels=4)


def test_explicit_zigzag_schedule(B, torch_cuda):
    n = 129
    sched = [(6, 2), (5, 2), (6, 1), (5, 2), (4, 2), (3, 2), (4, 1), (3, 2), (2, 2), (1, 2), (0, 2)]
    solve_and_compare(B, torch_cuda, 2, n, W.uniform(2, n, seed=8), schedule=sched)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_chained_path_with_revisits_and_coarse_end(B, torch_cuda, prec):
    """Chained transfers to coarser, finer and repeated levels, and a schedule
    that ends on a coarse level, give the bits of the whole-grid path."""
    torch = torch_cuda
    n = 129
    f = dev(torch, W.uniform(2, n, seed=18))
    sched = [(6, 2), (5, 1), (6, 1), (6, 2), (4, 3), (2, 1), (3, 2), (1, 2), (0, 1), (2, 2)]
    outs = []
    for blocked in (1, 2):
        s = B.Solver(2, n, schedule=sched, precision=prec, temporal_block=blocked)
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        s.solve_cycles(f, u, 2)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,sched", [
    (5, [(1, 2), (0, 1)]),
    (9, [(0, 3), (2, 1), (1, 2), (0, 5)]),
    (17, [(0, 4), (3, 2), (0, 2)]),
    (65, [(5, 2), (0, 2), (3, 2), (0, 9)]),
    (2049, [(9, 2), (4, 1), (0, 7)]),
    (1025, None),
    (9, [(1, 1), (0, 3)]),
    (257, [(1, 3), (0, 4), (2, 2), (1, 2), (0, 6)]),
    (1025, [(2, 1), (1, 3), (0, 2)]),
    (1025, [(3, 2), (2, 1), (1, 1), (0, 1), (2, 5), (1, 6), (0, 4)]),
    (1025, [(3, 2), (2, 3), (1, 2), (0, 1), (2, 1)]),
])
def test_level0_multi_iteration_pass_is_bitwise_identical(B, torch_cuda, n, sched, prec):
    """2D level 0 with several iterations per pass (level-blocked and chained
    paths) against one launch per iteration: level 0 first (from e = 0), in
    the middle (stored) and last (added into u), 1 to 9 iterations, grids
    narrower than one wave and row counts that are not multiples of the
    band; after level 1 (the chained path's first pass interpolates level
    1's lattice itself), also level 1 from e = 0 with a single iteration,
    and chains of adjacent compact lattices (each first pass interpolating
    the coarser lattice, from e = 0, with one and several iterations)."""
    torch = torch_cuda
    say("level-0 pass n=%d sched=%s prec=%s" % (n, sched, prec))
    f = dev(torch, W.uniform(2, n, seed=19))
    outs = []
    for blocked in (0, 1, 2):
        s = B.Solver(2, n, schedule=sched, precision=prec, temporal_block=blocked)
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        s.solve_cycles(f, u, 2)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,sched", [
    (5, [(1, 2), (0, 1)]),
    (9, [(0, 3), (2, 1), (1, 2), (0, 5)]),
    (33, [(4, 2), (0, 2), (3, 3), (1, 5), (0, 4)]),
    (65, [(5, 2), (2, 3), (1, 1), (0, 9)]),
    (129, None),
    (17, [(1, 1), (0, 1)]),
    (9, [(1, 3), (0, 3), (1, 2), (0, 2)]),
    (129, [(2, 1), (1, 3), (0, 2)]),
    (129, [(3, 2), (2, 1), (1, 1), (0, 3), (2, 3), (1, 2), (0, 1)]),
    (65, [(4, 2), (3, 2), (2, 2), (1, 1)]),
])
def test_3d_multi_iteration_pass_is_bitwise_identical(B, torch_cuda, n, sched, prec):
    """3D level 0 and the compact lattices with two iterations per pass
    (level-blocked and chained paths) against one launch per iteration:
    level 0 first, in the middle and last, odd and even iteration counts,
    grids smaller than one tile, and level 0 right after level 1 (one and
    two iterations in the pass that interpolates level 1's lattice, level
    1 from e = 0), and chains of adjacent compact lattices."""
    torch = torch_cuda
    say("3D pass n=%d sched=%s prec=%s" % (n, sched, prec))
    f = dev(torch, W.uniform(3, n, seed=20))
    outs = []
    for blocked in (0, 1, 2):
        s = B.Solver(3, n, schedule=sched, precision=prec, temporal_block=blocked)
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        s.solve_cycles(f, u, 2)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("n", [129, 257])
def test_variable_coefficient_fp64(B, torch_cuda, n):
    a, f = W.grf_problem(n, seed=9)
    solve_and_compare(B, torch_cuda, 2, n, f, a=a, stencil=B.DIFFUSION_5PT_2D)


def test_golden_histories(B, torch_cuda):
    torch = torch_cuda
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_histories.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        say("golden " + c["name"])
        d, n = c["d"], c["n"]
        f = W.sine2d(n) if c["input"] == "sine2d" else W.uniform(d, n, seed=c["seed"])
        s = B.Solver(d, n, max_i=c["max_i"])
        u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
        res = s.solve(dev(torch, f), u, tol=c["tol"])
        ho = np.array(c["history"])
        assert res["cycles"] == len(ho) - 1
        np.testing.assert_allclose(res["history"], ho, rtol=1e-5, atol=1e-12)


def test_tiny_grids(B, torch_cuda):
    torch = torch_cuda
    for d, n in ((2, 3), (2, 5), (3, 3), (3, 5)):
        say("tiny d=%d n=%d" % (d, n))
        f = W.uniform(d, n, seed=10)
        solve_and_compare(B, torch, d, n, f, tol=1e-12)


def test_nonzero_initial_guess_and_boundary_data(B, torch_cuda):
    """u0 carries Dirichlet data on the boundary and a guess inside; the
    boundary is never written."""
    torch = torch_cuda
    d, n = 2, 129
    rng = np.random.default_rng(11)
    f = W.uniform(d, n, seed=11)
    u0 = rng.standard_normal((n, n))
    s = B.Solver(d, n)
    u = dev(torch, u0)
    res = s.solve(dev(torch, f), u, tol=1e-10)
    ug = host(u)
    assert np.array_equal(ug[0], u0[0]) and np.array_equal(ug[-1], u0[-1])
    assert np.array_equal(ug[:, 0], u0[:, 0]) and np.array_equal(ug[:, -1], u0[:, -1])
    uo, ho = O.solve(d, n, f, u0=u0, fixed_cycles=res["cycles"])
    assert_u_close(ug, uo)


def test_repeat_solves_bitwise_identical(B, torch_cuda):
    torch = torch_cuda
    for d, n in ((2, 1025), (3, 65)):
        f = dev(torch, W.uniform(d, n, seed=12))
        s = B.Solver(d, n)
        outs = []
        for _ in range(2):
            u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
            s.solve(f, u, tol=1e-10)
            outs.append(host(u))
        assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d,n", [(2, 5), (2, 9), (2, 65), (2, 129), (2, 1025),
                                 (3, 5), (3, 9), (3, 17), (3, 33), (3, 65), (3, 129)])
def test_solve_cycle_equals_residual_then_step_cycle(B, torch_cuda, d, n, prec):
    """A solve's residual pass also restricts r_0 to level 1 (2D Laplacian;
    3D keeps separate residual and restriction launches); one solve cycle
    must equal the residual entry point followed by the step cycle, which
    restricts with the separate kernel: bit for bit, from a non-zero initial
    guess, for tile, band and wave counts with ragged ends."""
    torch = torch_cuda
    say("fused residual d=%d n=%d prec=%s" % (d, n, prec))
    rng = np.random.default_rng(500 + n)
    f = dev(torch, W.uniform(d, n, seed=21))
    u0 = dev(torch, rand_interior(rng, d, n))
    s = B.Solver(d, n, precision=prec)
    ua = u0.clone()
    s.solve_cycles(f, ua, 1)
    r0 = torch.zeros_like(u0)
    s.residual(f, u0, r0)
    ub = u0.clone()
    s.step_cycle(r0, ub)
    torch.cuda.synchronize()
    assert np.array_equal(host(ua), host(ub))


def test_residual_entry_point(B, torch_cuda):
    torch = torch_cuda
    for d, n in ((2, 257), (3, 33)):
        rng = np.random.default_rng(13)
        f = W.uniform(d, n, seed=13)
        u = rand_interior(rng, d, n)
        s = B.Solver(d, n)
        r = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
        rel = s.residual(dev(torch, f), dev(torch, u), r)
        ro, so = O.residual(d, n, f, u)
        fn = np.sqrt(O.norm2_interior(d, n, f))
        assert rel == pytest.approx(np.sqrt(so) / fn, rel=1e-12)
        assert np.max(np.abs(host(r) - ro)) <= 1e-12 * np.max(np.abs(ro))
        rel2 = s.residual(dev(torch, f), dev(torch, u))
        assert rel2 == pytest.approx(rel, rel=1e-12)


# ------------------------------------------------------------- error paths

def test_not_converged_leaves_last_iterate(B, torch_cuda):
    torch = torch_cuda
    n = 65
    f = W.uniform(2, n, seed=14)
    s = B.Solver(2, n, max_cycles=3)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=1e-300, raise_on_status=False)
    assert res["status"] == 7 and res["cycles"] == 3 and not res["converged"]
    uo, _ = O.solve(2, n, f, fixed_cycles=3)
    assert_u_close(host(u), uo)


def test_non_finite_source_is_reported(B, torch_cuda):
    torch = torch_cuda
    n = 65
    f = W.uniform(2, n, seed=15)
    f[10, 10] = np.nan
    s = B.Solver(2, n)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=1e-10, raise_on_status=False)
    assert res["status"] == 6


def test_diffusion_needs_coefficient(B, torch_cuda):
    torch = torch_cuda
    s = B.Solver(2, 33, stencil=B.DIFFUSION_5PT_2D)
    u = torch.zeros((33, 33), dtype=torch.float64, device="cuda")
    with pytest.raises(B.HomgError):
        s.solve(dev(torch, W.uniform(2, 33)), u)


# ------------------------------------------------------------- mixed precision

def lambda_min(d, n):
    """Smallest eigenvalue of the discrete -Laplacian on side n (closed form)."""
    h = 1.0 / (n - 1)
    return (4 * d / h ** 2) * np.sin(np.pi * h / 2) ** 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d,n", [(2, 257), (3, 65), (3, 257)])
def test_mixed_precision_refinement(B, torch_cuda, d, n, prec):
    """FP32 / BF16 sweeps under FP64 residual and update: the final FP64
    relative residual (recomputed by the oracle) reaches the tolerance and u
    lies within the rigorous bound of the FP64 oracle's u."""
    torch = torch_cuda
    say("mixed d=%d n=%d prec=%s" % (d, n, prec))
    f = W.normal(d, n, seed=16)
    s = B.Solver(d, n, precision=prec, max_cycles=200)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=1e-10, raise_on_status=False)
    ug = host(u)
    say("  status %d cycles %d final %.3e" % (res["status"], res["cycles"], res["final_relres"]))
    assert res["status"] == 0
    _, s2 = O.residual(d, n, f, ug)
    fn = np.sqrt(O.norm2_interior(d, n, f))
    assert np.sqrt(s2) / fn <= 1e-10 * (1 + 1e-6) + relres_floor(d, n, ug, f)
    uo, ho = O.solve(d, n, f, tol=1e-10)
    _, so = O.residual(d, n, f, uo)
    bound = (np.sqrt(s2) + np.sqrt(so)) / lambda_min(d, n)
    diff = np.linalg.norm(ug - uo)
    say("  |u - u_oracle| / |u_oracle| = %.3e (bound %.3e)" % (diff / np.linalg.norm(uo),
                                                              bound / np.linalg.norm(uo)))
    assert diff <= bound * (1 + 1e-6)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [257, 513])
def test_3d_reduced_precision_large_bands_bitwise(B, torch_cuda, prec, n):
    """3D in FP32 / BF16 at full sizes: level 0 walks 16-plane bands at 257^3
    (1760 blocks) and 32-plane bands at 513^3, the 257^3 lattice of the
    513^3 grid 16-plane bands, and the large compact lattices run
    multi-iteration passes.  One cycle must give the same bits with one
    launch per iteration, level blocking and chaining."""
    torch = torch_cuda
    f = dev(torch, W.uniform(3, n, seed=22))
    outs = []
    for blocked in (0, 1, 2):
        say("3D %d^3 %s temporal_block=%d" % (n, prec, blocked))
        s = B.Solver(3, n, precision=prec, temporal_block=blocked)
        u = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        s.solve_cycles(f, u, 1)
        outs.append(host(u))
        del s, u
        torch.cuda.empty_cache()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_513_cube(B, torch_cuda, prec):
    """The 3D 513^3 N(0,1) reduced-precision workload: the final FP64
    relative residual, recomputed by the oracle from the GPU's u, meets
    1e-10, and u lies within ||f - A u|| / lambda_min of the exact discrete
    solution (a rigorous bound, since A is SPD)."""
    torch = torch_cuda
    d, n = 3, 513
    say("mixed 513^3 %s: input" % prec)
    f = W.normal(d, n, seed=0)
    s = B.Solver(d, n, precision=prec)
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    say("mixed 513^3 %s: solve" % prec)
    res = s.solve(dev(torch, f), u, tol=1e-10)
    ug = host(u)
    del u
    say("mixed 513^3 %s: oracle residual (cycles %d)" % (prec, res["cycles"]))
    _, s2 = O.residual(d, n, f, ug)
    fn = np.sqrt(O.norm2_interior(d, n, f))
    assert np.sqrt(s2) / fn <= 1e-10 * (1 + 1e-6) + relres_floor(d, n, ug, f)
    bound = np.sqrt(s2) / lambda_min(d, n)
    say("  relres %.3e; |u - u*| / |u| <= %.3e" % (np.sqrt(s2) / fn, bound / np.linalg.norm(ug)))
    # white noise puts most of |f| in high modes and most of |u| in low ones:
    # |f| ~ 1.2e4, |u| ~ 0.14, so the bound is ~3e-7 relative at relres 1e-10
    assert bound <= 1e-5 * np.linalg.norm(ug)


# ------------------------------------------------------------- full sizes

@pytest.mark.parametrize("d,n", [(2, 4097), (3, 257)])
def test_full_size_fp64(B, torch_cuda, d, n):
    """The bench workloads at full size: one whole cycle element by element
    against the oracle, then the full solve with its final residual
    recomputed by the oracle."""
    torch = torch_cuda
    f = W.uniform(d, n, seed=0)
    fd = dev(torch, f)
    s = B.Solver(d, n)
    say("full size d=%d n=%d: one cycle" % (d, n))
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    res1 = s.solve_cycles(fd, u, 1)
    ug = host(u)
    uo, ho = O.solve(d, n, f, fixed_cycles=1)
    assert_u_close(ug, uo)
    assert abs(res1["history"][1] - ho[1]) <= 1e-6 * ho[1] + relres_floor(d, n, uo, f)
    say("full size d=%d n=%d: solve to 1e-10" % (d, n))
    u.zero_()
    res = s.solve(fd, u, tol=1e-10)
    ug = host(u)
    _, s2 = O.residual(d, n, f, ug)
    fn = np.sqrt(O.norm2_interior(d, n, f))
    assert np.sqrt(s2) / fn <= 1e-10 * (1 + 1e-6) + relres_floor(d, n, ug, f)
    say("  cycles %d final %.3e" % (res["cycles"], res["final_relres"]))


@pytest.mark.parametrize("d,n", [(2, 32769), (3, 1025)])
def test_maximum_sizes_eigenfunction(B, torch_cuda, d, n):
    """The largest grids the library accepts (8.6 GB per FP64 array, byte
    offsets far past 2^31): with f the discrete (1, 1, ...) eigenfunction
    times its eigenvalue, the discrete solution is that eigenfunction, and
    since it is the smallest eigenvalue's mode the relative error of u is at
    most the relative residual.  A property of the mathematics, not of the
    oracle (too slow at this size).  At these sizes 1e-10 lies below the
    FP64 rounding floor of the residual itself (16 eps || |A| |u| || / ||f||,
    about 1.4e-15 / h^2 for this mode: 1.5e-6 at 32769^2, 1.5e-9 at
    1025^3), so the solve runs to 20 times that floor, and the error bound
    carries the floor of the final residual too."""
    torch = torch_cuda
    say("maximum size d=%d n=%d" % (d, n))
    h = 1.0 / (n - 1)
    x = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device="cuda")
    sx = torch.sin(np.pi * x)
    sx[0] = 0.0
    sx[-1] = 0.0
    ue = sx[:, None] * sx[None, :] if d == 2 else sx[:, None, None] * sx[None, :, None] * sx[None, None, :]
    lam = d * (4.0 / h ** 2) * np.sin(np.pi * h / 2) ** 2
    f = ue * lam
    # |A| |u*| on the interior, for the rounding floor of the residual
    inn = (slice(1, -1),) * d
    aau = 2 * d * ue[inn].abs()
    for axis in range(d):
        for sh in (-1, 1):
            sl = [slice(1, -1)] * d
            sl[axis] = slice(1 + sh, n - 1 + sh)
            aau = aau + ue[tuple(sl)].abs()
    floor = 16 * EPS * float(torch.linalg.vector_norm(aau)) / (h * h) / float(torch.linalg.vector_norm(f[inn]))
    del aau
    tol = max(1e-10, 20 * floor)
    u = torch.zeros_like(f)
    s = B.Solver(d, n)
    res = s.solve(f, u, tol=tol)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(u - ue) / torch.linalg.vector_norm(ue))
    worst = float(torch.max(torch.abs(u - ue)))
    say("  floor %.2e tol %.2e cycles %d final relres %.3e rel err %.3e max err %.3e"
        % (floor, tol, res["cycles"], res["final_relres"], err, worst))
    assert res["converged"] and res["final_relres"] <= tol
    assert err <= (res["final_relres"] + 2 * floor) * (1 + 1e-6)
    # element by element: |e_i| <= ||e||_2 <= relres ||u*||_2
    assert worst <= (res["final_relres"] + 2 * floor) * float(torch.linalg.vector_norm(ue)) * (1 + 1e-6)
    s.close()
    del f, u, ue
    torch.cuda.empty_cache()
