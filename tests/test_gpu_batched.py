"""GPU tests of the batched solver (many problems advanced together, one launch per step).

Every problem of a batch must end exactly where the one-problem solver
(one launch per iteration, same precision) ends: the batched kernel runs the
same tile code with the same tiles, so u agrees bit for bit and the cycle
counts match (the residual norms to the rounding of their summation order).
The FP64 batch is also checked against the CPU oracle.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import homg as O

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_problem_solves(B, torch_cuda, prec):
    torch = torch_cuda
    sides = [65, 9, 129, 17, 33, 257, 65, 3, 5, 129, 33, 513]
    say("batch %s sides %s" % (prec, sides))
    fs = [dev(torch, W.uniform(2, s, seed=100 + i)) for i, s in enumerate(sides)]
    us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
    bs = B.BatchSolver(sides, precision=prec)
    res = bs.solve(fs, us, tol=1e-10)
    assert res["status"] == 0 and all(st == 0 for st in res["statuses"])
    for i, s in enumerate(sides):
        one = B.Solver(2, s, precision=prec, temporal_block=0)
        u1 = torch.zeros((s, s), dtype=torch.float64, device="cuda")
        r1 = one.solve(fs[i], u1, tol=1e-10)
        assert r1["cycles"] == res["cycles"][i], (s, r1["cycles"], res["cycles"][i])
        assert torch.equal(u1, us[i]), s
        # the single-problem solver sums the residual norm over other
        # partials (its residual is fused with the first restriction), so
        # the norms agree to the rounding of the summation order
        assert res["relres"][i] == pytest.approx(r1["final_relres"], rel=1e-14, abs=0)
    if prec == "fp64":
        for i in (0, 2, 5):
            s = sides[i]
            uo, ho = O.solve(2, s, fs[i].cpu().numpy(), fixed_cycles=res["cycles"][i])
            ug = us[i].cpu().numpy()
            assert np.linalg.norm(ug - uo) / np.linalg.norm(uo) <= 1e-11


def test_batch_repeat_and_tile_rows(B, torch_cuda):
    """Replaying the captured launch gives the same result; other tile
    shapes change only the order of the norm sums."""
    torch = torch_cuda
    sides = [129, 257, 65, 1025]
    fs = [dev(torch, W.uniform(2, s, seed=200 + i)) for i, s in enumerate(sides)]
    bs = B.BatchSolver(sides, precision="fp32")
    outs = []
    for rep in range(2):
        us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
        res = bs.solve(fs, us, tol=1e-10)
        outs.append((res, [u.clone() for u in us]))
    assert outs[0][0]["cycles"] == outs[1][0]["cycles"]
    assert all(torch.equal(a, b) for a, b in zip(outs[0][1], outs[1][1]))
    for s in set(sides):
        bs.set_tile_rows(s, 8)
    us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
    res = bs.solve(fs, us, tol=1e-10)
    for i, s in enumerate(sides):
        one = B.Solver(2, s)
        rel = one.residual(fs[i], us[i])
        assert rel <= 1e-10 * (1 + 1e-6)


def test_batch_uneven_workload_sample(B, torch_cuda, tmp_path):
    """A 96-problem draw of the uneven-size workload (sides from
    {65, ..., 1025}), FP32 sweeps with FP64 refinement, tuned tiles: every
    problem reaches 1e-10, checked with the FP64 residual entry point and, for
    the smallest problems, by the oracle."""
    torch = torch_cuda
    sides, fnp = W.batch2d(count=96, seed=1)
    fs = [dev(torch, f) for f in fnp]
    us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
    bs = B.BatchSolver(sides, precision="fp32")
    say("tuning")
    bs.tune(fs, us, tol=1e-10, cache_path=str(tmp_path / "tiles.txt"))
    for u in us:
        u.zero_()
    say("solving")
    res = bs.solve(fs, us, tol=1e-10)
    assert res["status"] == 0
    checked = 0
    for i, s in enumerate(sides):
        rel = B.Solver(2, s).residual(fs[i], us[i])
        assert rel <= 1e-10 * (1 + 1e-6), (i, s, rel)
        if s == 65 and checked < 3:
            _, so = O.residual(2, s, fnp[i], us[i].cpu().numpy())
            assert np.sqrt(so) / np.sqrt(O.norm2_interior(2, s, fnp[i])) <= 1e-10 * (1 + 1e-6)
            checked += 1
    # the cache round-trips
    bs2 = B.BatchSolver(sides, precision="fp32")
    bs2.tune(fs, us, tol=1e-10, cache_path=str(tmp_path / "tiles.txt"))


def test_batch_reports_unconverged_problems(B, torch_cuda):
    torch = torch_cuda
    sides = [33, 65]
    fs = [dev(torch, W.uniform(2, s, seed=300 + i)) for i, s in enumerate(sides)]
    us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
    bs = B.BatchSolver(sides, precision="fp64", max_cycles=2)
    res = bs.solve(fs, us, tol=1e-12, raise_on_status=False)
    assert res["status"] == 7 and res["statuses"] == [7, 7] and res["cycles"] == [2, 2]


def test_batch_pass_iterations_are_bitwise_identical(B, torch_cuda):
    """Level-0 passes of 1, 2, 3 or 4 iterations give the same iterates bit
    for bit (only the number of steps changes)."""
    torch = torch_cuda
    sides = [129, 65, 257, 17]
    fs = [dev(torch, W.uniform(2, s, seed=400 + i)) for i, s in enumerate(sides)]
    outs = []
    for its in (4, 1, 2, 3):
        say("batch pass iterations %d" % its)
        bs = B.BatchSolver(sides, precision="fp32")
        for s in set(sides):
            bs.set_pass_iters(s, its)
        us = [torch.zeros((s, s), dtype=torch.float64, device="cuda") for s in sides]
        res = bs.solve(fs, us, tol=1e-10)
        outs.append((res["cycles"], [u.clone() for u in us]))
    for cyc, us in outs[1:]:
        assert cyc == outs[0][0]
        assert all(torch.equal(a, b) for a, b in zip(us, outs[0][1]))


def test_batch_tuner_times_real_solves_and_restores_u(B, torch_cuda, tmp_path):
    """Every timed candidate starts from the caller's initial guess (a
    non-zero one here), which the tuner leaves in place; a tuning run whose
    guesses already meet tol is refused, since it would time no cycle."""
    torch = torch_cuda
    sides = [65, 129, 33]
    rng = np.random.default_rng(5)
    fs = [dev(torch, W.uniform(2, s, seed=500 + i)) for i, s in enumerate(sides)]
    u0 = []
    for s in sides:
        g = np.zeros((s, s))
        g[1:-1, 1:-1] = rng.standard_normal((s - 2, s - 2))
        u0.append(dev(torch, g))
    us = [u.clone() for u in u0]
    bs = B.BatchSolver(sides, precision="fp32")
    say("tuner from a non-zero guess")
    bs.tune(fs, us, tol=1e-10, cache_path=str(tmp_path / "t.txt"))
    assert all(torch.equal(a, b) for a, b in zip(us, u0))
    lines = open(tmp_path / "t.txt").read().split("\n")
    assert sum(1 for ln in lines if ln.strip()) == len(set(sides))
    for ln in lines:
        if ln.strip():
            key, side, rows, its = ln.split()
            assert int(side) in sides and int(rows) >= 1 and 1 <= int(its) <= 4
    res = bs.solve(fs, us, tol=1e-10)
    assert res["status"] == 0 and min(res["cycles"]) >= 1
    say("tuner on converged guesses")
    with pytest.raises(B.HomgError) as ei:
        B.BatchSolver(sides, precision="fp32").tune(fs, us, tol=1e-3)
    assert ei.value.status == 1
