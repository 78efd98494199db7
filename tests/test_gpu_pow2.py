"""GPU parity of the power-of-two grid strategy (Sec. 3) against its oracle
(oracle/pow2.py): whole cycles element by element, every iteration of a
cycle, whole solves at equal cycle counts, revisiting schedules, the three
execution forms bit for bit, and the full 4096^2 grid.  Tolerances as for
the nested grids (FP64: ~1e-16 per node formula, so 1e-12 of the largest
value for one cycle and 1e-11 relative in u for whole solves)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import homg as O
from oracle import pow2 as P2
from oracle import textbook as T

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


def uniform(N, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((N, N))
    f[1:-1, 1:-1] = rng.uniform(-1, 1, (N - 2, N - 2))
    return f


def close(got, want, bound):
    worst = np.max(np.abs(got - want))
    assert worst <= bound * np.max(np.abs(want)), (worst, np.max(np.abs(want)))


@pytest.mark.parametrize("N,max_i", [(4, 4), (8, 2), (64, 4), (128, 2), (256, 32)])
def test_one_cycle_matches_oracle(B, torch_cuda, N, max_i):
    torch = torch_cuda
    say("pow2 one cycle N=%d MaxI=%d" % (N, max_i))
    f = uniform(N, 40 + N)
    s = B.Solver(2, N, max_i=max_i, grid_layout="pow2")
    u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    s.solve_cycles(dev(torch, f), u, 1)
    uo, _ = P2.solve(N, f, max_i=max_i, fixed_cycles=1)
    close(u.cpu().numpy(), uo, 1e-12)


def test_every_iteration_matches_oracle(B, torch_cuda):
    """Each whole-grid state of one cycle (schedule prefixes), 128^2, MaxI 2,
    the polynomial source of Sec. 4 on the paper's 128^2 grid."""
    torch = torch_cuda
    N = 128
    f, _ = W.poly2d(N)
    k = P2.check_side(N)
    sched = P2.default_schedule(k, 2)
    r0, _ = O.residual(2, N, f, np.zeros_like(f))
    _, states = P2.mfmg_cycle(N, r0, sched, 0.8, keep_states=True)
    fd = dev(torch, f)
    flat = [m for m, it in sched for _ in range(it)]
    for upto in range(1, len(flat) + 1):
        prefix = []
        for m in flat[:upto]:
            if prefix and prefix[-1][0] == m:
                prefix[-1] = (m, prefix[-1][1] + 1)
            else:
                prefix.append((m, 1))
        s = B.Solver(2, N, levels=k, schedule=prefix, grid_layout="pow2")
        u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
        s.solve_cycles(fd, u, 1)
        close(u.cpu().numpy(), states[upto - 1], 1e-12)
        s.close()


@pytest.mark.parametrize("N,seed,max_i", [(16, 1, 4), (128, 2, 4), (512, 3, 8), (1024, 4, 4)])
def test_solve_matches_oracle(B, torch_cuda, N, seed, max_i):
    torch = torch_cuda
    say("pow2 solve N=%d" % N)
    f = uniform(N, seed)
    s = B.Solver(2, N, max_i=max_i, grid_layout="pow2")
    u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=1e-10)
    ug = u.cpu().numpy()
    uo, ho = P2.solve(N, f, max_i=max_i, fixed_cycles=res["cycles"])
    assert np.linalg.norm(ug - uo) <= 1e-11 * np.linalg.norm(uo)
    close(ug, uo, 1e-11)
    np.testing.assert_allclose(res["history"], ho, rtol=1e-6, atol=1e-14)
    _, s2 = O.residual(2, N, f, ug)
    assert np.sqrt(s2 / O.norm2_interior(2, N, f)) <= 1e-10 * (1 + 1e-6)
    if N <= 32:
        us = T.dense_solve(2, N, f)
        assert np.linalg.norm(ug - us) <= 1e-8 * np.linalg.norm(us)


def test_revisiting_schedule_and_execution_forms(B, torch_cuda):
    """A schedule that goes back to coarser levels matches the oracle, and
    the three execution forms give the same bits."""
    torch = torch_cuda
    N = 256
    f = uniform(N, 9)
    sched = [(7, 2), (6, 2), (7, 1), (6, 2), (5, 3), (4, 2), (5, 1), (3, 2), (2, 2), (1, 2), (0, 5), (1, 1), (0, 2)]
    outs = []
    for tb in (0, 1, 2):
        s = B.Solver(2, N, schedule=sched, temporal_block=tb, grid_layout="pow2")
        u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
        s.solve_cycles(dev(torch, f), u, 2)
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    uo, _ = P2.solve(N, f, schedule=sched, fixed_cycles=2)
    close(outs[0], uo, 1e-11)


def test_trace_and_l1_on_paper_grid(B, torch_cuda):
    """The Sec. 4 polynomial problem on the 128^2 power-of-two grid: the
    per-iteration L1 trace equals the oracle's."""
    torch = torch_cuda
    N = 128
    f, uex = W.poly2d(N)
    k = P2.check_side(N)
    for max_i in (2, 4, 32):
        s = B.Solver(2, N, max_i=max_i, temporal_block=0, grid_layout="pow2")
        u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
        errs = s.trace_cycle(dev(torch, f), u, dev(torch, uex))
        r0, _ = O.residual(2, N, f, np.zeros_like(f))
        _, states = P2.mfmg_cycle(N, r0, P2.default_schedule(k, max_i), 0.8, keep_states=True)
        want = [np.sum(np.abs(uex - e)) / np.sum(np.abs(uex)) for e in states]
        np.testing.assert_allclose(errs, want, rtol=1e-10)


def test_full_size_4096(B, torch_cuda):
    torch = torch_cuda
    N = 4096
    f = W.uniform(2, N, seed=0)
    fd = dev(torch, f)
    s = B.Solver(2, N, grid_layout="pow2")
    u = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    say("pow2 4096^2: one cycle")
    s.solve_cycles(fd, u, 1)
    uo, _ = P2.solve(N, f, fixed_cycles=1)
    close(u.cpu().numpy(), uo, 1e-11)
    say("pow2 4096^2: solve to 1e-10")
    u.zero_()
    res = s.solve(fd, u, tol=1e-10)
    _, s2 = O.residual(2, N, f, u.cpu().numpy())
    assert np.sqrt(s2 / O.norm2_interior(2, N, f)) <= 1e-10 * (1 + 1e-6)
    say("  cycles %d" % res["cycles"])


def test_nested_only_entry_points_refuse(B, torch_cuda):
    torch = torch_cuda
    s = B.Solver(2, 64, grid_layout="pow2")
    z = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(B.HomgError) as ei:
        s.step_sweeps(1, 1, z, torch.zeros((33, 33), dtype=torch.float64, device="cuda"), z)
    assert ei.value.status == 2
