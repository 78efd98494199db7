"""The in-cycle restriction of Sec. 2 (one extra array instead of the
restriction pyramid): same bits as the pyramid on every execution form and
precision, with schedules that revisit levels, end on a coarse level, skip
levels and run the one-workgroup coarse tail; and less device memory.  The
in-cycle form runs one restriction per launch, so the bitwise comparison
also pins the pyramid's multi-level restriction launch (its coarse end,
several levels per launch) to the single restrictions."""
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


CASES = [
    (2, 5, None), (2, 65, None), (2, 1025, None), (2, 2049, None),
    (2, 129, [(6, 2), (5, 2), (6, 1), (5, 2), (4, 2), (2, 3), (3, 1), (1, 2), (0, 2)]),
    (2, 257, [(3, 2), (7, 2), (1, 1), (0, 3), (5, 2)]),
    (3, 5, None), (3, 33, None), (3, 129, None), (3, 257, None), (3, 65, [(5, 2), (4, 1), (5, 1), (3, 2), (1, 2), (2, 1), (0, 3)]),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("d,n,sched", CASES)
def test_in_cycle_restriction_is_bitwise_identical(B, torch_cuda, d, n, sched, prec):
    torch = torch_cuda
    say("in-cycle d=%d n=%d sched=%s prec=%s" % (d, n, sched, prec))
    f = dev(torch, W.uniform(d, n, seed=31 + n))
    outs = {}
    for mode in ("pyramid", "in_cycle"):
        for tb in (0, 2):
            s = B.Solver(d, n, schedule=sched, precision=prec, temporal_block=tb, restriction=mode)
            u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
            res = s.solve_cycles(f, u, 2)
            outs[(mode, tb)] = (u.cpu().numpy(), res["history"])
            s.close()
    ref = outs[("pyramid", 2)]
    for key, (u, hist) in outs.items():
        assert np.array_equal(u, ref[0]), key
        assert hist == ref[1], key


def test_in_cycle_step_cycle_and_trace(B, torch_cuda):
    """The step-cycle entry point and the traced cycle also restart the
    chain correctly."""
    torch = torch_cuda
    n = 257
    f = W.uniform(2, n, seed=3)
    rng = np.random.default_rng(4)
    u0 = np.zeros((n, n))
    u0[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    outs = []
    for mode in ("pyramid", "in_cycle"):
        s = B.Solver(2, n, restriction=mode)
        r0 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        s.residual(dev(torch, f), dev(torch, u0), r0)
        acc = dev(torch, u0)
        s.step_cycle(r0, acc)
        t = B.Solver(2, n, restriction=mode, temporal_block=0)
        ut = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        errs = t.trace_cycle(dev(torch, f), ut, dev(torch, f))
        outs.append((acc.cpu().numpy(), ut.cpu().numpy(), errs))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_in_cycle_solve_matches_oracle_and_saves_memory(B, torch_cuda):
    torch = torch_cuda
    d, n = 3, 129
    f = W.uniform(d, n, seed=5)
    s = B.Solver(d, n, restriction="in_cycle")
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    res = s.solve(dev(torch, f), u, tol=1e-10)
    uo, _ = O.solve(d, n, f, fixed_cycles=res["cycles"])
    ug = u.cpu().numpy()
    assert np.max(np.abs(ug - uo)) <= 1e-11 * np.max(np.abs(uo))
    pyr = B.Solver(d, n).workspace_bytes()
    inc = s.workspace_bytes()
    say("workspace 129^3 FP64: pyramid %d B, in-cycle %d B" % (pyr, inc))
    assert inc < pyr
