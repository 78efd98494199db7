"""Property-based GPU parity: random small problems against the FP64 oracle.

Each example draws a dimension, a side 2^k + 1, an execution form (one
launch per iteration, level-blocked, chained), a level schedule (the
MFMG schedule for a drawn MaxI, or an explicit pattern of levels and
iteration counts, revisits and coarse endings included), a seed, a
coefficient (2D only: constant or exp(GRF)) and a cycle count, runs that
many cycles of HOMG with the residual restart through the C ABI, and
compares u element by element with the oracle's at the same cycle count
(within 1e-11 * max|u|, the whole-solve bound), together with the
residual history.  The examples are drawn deterministically
(derandomized), so every run checks the same cases.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import workloads as W
from oracle import homg as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def B(torch_cuda):
    import paper_1108_2045_amd as P
    return P


@st.composite
def cases(draw):
    d = draw(st.sampled_from([2, 3]))
    n = draw(st.sampled_from([5, 9, 17, 33, 65] if d == 2 else [5, 9, 17, 33]))
    levels = (n - 1).bit_length() - 1  # n = 2^k + 1: levels 0 .. k - 1
    form = draw(st.sampled_from([0, 1, 2]))
    if draw(st.booleans()):
        max_i, sched = draw(st.sampled_from([1, 2, 4, 8, 32])), None
    else:
        max_i = 4
        length = draw(st.integers(1, 7))
        sched = [(draw(st.integers(0, levels - 1)), draw(st.integers(1, 5))) for _ in range(length)]
    var = d == 2 and draw(st.booleans())
    seed = draw(st.integers(0, 2 ** 16))
    cycles = draw(st.integers(1, 3))
    return d, n, form, max_i, sched, var, seed, cycles


@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(case=cases())
def test_random_cases_match_oracle(B, torch_cuda, case):
    torch = torch_cuda
    d, n, form, max_i, sched, var, seed, cycles = case
    print("case d=%d n=%d form=%d max_i=%d sched=%s var=%s seed=%d cycles=%d"
          % (d, n, form, max_i, sched, var, seed, cycles), flush=True)
    f = W.normal(d, n, seed=seed)
    a = W.grf_problem(n, seed=seed)[0] if var else None
    s = B.Solver(d, n, max_i=max_i, schedule=sched, temporal_block=form,
                 stencil=B.DIFFUSION_5PT_2D if var else None)
    if var:
        s.set_coefficient(torch.from_numpy(a).to("cuda"))
    u = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    res = s.solve_cycles(torch.from_numpy(f).to("cuda"), u, cycles)
    torch.cuda.synchronize()
    s.close()
    ug = u.cpu().numpy()
    uo, ho = O.solve(d, n, f, a=a, max_i=max_i, schedule=sched, fixed_cycles=cycles)
    scale = np.max(np.abs(uo))
    assert np.max(np.abs(ug - uo)) <= 1e-11 * scale + 1e-300, (np.max(np.abs(ug - uo)), scale)
    hg = np.array(res["history"])
    assert len(hg) == len(ho)
    assert np.all(np.abs(hg - np.array(ho)) <= 1e-6 * np.array(ho) + 1e-13), (hg, ho)
