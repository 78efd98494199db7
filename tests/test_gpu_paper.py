"""GPU runs of the paper's Sec. 4 experiments against the oracle.

* The normalised L1 error kernel against the same sums in numpy.
* One MFMG cycle on the polynomial problem traced iteration by iteration
  (Fig. 4: error against work units) equals the oracle's per-iteration L1
  errors, at MaxI 4 and 32 on several resolutions.
* The first iterations of the cycle (Fig. 3): the GPU's whole-grid states
  equal the oracle's element by element, with the spike after iteration 1
  and the pyramid after iteration 2 in closed form.
* Revisiting level patterns (the schedule search) give the oracle's
  one-cycle L1 error.
The paper's printed values (31 iterations, 5% and 1.6%) stay parity
unpinned: its schedule figure is missing (tests/golden/paper_values.json).
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


def l1(uref, v):
    return np.sum(np.abs(uref - v)) / np.sum(np.abs(uref))


@pytest.mark.parametrize("d,n", [(2, 129), (2, 1025), (3, 33), (3, 65)])
def test_l1_error_kernel(B, torch_cuda, d, n):
    torch = torch_cuda
    rng = np.random.default_rng(60 + n)
    a = rng.standard_normal((n,) * d)
    b = a + 1e-3 * rng.standard_normal((n,) * d)
    s = B.Solver(d, n)
    got = s.l1_error(dev(torch, a), dev(torch, b))
    assert got == pytest.approx(l1(a, b), rel=1e-12)
    assert s.l1_error(dev(torch, a), dev(torch, a)) == 0.0


@pytest.mark.parametrize("max_i", [4, 32])
@pytest.mark.parametrize("n", [65, 129, 257])
def test_trace_matches_oracle_per_iteration(B, torch_cuda, n, max_i):
    """Fig. 4: the L1 error after every iteration of one cycle."""
    torch = torch_cuda
    from paper_1108_2045_amd import reproduce as R
    say("trace n=%d MaxI=%d" % (n, max_i))
    f, uex = W.poly2d(n)
    errs, levels = R.trace(dev(torch, f), dev(torch, uex), max_i=max_i)
    k = O.check_side(n)
    sched = O.default_schedule(k, max_i)
    r0, _ = O.residual(2, n, f, np.zeros_like(f))
    _, states = O.mfmg_cycle(2, n, r0, sched, O.default_omega(2), keep_states=True)
    want = [l1(uex, e) for e in states]
    assert len(errs) == len(want) == sum(it for _, it in sched)
    np.testing.assert_allclose(errs, want, rtol=1e-10)
    assert levels == [m for m, it in sched for _ in range(it)]
    # the one-cycle L1 of a solve equals the trace's last entry
    err, iters = R.one_cycle_l1(dev(torch, f), dev(torch, uex), max_i=max_i)
    assert iters == len(errs) and err == pytest.approx(errs[-1], rel=1e-12)


def test_fig3_first_iterations(B, torch_cuda):
    """Fig. 3 (129^2, MaxI 2): iteration 1 is a spike at the centre,
    iteration 2 the pyramid of that value with the centre relaxed again,
    iteration 3 the first of the next finer level -- element by element
    against the oracle."""
    torch = torch_cuda
    n = 129
    f, _ = W.poly2d(n)
    k = O.check_side(n)
    M = k - 1
    sched = O.default_schedule(k, 2)
    omega = O.default_omega(2)
    r0, _ = O.residual(2, n, f, np.zeros_like(f))
    _, states = O.mfmg_cycle(2, n, r0, sched, omega, keep_states=True)
    fd = dev(torch, f)
    for upto, prefix in ((1, [(M, 1)]), (2, [(M, 2)]), (3, [(M, 2), (M - 1, 1)]), (4, [(M, 2), (M - 1, 2)])):
        s = B.Solver(2, n, levels=k, schedule=prefix)
        u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        s.solve_cycles(fd, u, 1)
        got = u.cpu().numpy()
        want = states[upto - 1]
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), upto
    c = n // 2
    e1 = states[0]
    assert np.count_nonzero(e1) == 1 and e1[c, c] != 0.0
    x = np.linspace(0, 1, n)
    hat = 1 - 2 * np.abs(x - 0.5)
    pyr = e1[c, c] * np.outer(hat, hat)
    e2 = states[1]
    pyr[c, c] = e2[c, c]
    assert np.max(np.abs(e2 - pyr)) <= 1e-14 * abs(e1[c, c])


def test_schedule_search_matches_oracle(B, torch_cuda):
    """The search's one-cycle L1 errors of revisiting patterns equal the
    oracle's for the same explicit schedules."""
    torch = torch_cuda
    from paper_1108_2045_amd import reproduce as R
    n = 65
    f, uex = W.poly2d(n)
    fd, ud = dev(torch, f), dev(torch, uex)
    M = O.check_side(n) - 1
    cands = R.candidate_schedules(M, 4)
    assert len(cands) >= 20
    for name, sched in cands[::5]:
        say("pattern %s" % name)
        err, iters = R.one_cycle_l1(fd, ud, schedule=sched, max_i=4)
        u, _ = O.solve(2, n, f, schedule=sched, fixed_cycles=1)
        assert iters == sum(it for _, it in sched)
        assert err == pytest.approx(l1(uex, u), rel=1e-10), name
    res = R.search(fd, ud, max_is=(4,), keep=3)
    assert res["4"]["mfmg"]["wu"] == sum(it for _, it in O.default_schedule(M + 1, 4))
