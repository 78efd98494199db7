"""Runs of the paper's own experiments (Sec. 4) on the GPU solver.

The paper studies one MFMG cycle on its polynomial test problem: the
normalised L1 error against the analytic solution after every iteration,
plotted against work units (WU, one operation over the entire grid; one
HOMG iteration is one WU), for several resolutions and two caps MaxI on the
iterations per level (Fig. 4), and the first iterations of the cycle on a
128^2 grid (Fig. 3).  Its schedule figure (Fig. 1) is missing, and the text
allows level patterns that go back to a coarser level (Sec. 2), so this
module also searches over such patterns.

Everything here drives the C ABI (libhomg.so) through the binding: the
cycles, the L1 errors and the traces run in the library's HIP kernels.
Inputs (the right-hand side and the analytic solution at the nodes) are
passed in as GPU tensors by the caller.
"""
from . import homg as _h


def default_schedule(M, max_i, coarsest=2):
    """MFMG (Sec. 2, Fig. 1): `coarsest` iterations on level M, doubling on
    every finer level, capped at MaxI."""
    return [(m, min(coarsest << (M - m), max_i)) for m in range(M, -1, -1)]


def revisit_schedule(M, max_i, coarsest=2, back=1, repeats=1, finest=True, growth="double"):
    """A level pattern that goes back to coarser levels (Sec. 2, step (c)):
    descending from level M, after each level m < M the pattern climbs back
    to level m + back and descends to m again, `repeats` times (not after
    level 0 unless `finest`).  A visit of level j runs n_j iterations:
    `coarsest` doubled per finer level (growth "double") or `coarsest` on
    every level ("flat"), capped at MaxI."""
    def its(j):
        n = coarsest << (M - j) if growth == "double" else coarsest
        return max(1, min(n, max_i))
    sched = [(M, its(M))]
    for m in range(M - 1, -1, -1):
        sched.append((m, its(m)))
        if back <= 0 or (m == 0 and not finest):
            continue
        top = min(M, m + back)
        for _ in range(repeats):
            for j in range(m + 1, top + 1):
                sched.append((j, its(j)))
            for j in range(top - 1, m - 1, -1):
                sched.append((j, its(j)))
    return sched


def candidate_schedules(M, max_i):
    """Named level patterns for the search: MFMG and its revisiting variants
    (duplicates removed)."""
    out, seen = [], set()
    for coarsest in (1, 2):
        for growth in ("double", "flat"):
            for back in (0, 1, 2):
                for repeats in ((1,) if back == 0 else (1, 2)):
                    for finest in ((True,) if back == 0 else (True, False)):
                        s = revisit_schedule(M, max_i, coarsest, back, repeats, finest, growth)
                        key = tuple(s)
                        if key in seen:
                            continue
                        seen.add(key)
                        name = "c%d-%s-back%d-x%d%s" % (coarsest, growth, back, repeats,
                                                       "" if finest else "-nofinest")
                        out.append((name, s))
    return out


def one_cycle_l1(f, u_ref, schedule=None, max_i=4, levels=0, grid_layout="nested"):
    """Normalised L1 error after one MFMG cycle from u = 0 (FP64)."""
    import torch
    n, d = int(f.shape[0]), f.dim()
    s = _h.Solver(d, n, levels=levels, max_i=max_i, schedule=schedule, grid_layout=grid_layout)
    u = torch.zeros_like(f)
    s.solve_cycles(f, u, 1)
    err = s.l1_error(u_ref, u)
    iters = sum(it for _, it in s.schedule())
    s.close()
    return err, iters


def trace(f, u_ref, max_i=4, schedule=None, grid_layout="nested"):
    """L1 error after every iteration (WU) of one MFMG cycle from u = 0,
    with the level of each iteration."""
    import torch
    n, d = int(f.shape[0]), f.dim()
    s = _h.Solver(d, n, max_i=max_i, schedule=schedule, temporal_block=0, grid_layout=grid_layout)
    u = torch.zeros_like(f)
    errs = s.trace_cycle(f, u, u_ref)
    levels = [m for m, it in s.schedule() for _ in range(it)]
    s.close()
    return errs, levels


def fig4(problems, max_is=(4, 32), grid_layout="nested"):
    """Fig. 4 runs: for each (n, f, u_ref) and MaxI, the one-cycle L1 error
    and the curve sampled at the end of every level visit as (WU, L1)."""
    runs = []
    for n, f, u_ref in problems:
        for max_i in max_is:
            errs, levels = trace(f, u_ref, max_i=max_i, grid_layout=grid_layout)
            pts = [(k + 1, errs[k]) for k in range(len(errs))
                   if k + 1 == len(errs) or levels[k + 1] != levels[k]]
            runs.append({"n": n, "layout": grid_layout, "max_i": max_i, "wu": len(errs), "l1": errs[-1],
                         "curve": [[w, round(e, 6)] for w, e in pts]})
    return runs


def search(f, u_ref, max_is=(2, 4, 32), keep=4, grid_layout="nested"):
    """One-cycle L1 error and iteration count of every candidate level
    pattern, per MaxI; returns the MFMG entry, the best patterns by L1 and by
    L1 x WU, and the patterns with the paper's 31 iterations (MaxI 2)."""
    n = int(f.shape[0])
    M = n.bit_length() - 2  # n = 2^k + 1 (nested) or 2^k (power of two): M = k - 1
    res = {}
    for max_i in max_is:
        rows = []
        for name, sched in candidate_schedules(M, max_i):
            err, iters = one_cycle_l1(f, u_ref, schedule=sched, max_i=max_i, grid_layout=grid_layout)
            rows.append({"pattern": name, "wu": iters, "l1": err})
        rows.sort(key=lambda r: r["l1"])
        mfmg = next(r for r in rows if r["pattern"] == "c2-double-back0-x1")
        res[str(max_i)] = {
            "candidates": len(rows),
            "mfmg": mfmg,
            "best_l1": rows[:keep],
            "best_l1_x_wu": sorted(rows, key=lambda r: r["l1"] * r["wu"])[:keep],
            "with_31_iterations": [r for r in rows if r["wu"] == 31][:keep],
        }
    return res
