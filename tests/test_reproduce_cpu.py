"""Host-side checks of the level patterns used by the paper-reproduction
runs (paper_1108_2045_amd/reproduce.py); no GPU needed."""
from oracle import homg as O


def test_default_pattern_is_the_mfmg_schedule():
    from paper_1108_2045_amd import reproduce as R
    for k in (3, 7, 12):
        for max_i in (2, 4, 32):
            assert R.default_schedule(k - 1, max_i) == O.default_schedule(k, max_i)
            assert R.revisit_schedule(k - 1, max_i, back=0) == O.default_schedule(k, max_i)


def test_revisit_patterns_go_back_and_return():
    from paper_1108_2045_amd import reproduce as R
    s = R.revisit_schedule(6, 2, back=1, repeats=1)
    assert [m for m, _ in s] == [6, 5, 6, 5, 4, 5, 4, 3, 4, 3, 2, 3, 2, 1, 2, 1, 0, 1, 0]
    assert sum(it for _, it in s) == 38
    s = R.revisit_schedule(6, 4, back=2, repeats=1, finest=False)
    levels = [m for m, _ in s]
    assert levels[-1] == 0 and levels.count(0) == 1 and max(levels) == 6
    # every step moves one level at a time, and every level is visited
    assert all(abs(a - b) == 1 for a, b in zip(levels, levels[1:]))
    cands = R.candidate_schedules(6, 4)
    names = [n for n, _ in cands]
    assert len(names) == len(set(names)) and len(cands) >= 20
    assert len({tuple(s) for _, s in cands}) == len(cands)
    for _, s in cands:
        assert s[0][0] == 6 and s[-1][0] == 0 and all(1 <= it <= 4 for _, it in s)
