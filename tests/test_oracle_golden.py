"""Regression guard: the oracle reproduces its stored histories
(tests/golden/oracle_histories.json, written by tests/golden/make_golden.py
from oracle/ only)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import homg as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_histories.json")


def _cases():
    with open(GOLD) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_oracle_history_unchanged(case):
    f = W.sine2d(case["n"]) if case["input"] == "sine2d" else W.uniform(case["d"], case["n"], seed=case["seed"])
    _, hist = O.solve(case["d"], case["n"], f, tol=case["tol"], max_i=case["max_i"])
    assert len(hist) == len(case["history"])
    np.testing.assert_allclose(hist, case["history"], rtol=1e-9, atol=0)


def test_paper_values_fixture_is_cited():
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as fh:
        vals = json.load(fh)["values"]
    assert all("cite" in v and "status" in v for v in vals)
