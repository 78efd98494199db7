"""Write the stored expected values under tests/golden/ (calls only oracle/).

    python tests/golden/make_golden.py

oracle_histories.json: per-cycle relative residuals of the FP64 oracle for
small seeded problems (2D sine source on 129^2; 2D U[-1,1] on 65^2; 3D
U[-1,1] on 17^3), used as a regression guard on the oracle itself and as a
fixed expectation for the GPU path at the same sizes.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import homg as O  # noqa: E402

CASES = [
    {"name": "sine2d_129_maxi4", "d": 2, "n": 129, "input": "sine2d", "max_i": 4, "tol": 1e-10},
    {"name": "uniform2d_65_seed0_maxi4", "d": 2, "n": 65, "input": "uniform", "seed": 0, "max_i": 4, "tol": 1e-10},
    {"name": "uniform3d_17_seed0_maxi4", "d": 3, "n": 17, "input": "uniform", "seed": 0, "max_i": 4, "tol": 1e-10},
    {"name": "uniform2d_33_seed1_maxi32", "d": 2, "n": 33, "input": "uniform", "seed": 1, "max_i": 32, "tol": 1e-10},
]


def make_input(c):
    if c["input"] == "sine2d":
        return W.sine2d(c["n"])
    return W.uniform(c["d"], c["n"], seed=c["seed"])


def main():
    out = {"generator": "tests/golden/make_golden.py (oracle.homg.solve, FP64)", "cases": []}
    for c in CASES:
        f = make_input(c)
        _, hist = O.solve(c["d"], c["n"], f, tol=c["tol"], max_i=c["max_i"])
        out["cases"].append(dict(c, history=[float(x) for x in hist]))
    with open(os.path.join(HERE, "oracle_histories.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
