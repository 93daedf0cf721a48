"""Writes iterations.json: oracle PCG iteration counts to ||r||/||b|| < 1e-7
for workloads too large to re-solve on the CPU inside a GPU test.

Calls only the oracle and the seeded input generators.
Run from the repository root: python tests/golden/make_iters.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1908_00741_amd import inputs  # noqa: E402


def main():
    out = {}
    A = inputs.diffusion3d(128, 1.0, 2)
    b = inputs.uniform_rhs(A.n, 3)
    r = oracle.system(A, 8, 64).solve(b, tol=1e-7)
    out["diffusion128_s1_bs8_w64"] = {
        "matrix": "diffusion3d(128, sigma=1.0, seed=2)", "rhs": "uniform_rhs(n, 3)",
        "bs": 8, "w": 64, "tol": 1e-7, "iters": r.iters, "final_rel_res": float(r.hist[-1])}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "iterations.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
