"""Write the oracle's 1-NN of every query of the two full-size benchmark workloads.

    python tests/golden/make_full_size.py            # all four files (about 10 minutes on 8 cores)
    python tests/golden/make_full_size.py rw256_p1   # one of them

Calls only the fp64 C oracle (``oracle.native.nn_bruteforce``: banded DTW_p of the query
against every candidate by the Sec. 4 recursion, then the smallest (distance, index) key --
the definition of the nearest neighbour that Algorithms 2 and 3 reach exactly) and the seeded
input generator.  Inputs are the float32-rounded series widened to float64, what the device
sees.  Each output line is ``query index DTW_p^p`` with the pow-domain distance written with
17 significant digits.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import native  # noqa: E402
from paper_0811_3301_amd import gen  # noqa: E402

# name -> (workload, w, p)
CASES = {
    "rw256_p1": ("rw256", 26, 1),
    "rw256_p2": ("rw256", 26, 2),
    "shape512_w26": ("shape512", 26, 1),
    "shape512_w51": ("shape512", 51, 1),
}


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}_nn.txt")


def write(name: str) -> str:
    workload, w, p = CASES[name]
    db64, qs64 = gen.make_workload(workload)
    X = db64.astype(np.float32).astype(np.float64)
    Ys = qs64.astype(np.float32).astype(np.float64)
    idx, dpow = native.nn_bruteforce(X, Ys, w, p, 1)
    spec = gen.WORKLOADS[workload]
    lines = [
        f"# 1-NN under DTW_{p} (band w = {w}) of every query of workload '{workload}': "
        f"{spec['N']} x {spec['n']} database, {spec['Q']} queries, float32-rounded inputs.",
        "# Brute force over every candidate by the fp64 oracle (Sec. 4 recursion; ties to the smaller index).",
        "# Written by tests/golden/make_full_size.py.  Columns: query index DTW_p^p",
    ]
    for q in range(Ys.shape[0]):
        lines.append(f"{q} {int(idx[q, 0])} {float(dpow[q, 0]):.17g}")
    out = path_of(name)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def load(name: str):
    """(index [Q] int64, DTW_p^p [Q] float64) from a written file."""
    rows = np.loadtxt(path_of(name), comments="#", dtype=np.float64, ndmin=2)
    return rows[:, 1].astype(np.int64), rows[:, 2]


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        print(write(name), flush=True)
