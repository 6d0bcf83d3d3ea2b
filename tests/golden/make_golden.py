"""Writes the stored expected values under tests/golden/ that come from the
oracle (never from the HIP path).  Run:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from wgen import make_config  # noqa: E402


def main():
    wl = make_config("tiny")
    g = wl.graph
    M = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    P = len(wl.picks)
    with open(os.path.join(HERE, "tiny_order_matrix.txt"), "w") as f:
        f.write("# tiny workload (20x40 racks, w in 1..5, seed 20655): 8 picks and\n")
        f.write("# the 8x8 pick-to-pick distance matrix, row = source pick.\n")
        f.write("# Written by tests/golden/make_golden.py from the CPU oracle.\n")
        f.write("picks " + " ".join(str(int(p)) for p in wl.picks) + "\n")
        for i in range(P):
            f.write(" ".join(str(int(x)) for x in M[i * P:(i + 1) * P]) + "\n")


if __name__ == "__main__":
    main()
