"""Writes oracle_step_24x20.txt: the FP64 oracle's step on a seeded 24 x 20
world (3 channels, 15 kernels, localized genes, one blob).  Calls only the
oracle and the seeded input generators.  Run from the repository root:

    python tests/golden/make_oracle_fixture.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                     # noqa: E402
from paper_2304_05639_amd import inputs            # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_step_24x20.txt")


def compute():
    w = inputs.test_world(24, 20, seed=7, n_blobs=1)
    r = O.step(O.Desc.from_world(w), w.A, w.P)
    rows = [("sum_A1", float(r["A"].sum())), ("sum_P1", float(r["P"].sum())),
            ("sum_U", float(r["U"].sum())), ("n_alpha", int(r["alpha"].sum()))]
    for (c, y, x) in [(0, 12, 10), (1, 3, 17), (2, 23, 0), (0, 0, 0), (2, 11, 9)]:
        rows.append((f"A1[{c},{y},{x}]", float(r["A"][c, y, x])))
    for (p, k, y, x) in [(0, 0, 12, 10), (1, 14, 11, 9), (2, 7, 13, 11)]:
        rows.append((f"P1[{p},{k},{y},{x}]", float(r["P"][p, k, y, x])))
    for (k, y, x) in [(0, 12, 10), (9, 5, 5), (14, 20, 15)]:
        rows.append((f"U[{k},{y},{x}]", float(r["U"][k, y, x])))
    return rows


if __name__ == "__main__":
    with open(OUT, "w") as f:
        f.write("# FP64 oracle step of inputs.test_world(24, 20, seed=7, n_blobs=1);\n"
                "# written by tests/golden/make_oracle_fixture.py\n")
        for k, v in compute():
            f.write(f"{k} {v!r}\n")
    print(OUT)
