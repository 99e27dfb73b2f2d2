"""Writes the small polynomial-product fixtures in this folder.

It calls only the CPU oracle (plain schoolbook products modulo P) on seeded
inputs; run it from the repository root:  python tests/golden/make_golden.py
Each line: P da db a_0..a_da b_0..b_db c_0..c_(da+db).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

PRIMES = (2013265921, 1811939329, 2113929217, 1711276033, 1107296257, 2130706433, 1224736769, 2088763393)


def main():
    rng = np.random.default_rng(20160903)
    lines = ["# polynomial products modulo P, written by make_golden.py (oracle schoolbook)"]
    shapes = [(0, 0), (0, 3), (1, 1), (2, 5), (7, 7), (15, 16), (33, 30), (64, 63)]
    for i, (da, db) in enumerate(shapes):
        P = PRIMES[i % len(PRIMES)]
        a = rng.integers(0, P, da + 1, dtype=np.uint32)
        b = rng.integers(0, P, db + 1, dtype=np.uint32)
        c = oracle.polymul_schoolbook(P, a, b)
        lines.append(" ".join(str(int(x)) for x in [P, da, db, *a, *b, *c]))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "polymul_small.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
