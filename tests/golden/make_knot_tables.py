"""Write the optimal-knot tables used as fixed inputs by the GPU parity tests.

Calls only the oracle (oracle.lut.knot_table, Sec. 3.4 of the paper).  Each
file holds theta_1..theta_P (units of the smoothing length) for the table
abscissae Lambda_i = (i + 1/2) q / n, one row per line, written with 17
significant digits so that they read back bit-exactly.

    python tests/golden/make_knot_tables.py            # all tables
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lut  # noqa: E402

TABLES = [
    ("cubic", 4, 2, 4096),
    ("wendland", 4, 3, 4096),
    ("cubic", 3, 3, 256),
    ("wendland", 2, 2, 256),
    ("cubic", 1, 2, 128),
    ("cubic", 5, 2, 128),
    ("wendland", 6, 4, 128),
    ("cubic", 4, 4, 256),
    ("wendland", 4, 1, 256),
    ("wendland_c4", 4, 3, 64),
    ("wendland_c6", 2, 2, 64),
    ("wendland_grad", 4, 3, 64),
    ("wendland_grad", 4, 3, 1024),
    ("wendland_grad", 4, 3, 4096),
    ("wendland_c4_grad", 3, 2, 64),
    ("wendland_c6_grad", 2, 2, 64),
    ("wendland", 4, 2, 4096),
    ("wendland", 4, 4, 4096),
]


def path(kind, K, D, n):
    return os.path.join(HERE, f"knots_{kind}_K{K}_D{D}_n{n}.txt")


def write(kind, K, D, n, pool):
    lams, th, e2 = lut.knot_table(kind, K, D, n, pool=pool)
    with open(path(kind, K, D, n), "w") as f:
        f.write(f"# optimal knots theta_1..theta_P, kernel={kind} K={K} D={D} n={n}; "
                f"row i: Lambda_i = (i + 1/2) * 2 / n; written by tests/golden/make_knot_tables.py (oracle only)\n")
        for row in th:
            f.write(" ".join(repr(float(x)) for x in row) + "\n")


def load(kind, K, D, n):
    return np.loadtxt(path(kind, K, D, n), ndmin=2)


if __name__ == "__main__":
    with Pool(int(os.environ.get("NPROC", "8"))) as pool:
        for spec in TABLES:
            if len(sys.argv) > 1 and os.path.exists(path(*spec)):
                continue
            print("table", spec, flush=True)
            write(*spec, pool)
