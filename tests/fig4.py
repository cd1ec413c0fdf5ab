"""Loader for the Fig. 4 values stored in tests/golden/fig4_errors.txt."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    out = {"E": {}, "Q": {}, "C": {}}
    with open(os.path.join(HERE, "golden", "fig4_errors.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, K, D, v = line.split()
            if kind == "Q":
                out["Q"][int(D)] = float(v)
            else:
                out[kind][(int(K), int(D))] = float(v)
    return out
