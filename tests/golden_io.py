"""Reader for the hand-derived fixtures in tests/golden/ (format only)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    n = None
    qubits = None
    U = None
    tin, tout = {}, {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "n":
                n = int(tok[1])
            elif tok[0] == "qubits":
                qubits = tuple(int(x) for x in tok[1:])
            elif tok[0] == "U":
                v = np.array([float(x) for x in tok[1:]])
                d = 1 << len(qubits)
                U = (v[0::2] + 1j * v[1::2]).reshape(d, d)
            elif tok[0] in ("in", "out"):
                (tin if tok[0] == "in" else tout)[int(tok[1])] = (float(tok[2]), float(tok[3]))
    return n, qubits, U, tin, tout


def names():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
