"""Reader for the small text fixtures under tests/golden/ (values printed in the paper)."""
import math
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_R = 1.0 / math.sqrt(2.0)
TOKENS = {"0": 0, "1": 1, "-1": -1, "r": _R, "-r": -_R, "i": 1j, "-i": -1j, "ir": 1j * _R, "-ir": -1j * _R}


def token(t, E=None):
    if t == "E":
        return E
    return complex(TOKENS[t])


def parse_gate(spec):
    parts = spec.split()
    name, qubits = parts[0], tuple(int(x) for x in parts[1:])
    return (name, qubits, None)


def load(name):
    """Return dict with 'qubits', 'gates' (plain gate tuples), 'matrix' or 'state'."""
    out = {}
    rows = []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("qubits:"):
                out["qubits"] = int(line.split(":")[1])
            elif line.startswith("gates:"):
                out["gates"] = [parse_gate(s) for s in line.split(":", 1)[1].split(";")]
            elif line.startswith("state:"):
                out["state"] = np.array([token(t) for t in line.split(":", 1)[1].split()])
            else:
                rows.append([token(t) for t in line.split()])
    if rows:
        out["matrix"] = np.array(rows, dtype=np.complex128)
    return out


def load_table1():
    """{name: function(phi) -> 2x2} from table1_gates.txt."""
    table = {}
    with open(os.path.join(HERE, "table1_gates.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, body = line.split(":")
            r0, r1 = [row.split() for row in body.split(";")]
            table[name.strip()] = (lambda r0=r0, r1=r1: (lambda phi=None: np.array(
                [[token(t, np.exp(1j * phi) if phi is not None else None) for t in r0],
                 [token(t, np.exp(1j * phi) if phi is not None else None) for t in r1]], dtype=np.complex128)))()
    return table
