"""Gate matrices in complex128 (oracle; test infrastructure only).

Sources:
* H, X, Y, Z and the phase shift R_phi: Section 2.3, Table 1.
* S and T are named in Section 5.2.2 without matrices; the textbook
  S = diag(1, i) and T = diag(1, e^{i pi/4}) are used (so S = R_{pi/2},
  T = R_{pi/4}).
* RX, RY, RZ are not in the paper; the standard half-angle rotations
  exp(-i theta sigma/2) are used.
* A controlled gate is Eq. 7 on the two-qubit basis ordered (control, target),
  i.e. block-diagonal [[I, 0], [0, U]]; CNOT is Eq. 8 (U = X), CY has U = Y, CZ has U = Z
  and CR_phi has U = R_phi.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)  # |0><0|
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)  # |1><1|


def one_qubit(name: str, theta=None) -> np.ndarray:
    """2x2 complex128 matrix of a one-qubit gate, indexed [out bit][in bit]."""
    r2 = 1.0 / math.sqrt(2.0)
    if name == "H":
        m = [[r2, r2], [r2, -r2]]
    elif name == "X":
        m = [[0, 1], [1, 0]]
    elif name == "Y":
        m = [[0, -1j], [1j, 0]]
    elif name == "Z":
        m = [[1, 0], [0, -1]]
    elif name == "S":
        m = [[1, 0], [0, 1j]]
    elif name == "T":
        m = [[1, 0], [0, cmath.exp(1j * math.pi / 4)]]
    elif name == "R":
        m = [[1, 0], [0, cmath.exp(1j * theta)]]
    elif name in ("RX", "RY", "RZ"):
        c, s = math.cos(theta / 2), math.sin(theta / 2)
        if name == "RX":
            m = [[c, -1j * s], [-1j * s, c]]
        elif name == "RY":
            m = [[c, -s], [s, c]]
        else:
            m = [[cmath.exp(-0.5j * theta), 0], [0, cmath.exp(0.5j * theta)]]
    else:
        raise ValueError(f"not a one-qubit gate: {name}")
    return np.array(m, dtype=np.complex128)


def controlled_target(name: str, theta=None) -> np.ndarray:
    """The single-qubit U that a controlled gate applies to its target."""
    if name == "CNOT":
        return one_qubit("X")
    if name == "CY":
        return one_qubit("Y")
    if name == "CZ":
        return one_qubit("Z")
    if name == "CR":
        return one_qubit("R", theta)
    raise ValueError(f"not a controlled gate: {name}")

