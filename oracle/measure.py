"""Measurement of a simulated state (test infrastructure only).

The paper's Simulator interface has a second method beside the full-state one:
it simulates the circuit and returns only the collapsed state, chosen with the
probabilities that the state vector gives (Section 5.2.3).  With every qubit
measured, the collapsed state is a basis state |i>, drawn with probability
p_i = |psi_i|^2 / sum_j |psi_j|^2 (Section 2.2, Eq. 1-3).

The draw is inverse-CDF sampling and the random numbers are inputs: given a
uniform u in [0, 1), the outcome is the smallest i whose cumulative
probability C_i = p_0 + ... + p_i exceeds u * C_{N-1}.  The oracle accumulates C
in float64 from index 0 upwards.
"""
from __future__ import annotations

import numpy as np


def cumulative(prob) -> np.ndarray:
    """C_i = p_0 + ... + p_i, accumulated left to right in float64."""
    p = np.asarray(prob, dtype=np.float64).ravel()
    out = np.empty_like(p)
    s = 0.0
    for i in range(p.size):
        s += p[i]
        out[i] = s
    return out


def sample(prob, uniforms) -> np.ndarray:
    """Outcome per uniform: the smallest i with u * C_{N-1} < C_i (int64)."""
    c = cumulative(prob)
    u = np.asarray(uniforms, dtype=np.float64).ravel()
    out = np.searchsorted(c, u * c[-1], side="right")
    return np.minimum(out, c.size - 1).astype(np.int64)


def collapse(n: int, outcome: int) -> np.ndarray:
    """The collapsed state after measuring every qubit with result `outcome`: the basis vector |outcome>."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[outcome] = 1.0
    return psi
